// Filter with hit selection: on every layer a track has several candidate
// hits; after the propagation each candidate gets the chi-square a Kalman
// update with it would add, and the candidate with the smallest chi-square
// not above the gate updates the state (the search step of track finding
// that the paper's benchmark leaves out between propagation and update,
// Sec. 3.1).  No qualifying candidate: the layer is a hole and the state is
// the prediction.  A candidate with non-finite values or a residual
// covariance that is not positive definite takes no part.
//
// One lane per track, the state in registers across its layers (as in the
// plain step); per layer the lane streams its candidates (9 floats each),
// keeping the best one's hit in registers, then runs the ordinary update
// with it.  The decision's chi-square is computed with the same expressions
// (and precision) as the update's, so the chi-square that decides is the one
// that is added.  The precision flags select the update as in the plain step:
// FP64 residual-covariance inverse and gain, optionally the Joseph form.
#include "kf_device.h"
#include "kf_internal.h"
#include "kf_lanes.h"

namespace kf {

namespace {

// Chi-square of an update of the prediction (q, Pt) with hit (m, V), and
// whether the candidate takes part (finite, residual covariance positive
// definite).  R: the arithmetic of the update that follows -- float for the
// FP32 update, double when S^-1 is taken in FP64 (the precision form) -- and
// CHOL its form (update_f32 on cylinders: the Cholesky factor of S), so the
// chi-square that decides is the one added.
template <class R, bool CHOL>
__device__ __forceinline__ bool candidate_chi2(const float q[6], const float Pt[21], const float m[3],
                                               const float V[6], float& chi2) {
  const R r0 = R(m[0] - q[0]), r1 = R(m[1] - q[1]), r2 = R(m[2] - q[2]);
  const R S00 = R(Pt[0] + V[0]), S10 = R(Pt[1] + V[1]), S11 = R(Pt[2] + V[2]);
  const R S20 = R(Pt[3] + V[3]), S21 = R(Pt[4] + V[4]), S22 = R(Pt[5] + V[5]);
  const bool in_ok = fin(r0) & fin(r1) & fin(r2) & fin(S00) & fin(S10) & fin(S11) & fin(S20) & fin(S21) & fin(S22);
  if constexpr (CHOL) {
    const Chol3<R> L = chol3(S00, S10, S11, S20, S21, S22);
    R z0, z1, z2;
    L.solve(r0, r1, r2, z0, z1, z2);
    const R c = z0 * z0 + z1 * z1 + z2 * z2;
    chi2 = float(c);
    return in_ok & L.pd & fin(c);
  }
  const R c00 = S11 * S22 - S21 * S21;
  const R c10 = S20 * S21 - S10 * S22;
  const R c11 = S00 * S22 - S20 * S20;
  const R c20 = S10 * S21 - S11 * S20;
  const R c21 = S10 * S20 - S00 * S21;
  const R c22 = S00 * S11 - S10 * S10;
  const R det = S00 * c00 + S10 * c10 + S20 * c20;
  const bool pd = (S00 > R(0)) & (c22 > R(0)) & (det > R(0));
  const R rdet = rcp_t(det);
  const R i00 = c00 * rdet, i10 = c10 * rdet, i11 = c11 * rdet;
  const R i20 = c20 * rdet, i21 = c21 * rdet, i22 = c22 * rdet;
  const R t0 = i00 * r0 + i10 * r1 + i20 * r2;
  const R t1 = i10 * r0 + i11 * r1 + i21 * r2;
  const R t2 = i20 * r0 + i21 * r1 + i22 * r2;
  const R c = r0 * t0 + r1 * t1 + r2 * t2;
  chi2 = float(c);
  return in_ok & pd & fin(c) & fin(chi2);
}

// STREAM: every track runs all layers (no per-track counts), so every wave
// reads whole rows of candidates, each once, and the state and candidate
// arrays carry the non-temporal hint (element-major layouts); waves of
// tracks with different layer counts read partial rows and keep the default.
template <int KIND, bool STREAM>
constexpr int gate_policy() {
  return STREAM ? once_policy<KIND>() : 0;
}
template <int KIND, bool WIDE, bool STREAM>
using GateLanes = Lanes<KIND, WIDE, 4, gate_policy<KIND, STREAM>()>;

template <int KIND, bool WIDE, bool STREAM>
struct Candidates {
  static constexpr int P = gate_policy<KIND, STREAM>();
  const GateArgs& a;
  const GateLanes<KIND, WIDE, STREAM>& ln;
  LaneRef<WIDE> pos, cov;
  int Ep, Ec;
  __device__ __forceinline__ Candidates(const GateArgs& a_, const GateLanes<KIND, WIDE, STREAM>& ln_, int64_t i)
      : a(a_), ln(ln_), Ep(3 * a_.M), Ec(6 * a_.M) {
    pos = lane_ref<KIND, WIDE>(i, a.n, Ep, a.L, a.lay);
    cov = lane_ref<KIND, WIDE>(i, a.n, Ec, a.L, a.lay);
  }
  // candidate j of layer k (both wave-uniform)
  __device__ __forceinline__ void load(int k, int j, float m[3], float V[6]) const {
    if constexpr (!WIDE) {
      const __amdgpu_buffer_rsrc_t rp = buf_rsrc(a.cand_pos, pos.bytes);
      const __amdgpu_buffer_rsrc_t rc = buf_rsrc(a.cand_cov, cov.bytes);
      if (KIND == KF_AOS) {
        buf_ld_rec<3, P>(rp, pos.boff, uint32_t(ln.uni(Ep, k, 3 * j)) * 4u, m);
        buf_ld_rec<6, P>(rc, cov.boff, uint32_t(ln.uni(Ec, k, 6 * j)) * 4u, V);
      } else {
#pragma unroll
        for (int e = 0; e < 3; ++e) m[e] = buf_ld<P>(rp, pos.boff, uint32_t(ln.uni(Ep, k, 3 * j + e)) * 4u);
#pragma unroll
        for (int e = 0; e < 6; ++e) V[e] = buf_ld<P>(rc, cov.boff, uint32_t(ln.uni(Ec, k, 6 * j + e)) * 4u);
      }
    } else if (KIND == KF_AOS) {
      ld_rec<3>(pos.at(a.cand_pos, ln.uni(Ep, k, 3 * j)), m);
      ld_rec<6>(cov.at(a.cand_cov, ln.uni(Ec, k, 6 * j)), V);
    } else {
#pragma unroll
      for (int e = 0; e < 3; ++e) m[e] = *pos.at(a.cand_pos, ln.uni(Ep, k, 3 * j + e));
#pragma unroll
      for (int e = 0; e < 6; ++e) V[e] = *cov.at(a.cand_cov, ln.uni(Ec, k, 6 * j + e));
    }
  }
};

// One layer: propagate, select, update.  Returns status bits; on success
// (p, C, d) hold the new state and `best` the candidate used (-1: a hole).
template <int GEOM, bool ZIN, int PREC, int KIND, bool WIDE, bool STREAM>
__device__ __forceinline__ uint32_t gate_layer(const Candidates<KIND, WIDE, STREAM>& cands, int k, float p[6], float C[21],
                                               DirT<float>& d, float& chi2, int& best) {
  float q[6], Pt[21];
  DirT<float> dq = d;
  // candidates are fetched ahead of their evaluation (see the loop below);
  // on planes the first two before the propagation, which does not need
  // them (1.078 -> 1.067 ms)
  float mn[3] = {0.0f, 0.0f, 0.0f}, Vn[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};  // the next candidate
  float mm[3] = {0.0f, 0.0f, 0.0f}, Vm[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};  // planes: the one after
  if constexpr (GEOM == 0) {
    if (cands.a.M > 0) cands.load(k, 0, mn, Vn);
    if (cands.a.M > 1) cands.load(k, 1, mm, Vm);
  }
  const uint32_t fp = propagate<GEOM, ZIN, float>(p, C, dq, cands.a.layer[k], cands.a.b, q, Pt);
  bool fin_ok = true;
#pragma unroll
  for (int e = 0; e < 6; ++e) fin_ok = fin_ok & fin(q[e]);
#pragma unroll
  for (int e = 0; e < 21; ++e) fin_ok = fin_ok & fin(Pt[e]);
  if (fp) return fp;
  if (!fin_ok) return S_NONFINITE;
  best = -1;
  float bchi = __builtin_inff();
  float mb[3] = {0.0f, 0.0f, 0.0f}, Vb[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  // candidates are fetched ahead of their evaluation: planes two ahead,
  // cylinders one (8 candidates: p2z 1.130 -> 1.107 ms one ahead, 1.082 ms
  // two ahead; p2r 1.310 -> 1.168 ms one ahead, 1.256 ms two ahead, where
  // the longer step's registers run short -- as they do when the two forms
  // share one array-based loop: 8 bytes of spill there cost p2r 8 %)
  if constexpr (GEOM != 0)
    if (cands.a.M > 0) cands.load(k, 0, mn, Vn);
  for (int j = 0; j < cands.a.M; ++j) {
    float m[3], V[6], c;
#pragma unroll
    for (int e = 0; e < 3; ++e) m[e] = mn[e];
#pragma unroll
    for (int e = 0; e < 6; ++e) V[e] = Vn[e];
    if constexpr (GEOM == 0) {
#pragma unroll
      for (int e = 0; e < 3; ++e) mn[e] = mm[e];
#pragma unroll
      for (int e = 0; e < 6; ++e) Vn[e] = Vm[e];
      if (j + 2 < cands.a.M) cands.load(k, j + 2, mm, Vm);
    } else {
      if (j + 1 < cands.a.M) cands.load(k, j + 1, mn, Vn);
    }
    const bool ok = PREC == PREC_F32 ? candidate_chi2<float, GEOM == 1>(q, Pt, m, V, c)
                                     : candidate_chi2<double, false>(q, Pt, m, V, c);
    const bool take = ok & (c <= cands.a.gate) & (c < bchi);
    best = take ? j : best;
    bchi = take ? c : bchi;
#pragma unroll
    for (int e = 0; e < 3; ++e) mb[e] = take ? m[e] : mb[e];
#pragma unroll
    for (int e = 0; e < 6; ++e) Vb[e] = take ? V[e] : Vb[e];
  }
  if (best >= 0) {
    const float phi = q[4], theta = q[5];
    float dchi;
    const uint32_t fu = update<GEOM, PREC, float>(q, Pt, mb, Vb, dchi);
    if (fu) return fu;
    rotate_by(dq.sp, dq.cp, q[4] - phi, q[4]);
    rotate_by(dq.st, dq.ct, q[5] - theta, q[5]);
    chi2 += dchi;
  }
#pragma unroll
  for (int e = 0; e < 6; ++e) p[e] = q[e];
#pragma unroll
  for (int e = 0; e < 21; ++e) C[e] = Pt[e];
  d = dq;
  return 0u;
}

}  // namespace

// Cylinders: compiled for 4 waves per SIMD (142 VGPRs and 3 waves otherwise;
// at 4 it spills 24 bytes per lane: 1.380 -> 1.326 ms on the barrel sample).
template <int GEOM, int PREC, int KIND, bool WIDE, bool STREAM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GEOM == 1 && PREC == 0 ? 4 : 1, 8)))
kf_gate_kernel(const GateArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const GateLanes<KIND, WIDE, STREAM> ln(i, a.n, a.L, a.lay);
  const Candidates<KIND, WIDE, STREAM> cands(a, ln, i);
  int nl = a.nlay ? a.nlay[i] : a.L;
  nl = nl < 0 ? 0 : (nl > a.L ? a.L : nl);
  float p[6], C[21];
  ln.template ld_all<6>(ln.par, a.par_in, 0, p);
  ln.template ld_all<21>(ln.cov, a.cov_in, 0, C);
  uint32_t flags = 0;
#pragma unroll
  for (int e = 0; e < 6; ++e) flags |= fin(p[e]) ? 0u : S_NONFINITE;
#pragma unroll
  for (int e = 0; e < 21; ++e) flags |= fin(C[e]) ? 0u : S_NONFINITE;
  float chi2 = 0.0f;
  int done = 0;
  DirT<float> d;
  dir_init(p, d);
  for (int k = 0; k < nl && !flags; ++k) {
    int best = -1;
    const uint32_t f = (GEOM == 0 && k > 0) ? gate_layer<GEOM, true, PREC>(cands, k, p, C, d, chi2, best)
                                            : gate_layer<GEOM, false, PREC>(cands, k, p, C, d, chi2, best);
    if (f) {
      flags = f;
      break;
    }
    if (a.chosen) a.chosen[int64_t(k) * a.n + i] = best;
    done = k + 1;
  }
  ln.template st_all<6>(ln.par, a.par_out, 0, p);
  ln.template st_all<21>(ln.cov, a.cov_out, 0, C);
  if (a.chi2) a.chi2[i] = chi2;
  if (a.status) a.status[i] = int32_t(flags | (uint32_t(done) << 16));
}

template <int GEOM, int PREC, bool WIDE>
static hipError_t launch_kind(int block, const GateArgs& a, hipStream_t s) {
  const dim3 grid(unsigned((a.n + block - 1) / block));
  const bool stream = a.nlay == nullptr;
  if (a.lay.kind == KF_AOS)
    hipLaunchKernelGGL((kf_gate_kernel<GEOM, PREC, KF_AOS, WIDE, false>), grid, dim3(block), 0, s, a);
  else if (a.lay.kind == KF_AOSOA && stream)
    hipLaunchKernelGGL((kf_gate_kernel<GEOM, PREC, KF_AOSOA, WIDE, true>), grid, dim3(block), 0, s, a);
  else if (a.lay.kind == KF_AOSOA)
    hipLaunchKernelGGL((kf_gate_kernel<GEOM, PREC, KF_AOSOA, WIDE, false>), grid, dim3(block), 0, s, a);
  else if (stream)
    hipLaunchKernelGGL((kf_gate_kernel<GEOM, PREC, KF_SOA, WIDE, true>), grid, dim3(block), 0, s, a);
  else
    hipLaunchKernelGGL((kf_gate_kernel<GEOM, PREC, KF_SOA, WIDE, false>), grid, dim3(block), 0, s, a);
  return hipGetLastError();
}

template <int PREC>
static hipError_t launch_prec(int geom, bool wide, int block, const GateArgs& a, hipStream_t s) {
  if (geom == 0) return wide ? launch_kind<0, PREC, true>(block, a, s) : launch_kind<0, PREC, false>(block, a, s);
  return wide ? launch_kind<1, PREC, true>(block, a, s) : launch_kind<1, PREC, false>(block, a, s);
}

hipError_t launch_gate(int geom, int prec, int block, const GateArgs& a, hipStream_t s) {
  // 64-bit addressing once any array reaches 4 GiB (the candidates' covariances are the largest)
  const bool wide = layout_floats(a.n, 6 * a.M, a.L, a.lay) * 4 >= (int64_t(1) << 32) || needs_wide(a.n, a.L, a.lay);
  if (prec == PREC_F32) return launch_prec<PREC_F32>(geom, wide, block, a, s);
  if (prec == PREC_F64) return launch_prec<PREC_F64>(geom, wide, block, a, s);
  return launch_prec<PREC_F64_JOSEPH>(geom, wide, block, a, s);
}

}  // namespace kf

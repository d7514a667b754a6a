// The batched Kalman-filter step kernel for gfx950: one lane per track,
// state in registers across all of its layers, coalesced loads of the
// track/hit arrays in SoA or AoSoA form.
#include "kf_device.h"
#include "kf_internal.h"
#include "kf_lanes.h"

namespace kf {

// Load one layer's hit (position and covariance) for this lane.
template <bool WIDE>
__device__ __forceinline__ void load_hit(const StepArgs& a, const Lanes<WIDE>& ln, int k, float m[3], float V[6]) {
#pragma unroll
  for (int e = 0; e < 3; ++e) m[e] = ln.hp.ld(a.hit_pos, ln.uni(3, k, e));
#pragma unroll
  for (int e = 0; e < 6; ++e) V[e] = ln.hc.ld(a.hit_cov, ln.uni(6, k, e));
}

// One layer: propagate to surface `target`, transport the covariance, update
// with hit (m, V).  On success the state (p, C) and chi2 advance in place and 0
// is returned; otherwise the status bits, with (p, C) left undefined.
// One layer: propagate to surface `target`, transport the covariance, update
// with hit (m, V).  On success the state (p, C) and chi2 advance in place and 0
// is returned; otherwise the status bits, with (p, C) left undefined.
template <int GEOM, int PREC>
__device__ __forceinline__ uint32_t layer_step(float p[6], float C[21], const float m[3], const float V[6],
                                               float target, float b, float& chi2) {
  float q[6], Pt[21];
  const uint32_t fp = propagate<GEOM>(p, C, target, b, q, Pt);
  float dchi;
  const uint32_t fu = update<GEOM, PREC>(q, Pt, m, V, dchi);
#pragma unroll
  for (int e = 0; e < 6; ++e) p[e] = q[e];
#pragma unroll
  for (int e = 0; e < 21; ++e) C[e] = Pt[e];
  chi2 += dchi;
  return fp ? fp : fu;
}

template <bool WIDE>
__device__ __forceinline__ bool load_state(const StepArgs& a, const Lanes<WIDE>& ln, float p[6], float C[21]) {
  bool ok = true;
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    p[e] = ln.par.ld(a.par_in, ln.uni(6, 0, e));
    ok = ok & fin(p[e]);
  }
#pragma unroll
  for (int e = 0; e < 21; ++e) {
    C[e] = ln.cov.ld(a.cov_in, ln.uni(21, 0, e));
    ok = ok & fin(C[e]);
  }
  return ok;
}

// The layer loop updates the state in place, so the pre-layer state is not
// kept alive in registers for the failure path.  A track that fails at layer
// k (rare) instead re-reads its input -- untouched until the final store,
// also in place -- and re-applies layers 0..k-1 after the loop.
template <int GEOM, int PREC, bool WIDE>
__global__ void __launch_bounds__(256) kf_step_kernel(const StepArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const Lanes<WIDE> ln(i, a.n, a.L, a.lay);
  const int L = a.L;

  float p[6], C[21];
  uint32_t flags = load_state(a, ln, p, C) ? 0u : S_NONFINITE;
  int nl = a.nlay ? a.nlay[i] : L;
  nl = nl < 0 ? 0 : (nl > L ? L : nl);
  float chi2 = 0.0f;
  int k = 0;
  if (!flags && nl > 0) {
    // hits of the next layer are fetched one layer ahead
    float mn[3], Vn[6];
    load_hit(a, ln, 0, mn, Vn);
    for (; k < nl; ++k) {
      float m[3], V[6];
#pragma unroll
      for (int e = 0; e < 3; ++e) m[e] = mn[e];
#pragma unroll
      for (int e = 0; e < 6; ++e) V[e] = Vn[e];
      load_hit(a, ln, k + 1 < L ? k + 1 : k, mn, Vn);  // wave-uniform index, always in bounds
      if (a.ckpt) {
#pragma unroll
        for (int e = 0; e < 6; ++e) ln.ck.st(a.ckpt, ln.uni(27, k, e), p[e]);
#pragma unroll
        for (int e = 0; e < 21; ++e) ln.ck.st(a.ckpt, ln.uni(27, k, 6 + e), C[e]);
      }
      const uint32_t f = layer_step<GEOM, PREC>(p, C, m, V, a.layer[k], a.b, chi2);
      if (f) {
        flags = f;
        break;
      }
    }
  }
  const int done = k;
  if (flags) {
    // recompute the state from before the failing layer
    load_state(a, ln, p, C);
    chi2 = 0.0f;
    for (int j = 0; j < done; ++j) {
      float m[3], V[6];
      load_hit(a, ln, j, m, V);
      layer_step<GEOM, PREC>(p, C, m, V, a.layer[j], a.b, chi2);
    }
  }
#pragma unroll
  for (int e = 0; e < 6; ++e) ln.par.st(a.par_out, ln.uni(6, 0, e), p[e]);
#pragma unroll
  for (int e = 0; e < 21; ++e) ln.cov.st(a.cov_out, ln.uni(21, 0, e), C[e]);
  if (a.chi2) a.chi2[i] = chi2;
  if (a.status) a.status[i] = int32_t(flags | (uint32_t(done) << KF_S_LAYERS_SHIFT));
}

template <int GEOM, int PREC, bool WIDE>
static hipError_t launch_one(int block, const StepArgs& a, hipStream_t s) {
  const int64_t grid = (a.n + block - 1) / block;
  hipLaunchKernelGGL((kf_step_kernel<GEOM, PREC, WIDE>), dim3(unsigned(grid)), dim3(block), 0, s, a);
  return hipGetLastError();
}

template <int GEOM, bool WIDE>
static hipError_t launch_prec(int prec, int block, const StepArgs& a, hipStream_t s) {
  if (prec == 0) return launch_one<GEOM, PREC_F32, WIDE>(block, a, s);
  if (prec == 1) return launch_one<GEOM, PREC_F64, WIDE>(block, a, s);
  return launch_one<GEOM, PREC_F64_JOSEPH, WIDE>(block, a, s);
}

hipError_t launch_step(int geom, int prec, int block, int tpt, const StepArgs& a, hipStream_t s) {
  (void)tpt;
  const bool wide = needs_wide(a.n, a.L, a.lay);
  if (geom == 0) return wide ? launch_prec<0, true>(prec, block, a, s) : launch_prec<0, false>(prec, block, a, s);
  return wide ? launch_prec<1, true>(prec, block, a, s) : launch_prec<1, false>(prec, block, a, s);
}

// ---------------------------------------------------------------- pack/unpack
__global__ void __launch_bounds__(256) kf_pack_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                      int32_t E, int32_t L, int64_t n, TrackLayout lay,
                                                      int to_layout) {
  const int64_t total = int64_t(E) * L * n;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += int64_t(gridDim.x) * blockDim.x) {
    // SoA index t = (l*E + e)*n + i
    const int64_t i = t % n;
    const int64_t le = t / n;
    const int l = int(le / E), e = int(le % E);
    const int64_t o = layout_offset(i, n, E, L, l, e, lay);
    if (to_layout)
      dst[o] = src[t];
    else
      dst[t] = src[o];
  }
}

hipError_t launch_pack(const float* src, float* dst, int32_t E, int32_t L, int64_t n, TrackLayout lay,
                       bool to_layout, hipStream_t s) {
  const int64_t total = int64_t(E) * L * n;
  int64_t grid = (total + 255) / 256;
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(kf_pack_kernel, dim3(unsigned(grid)), dim3(256), 0, s, src, dst, E, L, n, lay,
                     to_layout ? 1 : 0);
  return hipGetLastError();
}

}  // namespace kf

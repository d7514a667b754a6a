// The batched Kalman-filter step kernel for gfx950: one lane per track,
// state in registers across all of its layers, coalesced loads of the
// track/hit arrays in SoA, AoSoA or AoS form.
#include "kf_internal.h"
#include "kf_lanes.h"
#include "kf_track.h"

namespace kf {

// T: the arrays' scalar (float; double in the FP64 form, which addresses with
// 64-bit pointers, WIDE).
template <int KIND, bool WIDE, class T = float>
struct LaidOutState {
  const StepArgsT<T>& a;
  const Lanes<KIND, WIDE, sizeof(T)>& ln;
  __device__ __forceinline__ bool load(T p[6], T C[21]) const {
    ln.template ld_all<6>(ln.par, a.par_in, 0, p);
    ln.template ld_all<21>(ln.cov, a.cov_in, 0, C);
    bool ok = true;
#pragma unroll
    for (int e = 0; e < 6; ++e) ok = ok & fin(p[e]);
#pragma unroll
    for (int e = 0; e < 21; ++e) ok = ok & fin(C[e]);
    return ok;
  }
  __device__ __forceinline__ void store(const T p[6], const T C[21]) const {
    ln.template st_all<6>(ln.par, a.par_out, 0, p);
    ln.template st_all<21>(ln.cov, a.cov_out, 0, C);
  }
};

template <int KIND, bool WIDE, class T = float>
struct LaidOutHits {
  using Off = typename LaneRef<WIDE>::Off;
  const StepArgsT<T>& a;
  const Lanes<KIND, WIDE, sizeof(T)>& ln;
  Off hp_last, hc_last;  // this lane's offsets of its last layer
  __device__ __forceinline__ LaidOutHits(const StepArgsT<T>& a_, const Lanes<KIND, WIDE, sizeof(T)>& ln_, int nl)
      : a(a_), ln(ln_) {
    const int last = nl > 0 ? nl - 1 : 0;
    hp_last = ln.template layer_off<3>(ln.hp, last);
    hc_last = ln.template layer_off<6>(ln.hc, last);
  }
  __device__ __forceinline__ void load(int k, T m[3], T V[6]) const {
    ln.template ld_all<3>(ln.hp, a.hit_pos, k, m);
    ln.template ld_all<6>(ln.hc, a.hit_cov, k, V);
  }
  // element-major float layouts can go through the LDS ring; AoS records
  // (and FP64 arrays) are fetched into registers
  static constexpr bool kStaged = KIND != KF_AOS && sizeof(T) == 4;
  __device__ __forceinline__ int next(int k) const { return k + 1 < a.L ? k + 1 : k; }
  __device__ __forceinline__ int n_layers() const { return a.L; }
  // layer min(j, the track's last layer); j is wave-uniform
  template <int POLICY>
  __device__ __forceinline__ void stage(int j, float* slot) const {
    const int ju = j < a.L - 1 ? j : a.L - 1;
    ln.template stage<3, POLICY>(ln.hp, a.hit_pos, ju, hp_last, slot);
    ln.template stage<6, POLICY>(ln.hc, a.hit_cov, ju, hc_last, slot + 3 * 64);
  }
};

// FULL: per-track layer counts and checkpoints in an element-major layout
// -- every lane writes every checkpoint row up to the wave's longest track,
// nl_wave (slots of a track's unreached layers then hold its final state).
// Whole rows avoid partially written lines, which memory completes by
// read-modify-write: the barrel filter with checkpoints went from 1.48 to
// 0.60 ms (SoA, 960k tracks).  AoS records gain nothing (1.02 -> 1.22 ms):
// their lines are shared by neighbouring lanes' records either way.
template <int KIND, bool WIDE, class T = float, bool FULL = false>
struct LaidOutCkpt {
  static constexpr bool kFullRows = FULL;
  const StepArgsT<T>& a;
  const Lanes<KIND, WIDE, sizeof(T)>& ln;
  int nl_wave;
  __device__ __forceinline__ void operator()(int k, const T p[6], const T C[21]) const {
    if (!a.ckpt || (k & ((1 << a.ck_shift) - 1))) return;
    T s[27];
#pragma unroll
    for (int e = 0; e < 6; ++e) s[e] = p[e];
#pragma unroll
    for (int e = 0; e < 21; ++e) s[6 + e] = C[e];
    // written once here, read back by another kernel: not kept in cache
    ln.template st_all<27, T, once_policy<KIND>()>(ln.ck, a.ckpt, k >> a.ck_shift, s);
  }
};

// Build option: ask the register allocator for at least KF_STEP_MIN_WAVES
// waves per SIMD (it spills to scratch memory to get there).
#ifdef KF_STEP_MIN_WAVES
#define KF_STEP_OCCUPANCY __attribute__((amdgpu_waves_per_eu(KF_STEP_MIN_WAVES, 8)))
#else
#define KF_STEP_OCCUPANCY
#endif

// How a step kernel fetches its hits.  Planes: the layer step is short, so
// element-major layouts bring the hits through the per-wave LDS ring with
// three layers in flight.  Cylinders: the Newton search makes the step
// long enough for one layer of register prefetch to cover the latency, and
// each lane then loads only its own hit, without the ring's per-layer copies
// and LDS reads (5 % faster on the barrel sample in SoA and AoSoA).
template <int GEOM, int KIND, bool WIDE>
constexpr bool ring_staged() {
  return LaidOutHits<KIND, WIDE>::kStaged && GEOM == 0;
}

// dynamic LDS: kRingFloats per wave of the block (kernels that stage through the ring).
// STREAM: every track runs all a.L layers, so each staged hit is read once
// (no wave re-reads the last layers of finished tracks) and the copies carry
// the non-temporal hint.
// Cylinders with per-track layer counts: a wave runs as many layers as its
// longest track, and tracks stop where the helix no longer reaches a cylinder
// (on the barrel sample 36 % of the lanes idle).  Each group of KF_CYL_SORT
// consecutive tracks is therefore handed to its threads longest first, so
// that a wave's tracks have similar lengths (1.27x fewer lane-layers for
// groups of 128).  With register prefetch every lane loads its own hits, so
// the permutation costs only a wider spread of each load: a 128-track group
// spans 4 cache lines per element row instead of 2 (SoA; AoS records are
// contiguous), while 256-track groups cost more than they save.  0 disables.
#ifndef KF_CYL_SORT
#define KF_CYL_SORT 128
#endif
// The track this thread runs, longest first within each group of G threads
// of the block (a counting sort of the layer counts in LDS; G <= 256).
template <int G>
__device__ __forceinline__ int64_t by_length(const StepArgs& a) {
  __shared__ int cnt[256 / G][KF_MAX_LAYERS + 2];
  __shared__ int off[256 / G][KF_MAX_LAYERS + 2];
  __shared__ int perm[256];
  const int t = int(threadIdx.x), nt = int(blockDim.x);
  const int gs = nt < G ? nt : G;  // group size
  const int g = t / gs, lt = t - g * gs;
  const int ng = nt / gs;
  const int64_t i0 = int64_t(blockIdx.x) * nt;
  int key = a.L + 1;  // no track: last
  if (i0 + t < a.n) {
    int nl = a.nlay[i0 + t];
    nl = nl < 0 ? 0 : (nl > a.L ? a.L : nl);
    key = a.L - nl;
  }
  for (int j = t; j < ng * (KF_MAX_LAYERS + 2); j += nt) cnt[j / (KF_MAX_LAYERS + 2)][j % (KF_MAX_LAYERS + 2)] = 0;
  __syncthreads();
  const int r = atomicAdd(&cnt[g][key], 1);
  __syncthreads();
  // exclusive prefix of each group's counts (a serial sum per entry: at most
  // KF_MAX_LAYERS + 1 terms)
  for (int j = t; j < ng * (KF_MAX_LAYERS + 2); j += nt) {
    const int gg = j / (KF_MAX_LAYERS + 2), kk = j % (KF_MAX_LAYERS + 2);
    int excl = 0;
    for (int k = 0; k < kk; ++k) excl += cnt[gg][k];
    off[gg][kk] = excl;
  }
  __syncthreads();
  perm[g * gs + off[g][key] + r] = lt;
  __syncthreads();
  return i0 + g * gs + perm[t];
}

// FULL: checkpoints with per-track layer counts (see LaidOutCkpt).
template <int GEOM, int PREC, int KIND, bool WIDE, bool STREAM, bool FULL = false>
__global__ void __launch_bounds__(256) KF_STEP_OCCUPANCY kf_step_kernel(const StepArgs a) {
  extern __shared__ float kf_lds[];
  float* ring = kf_lds + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)) * kRingFloats;
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  // (not with checkpoints: a permuted group's two waves would share every
  // line of the checkpoint rows, each writing half of it at a different time)
  if constexpr (GEOM == 1 && KF_CYL_SORT > 0 && !FULL) {
    if (a.nlay) i = by_length<KF_CYL_SORT>(a);
  }
  int nl = 0;
  if (i < a.n) {
    nl = a.nlay ? a.nlay[i] : a.L;
    nl = nl < 0 ? 0 : (nl > a.L ? a.L : nl);
  }
  // every lane is still active here (full blocks): the wave's longest track
  const int nl_wave = FULL ? wave_max(nl) : 0;
  if (i >= a.n) return;
  const Lanes<KIND, WIDE> ln(i, a.n, a.L, a.lay, a.Lck);
  float chi2;
  uint32_t status;
  const LaidOutHits<KIND, WIDE> hits(a, ln, nl);
  const LaidOutCkpt<KIND, WIDE, float, FULL> ckpt{a, ln, nl_wave};
  if constexpr (ring_staged<GEOM, KIND, WIDE>()) {
    LayerRing<LaidOutHits<KIND, WIDE>, STREAM ? kStreamPolicy : 0> stager(hits, ring);
    run_track<GEOM, PREC>(LaidOutState<KIND, WIDE>{a, ln}, hits, stager, ckpt, nl, a.layer, a.b, chi2, status);
  } else {
    RegStager<LaidOutHits<KIND, WIDE>> stager(hits);
    run_track<GEOM, PREC>(LaidOutState<KIND, WIDE>{a, ln}, hits, stager, ckpt, nl, a.layer, a.b, chi2, status);
  }
  if (a.chi2) a.chi2[i] = chi2;
  if (a.status) a.status[i] = int32_t(status);
}

template <int GEOM, int PREC, int KIND, bool WIDE>
static hipError_t launch_one(int block, const StepArgs& a, hipStream_t s) {
  const int64_t grid = (a.n + block - 1) / block;
  constexpr bool kStaged = ring_staged<GEOM, KIND, WIDE>();
  const size_t lds = kStaged ? size_t(block / 64) * kRingFloats * sizeof(float) : 0;
  // copies straight into LDS address it through the low 16 bits of M0
  static_assert(4 * kRingFloats * sizeof(float) <= 65536, "a 256-thread block's rings must lie in 64 KiB of LDS");
  if (kStaged && !a.nlay)
    hipLaunchKernelGGL((kf_step_kernel<GEOM, PREC, KIND, WIDE, kStaged>), dim3(unsigned(grid)), dim3(block), lds, s,
                       a);
  else if (a.ckpt && a.nlay && PREC == PREC_F32 && KIND != KF_AOS)
    hipLaunchKernelGGL((kf_step_kernel<GEOM, PREC, KIND, WIDE, false, true>), dim3(unsigned(grid)), dim3(block), lds,
                       s, a);
  else
    hipLaunchKernelGGL((kf_step_kernel<GEOM, PREC, KIND, WIDE, false>), dim3(unsigned(grid)), dim3(block), lds, s, a);
  return hipGetLastError();
}

template <int GEOM, int PREC, bool WIDE>
static hipError_t launch_kind(int block, const StepArgs& a, hipStream_t s) {
  if (a.lay.kind == KF_AOS) return launch_one<GEOM, PREC, KF_AOS, WIDE>(block, a, s);
  if (a.lay.kind == KF_AOSOA) return launch_one<GEOM, PREC, KF_AOSOA, WIDE>(block, a, s);
  return launch_one<GEOM, PREC, KF_SOA, WIDE>(block, a, s);
}

template <int GEOM, bool WIDE>
static hipError_t launch_prec(int prec, int block, const StepArgs& a, hipStream_t s) {
  if (prec == 0) return launch_kind<GEOM, PREC_F32, WIDE>(block, a, s);
  if (prec == 1) return launch_kind<GEOM, PREC_F64, WIDE>(block, a, s);
  return launch_kind<GEOM, PREC_F64_JOSEPH, WIDE>(block, a, s);
}

hipError_t launch_step(int geom, int prec, int block, int tpt, const StepArgs& a, hipStream_t s) {
  (void)tpt;
  const bool wide = needs_wide(a.n, a.L, a.lay);
  if (geom == 0) return wide ? launch_prec<0, true>(prec, block, a, s) : launch_prec<0, false>(prec, block, a, s);
  return wide ? launch_prec<1, true>(prec, block, a, s) : launch_prec<1, false>(prec, block, a, s);
}

// ---------------------------------------------------------------- FP64 form
// The same step in FP64 end to end (arrays, field constant, layer table and
// arithmetic).  Planes fetch their hits one layer ahead into registers (two
// layers ahead was slower: 0.383 against 0.375 ms per launch on the plane
// sample).  The cylinder step's double state fills the 256 VGPRs that leave
// room for two waves per SIMD (253, no spills), so it loads each layer's hit
// at the top of that layer, where the search covers the latency; with the
// one-layer prefetch it would spill.
template <int GEOM, int PREC, int KIND>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
kf_step_kernel_f64(const StepArgsT<double> a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const Lanes<KIND, true, 8> ln(i, a.n, a.L, a.lay, a.Lck);
  int nl = a.nlay ? a.nlay[i] : a.L;
  nl = nl < 0 ? 0 : (nl > a.L ? a.L : nl);
  double chi2;
  uint32_t status;
  const LaidOutHits<KIND, true, double> hits(a, ln, nl);
  using Stager = std::conditional_t<GEOM == 1, DirectStager<LaidOutHits<KIND, true, double>, double>,
                                    RegStager<LaidOutHits<KIND, true, double>, double>>;
  Stager stager(hits);
  run_track<GEOM, PREC>(LaidOutState<KIND, true, double>{a, ln}, hits, stager, NoCkpt{}, nl, a.layer, a.b, chi2,
                        status);
  if (a.chi2) a.chi2[i] = chi2;
  if (a.status) a.status[i] = int32_t(status);
}

template <int GEOM, int PREC>
static hipError_t launch_f64_kind(int block, const StepArgsT<double>& a, hipStream_t s) {
  const int64_t grid = (a.n + block - 1) / block;
  if (a.lay.kind == KF_AOS)
    hipLaunchKernelGGL((kf_step_kernel_f64<GEOM, PREC, KF_AOS>), dim3(unsigned(grid)), dim3(block), 0, s, a);
  else if (a.lay.kind == KF_AOSOA)
    hipLaunchKernelGGL((kf_step_kernel_f64<GEOM, PREC, KF_AOSOA>), dim3(unsigned(grid)), dim3(block), 0, s, a);
  else
    hipLaunchKernelGGL((kf_step_kernel_f64<GEOM, PREC, KF_SOA>), dim3(unsigned(grid)), dim3(block), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_step_f64(int geom, int prec, int block, const StepArgsT<double>& a, hipStream_t s) {
  // prec 0: plain update; 2: Joseph update (both in FP64, as everything here)
  if (geom == 0) return prec == 2 ? launch_f64_kind<0, PREC_F64_JOSEPH>(block, a, s) : launch_f64_kind<0, PREC_F32>(block, a, s);
  return prec == 2 ? launch_f64_kind<1, PREC_F64_JOSEPH>(block, a, s) : launch_f64_kind<1, PREC_F32>(block, a, s);
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

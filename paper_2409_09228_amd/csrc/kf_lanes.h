// Per-lane addressing of the track and hit arrays.
//
// Element e of a track (E elements per track and layer) on layer l sits at
//   lane_offset(E) + l * layer_stride(E) + e * es        floats from the base:
//   SoA:      lane_offset = i,                      layer_stride = E*n,  es = n
//   AoSoA-B:  lane_offset = (i/B)*(E*L*B) + i%B,    layer_stride = E*B,  es = B
//   AoS:      lane_offset = i*E,                    layer_stride = n*E,  es = 1
// Only the first term differs between the lanes of a wave, so every load is a
// wave-uniform base plus a per-lane byte offset computed once per track: no
// per-element address arithmetic in the layer loop beyond one add.  Byte
// offsets are 32-bit unless an array spans 4 GiB or more (WIDE).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "kf_internal.h"

namespace kf {

__host__ __device__ inline int64_t layout_offset(int64_t i, int64_t n, int E, int L, int l, int e, TrackLayout lay) {
  if (lay.kind == KF_AOS) return (int64_t(l) * n + i) * E + e;
  if (lay.kind == KF_SOA) return (int64_t(l) * E + e) * n + i;
  const int64_t B = int64_t(1) << lay.shift;
  return (i >> lay.shift) * (int64_t(E) * L * B) + (i & (B - 1)) + (int64_t(l) * E + e) * B;
}

// Floats spanned by one array of E elements per track and L layers.
inline int64_t layout_floats(int64_t n, int E, int L, TrackLayout lay) {
  if (lay.kind == KF_AOSOA) {
    const int64_t B = int64_t(1) << lay.shift;
    return ((n + B - 1) / B) * B * E * (L > 0 ? L : 1);
  }
  return n * E * (L > 0 ? L : 1);
}

// Largest array of a launch: checkpoints (27 per layer).
inline bool needs_wide(int64_t n, int L, TrackLayout lay) {
  return layout_floats(n, 27, L, lay) * 4 >= (int64_t(1) << 32);
}

// N consecutive floats (4-byte aligned) as one record: the compiler emits
// multi-dword loads/stores (dwordx2/x3/x4) instead of N dword accesses.
template <int N>
struct __attribute__((packed, aligned(4))) FRec {
  float v[N];
};
template <int N>
__device__ __forceinline__ void ld_rec(const float* p, float* dst) {
  FRec<N> r;
  __builtin_memcpy(&r, p, sizeof(r));
#pragma unroll
  for (int i = 0; i < N; ++i) dst[i] = r.v[i];
}
template <int N>
__device__ __forceinline__ void st_rec(float* p, const float* src) {
  FRec<N> r;
#pragma unroll
  for (int i = 0; i < N; ++i) r.v[i] = src[i];
  __builtin_memcpy(p, &r, sizeof(r));
}

template <bool WIDE>
struct LaneRef {
  using Off = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
  Off boff;  // byte offset of this lane's element 0, layer 0
  __device__ __forceinline__ float ld(const float* base, int64_t uni) const {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base + uni) + boff);
  }
  __device__ __forceinline__ void st(float* base, int64_t uni, float v) const {
    *reinterpret_cast<float*>(reinterpret_cast<char*>(base + uni) + boff) = v;
  }
  __device__ __forceinline__ const float* at(const float* base, int64_t uni) const {
    return reinterpret_cast<const float*>(reinterpret_cast<const char*>(base + uni) + boff);
  }
  __device__ __forceinline__ float* at(float* base, int64_t uni) const {
    return reinterpret_cast<float*>(reinterpret_cast<char*>(base + uni) + boff);
  }
};

template <int KIND, bool WIDE>
struct Lanes {
  LaneRef<WIDE> par, cov, hp, hc, ck;
  int64_t es, n;
  __device__ __forceinline__ Lanes(int64_t i, int64_t n_, int L, TrackLayout lay) : n(n_) {
    using Off = typename LaneRef<WIDE>::Off;
    if (KIND == KF_AOSOA) {
      const int64_t B = int64_t(1) << lay.shift;
      const int64_t blk = i >> lay.shift, lane = i & (B - 1);
      es = B;
      par.boff = Off((blk * 6 * B + lane) * 4);
      cov.boff = Off((blk * 21 * B + lane) * 4);
      hp.boff = Off((blk * 3 * L * B + lane) * 4);
      hc.boff = Off((blk * 6 * L * B + lane) * 4);
      ck.boff = Off((blk * 27 * L * B + lane) * 4);
    } else if (KIND == KF_AOS) {
      es = 1;
      par.boff = Off(i * 6 * 4);
      cov.boff = Off(i * 21 * 4);
      hp.boff = Off(i * 3 * 4);
      hc.boff = Off(i * 6 * 4);
      ck.boff = Off(i * 27 * 4);
    } else {
      es = n;
      par.boff = cov.boff = hp.boff = hc.boff = ck.boff = Off(i * 4);
    }
  }
  // E consecutive elements of one layer (AoS records) from / to array `base`
  template <int E>
  __device__ __forceinline__ void ld_all(const LaneRef<WIDE>& r, const float* base, int l, float* dst) const {
    if (KIND == KF_AOS) {
      ld_rec<E>(r.at(base, uni(E, l, 0)), dst);
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) dst[e] = r.ld(base, uni(E, l, e));
    }
  }
  template <int E>
  __device__ __forceinline__ void st_all(const LaneRef<WIDE>& r, float* base, int l, const float* src) const {
    if (KIND == KF_AOS) {
      st_rec<E>(r.at(base, uni(E, l, 0)), src);
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) r.st(base, uni(E, l, e), src[e]);
    }
  }
  // wave-uniform part of the offset of element e (of E) on layer l
  __device__ __forceinline__ int64_t uni(int E, int l, int e) const {
    const int64_t lstride = KIND == KF_AOS ? n * E : int64_t(E) * es;
    return int64_t(l) * lstride + int64_t(e) * es;
  }
};

}  // namespace kf

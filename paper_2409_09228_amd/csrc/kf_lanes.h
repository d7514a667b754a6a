// Per-lane addressing of the track and hit arrays.
//
// Element e of a track (E elements per track and layer, L layers) on layer l
// sits at   lane_offset(E, L) + (l*E + e) * es   floats from the array base:
//   SoA:      lane_offset = i,                       es = n
//   AoSoA-B:  lane_offset = (i/B)*(E*L*B) + i%B,     es = B
// The second term is the same for every lane of a wave, so each load is a
// scalar base plus a per-lane byte offset that is computed once per track --
// no per-element 64-bit address arithmetic in the layer loop.  Byte offsets
// are 32-bit unless an array spans 4 GiB or more (WIDE).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "kf_internal.h"

namespace kf {

__host__ __device__ inline int64_t layout_offset(int64_t i, int64_t n, int E, int L, int l, int e, TrackLayout lay) {
  if (!lay.aos) return (int64_t(l) * E + e) * n + i;
  const int64_t B = int64_t(1) << lay.shift;
  return (i >> lay.shift) * (int64_t(E) * L * B) + (i & (B - 1)) + (int64_t(l) * E + e) * B;
}

// Largest array of a launch: hits (6 per layer) or checkpoints (27 per layer).
inline bool needs_wide(int64_t n, int L, TrackLayout lay) {
  const int64_t B = lay.aos ? (int64_t(1) << lay.shift) : 1;
  const int64_t padded = lay.aos ? ((n + B - 1) / B) * B : n;
  const int64_t Lm = L > 1 ? L : 1;
  const int64_t floats = padded * 27 * Lm;
  return floats * 4 >= (int64_t(1) << 32);
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
};

template <bool WIDE>
struct Lanes {
  LaneRef<WIDE> par, cov, hp, hc, ck;
  int64_t es;
  __device__ __forceinline__ Lanes(int64_t i, int64_t n, int L, TrackLayout lay) {
    using Off = typename LaneRef<WIDE>::Off;
    if (lay.aos) {
      const int64_t B = int64_t(1) << lay.shift;
      const int64_t blk = i >> lay.shift, lane = i & (B - 1);
      es = B;
      par.boff = Off((blk * 6 * B + lane) * 4);
      cov.boff = Off((blk * 21 * B + lane) * 4);
      hp.boff = Off((blk * 3 * L * B + lane) * 4);
      hc.boff = Off((blk * 6 * L * B + lane) * 4);
      ck.boff = Off((blk * 27 * L * B + lane) * 4);
    } else {
      es = n;
      par.boff = cov.boff = hp.boff = hc.boff = ck.boff = Off(i * 4);
    }
  }
  // wave-uniform part of the offset of element e (of E) on layer l
  __device__ __forceinline__ int64_t uni(int E, int l, int e) const { return (int64_t(l) * E + e) * es; }
};

}  // namespace kf

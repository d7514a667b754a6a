// The per-track layer loop shared by the plain and the persistent kernels.
//
// A lane owns one track: it reads the 27-number state once, runs every layer
// with the state in registers, and writes it once.  The loop updates the
// state in place, so the pre-layer state is never kept alive in registers
// for the failure path; a track that fails at layer k (rare) re-reads its
// input -- untouched until the final store, also when the call is in place --
// and re-applies layers 0..k-1 after the loop.
#pragma once

#include "kf_device.h"

namespace kf {

// One layer: propagate to surface `target`, transport the covariance, update
// with hit (m, V).  On success the state (p, C), the sin/cos of its direction
// angles d, and chi2 advance in place and 0 is returned; otherwise the status
// bits, with (p, C, d) left undefined.  ZIN: C carries the zero z row and
// column of a preceding plane update.
template <int GEOM, int PREC, bool ZIN, class T>
__device__ __forceinline__ uint32_t layer_step(T p[6], T C[21], DirT<T>& d, const T m[3], const T V[6], T target, T b,
                                               T& chi2) {
  T q[6], Pt[21];
  const uint32_t fp = propagate<GEOM, ZIN, T>(p, C, d, target, b, q, Pt);
  const T phi = q[4], theta = q[5];
  T dchi;
  const uint32_t fu = update<GEOM, PREC, T>(q, Pt, m, V, dchi);
  rotate_by(d.sp, d.cp, q[4] - phi, q[4]);
  rotate_by(d.st, d.ct, q[5] - theta, q[5]);
#pragma unroll
  for (int e = 0; e < 6; ++e) p[e] = q[e];
#pragma unroll
  for (int e = 0; e < 21; ++e) C[e] = Pt[e];
  chi2 += dchi;
  return fp ? fp : fu;
}

// Hits are staged through LDS: every wave owns a ring of kRing slots, one
// layer of hits each (9 floats x 64 lanes, element-major so that both the
// copy into LDS and the read back are lane-contiguous).  Layer k + kRing is
// requested when layer k is read, so kRing layers are in flight per wave
// without holding registers for them.  The copies go straight from memory to
// LDS and complete in order, so reading slot k only needs the wave's
// vector-memory counter down to the 9 (kRing - 1) copies issued after it.
#ifndef KF_RING
#define KF_RING 3  // build option: layers of hits in flight per wave
#endif
constexpr int kRing = KF_RING;
constexpr int kSlotFloats = 9 * 64;
constexpr int kRingFloats = kRing * kSlotFloats;  // per wave

// s_waitcnt with only the vector-memory count constrained (gfx9 encoding:
// vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
template <int N>
__device__ __forceinline__ void wait_vmem() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}
// s_waitcnt lgkmcnt(0): this wave's LDS reads have returned
__device__ __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14)); }

__device__ __forceinline__ void read_slot(const float* slot, int lane, float m[3], float V[6]) {
#pragma unroll
  for (int e = 0; e < 3; ++e) m[e] = slot[e * 64 + lane];
#pragma unroll
  for (int e = 0; e < 6; ++e) V[e] = slot[(3 + e) * 64 + lane];
}

// IO concepts used below:
//   state.load(p, C) -> bool all-finite;  state.store(p, C)
//   hits.load(l, m, V): the hit of layer l into registers (the recompute path)
//   stager: the hits of layers 0, 1, ... in order --
//     begin(): start fetching (the track has at least one layer)
//     get(k, m, V): layer k's hit
//     end(): nothing of this track is in flight any more
//     kCooperative: lanes fetch for each other, so every lane of the wave
//       must call get() for every layer: the wave's tracks then share one
//       layer count and a failing track does not leave the loop early
//   ckpt(k, p, C): called before layer k (may do nothing)
//   Ckpt::kFullRows: every lane of a wave must call ckpt for every layer up
//     to the wave's longest track (checkpoint rows are then written whole;
//     a lane past its own track stores its final state)
struct NoCkpt {
  static constexpr bool kFullRows = false;
  template <class T>
  __device__ __forceinline__ void operator()(int, const T*, const T*) const {}
};

// the largest v over the wave's lanes; every lane of the wave must be active
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const int o = __shfl_xor(v, d, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Hits fetched one layer ahead into registers (AoS records: multi-dword loads
// serve them better than one-dword copies).  hits.next(k): the in-bounds
// layer to prefetch after layer k.
template <class Hits, class T = float>
struct RegStager {
  static constexpr bool kCooperative = false;
  const Hits& h;
  T mn[3], Vn[6];
  __device__ __forceinline__ explicit RegStager(const Hits& h_) : h(h_) {}
  __device__ __forceinline__ void begin() { h.load(0, mn, Vn); }
  __device__ __forceinline__ void get(int k, T m[3], T V[6]) {
#pragma unroll
    for (int e = 0; e < 3; ++e) m[e] = mn[e];
#pragma unroll
    for (int e = 0; e < 6; ++e) V[e] = Vn[e];
    h.load(h.next(k), mn, Vn);
  }
  __device__ __forceinline__ void end() {}
};

// Hits loaded when their layer comes, with nothing held in registers in
// between: for a step whose own state leaves no room for a prefetched layer
// (the FP64 cylinder step), where occupancy does the hiding instead.
template <class Hits, class T = float>
struct DirectStager {
  static constexpr bool kCooperative = false;
  const Hits& h;
  __device__ __forceinline__ explicit DirectStager(const Hits& h_) : h(h_) {}
  __device__ __forceinline__ void begin() {}
  __device__ __forceinline__ void get(int k, T m[3], T V[6]) { h.load(k, m, V); }
  __device__ __forceinline__ void end() {}
};

// Element-major hits through this wave's LDS ring (kRingFloats at `ring`).
// hits.stage<POLICY>(j, slot): start copying the hit of layer min(j, the
// track's last layer) into the slot (j wave-uniform), with cache policy
// POLICY.  hits.n_layers(): the layer table's length L.  Layers from L on
// are never copied (no track has them): near the end of the table fewer
// than kRing - 1 copies follow the slot being read, and the wait is for all
// of them.
template <class Hits, int POLICY = 0>
struct LayerRing {
  static constexpr bool kCooperative = false;
  const Hits& h;
  float* ring;
  int s;
  __device__ __forceinline__ LayerRing(const Hits& h_, float* ring_) : h(h_), ring(ring_), s(0) {}
  __device__ __forceinline__ void begin() {
#pragma unroll
    for (int i = 0; i < kRing; ++i)
      if (i < h.n_layers()) h.template stage<POLICY>(i, ring + i * kSlotFloats);
  }
  __device__ __forceinline__ void get(int k, float m[3], float V[6]) {
    float* slot = ring + s * kSlotFloats;
    if (k + kRing - 1 < h.n_layers())
      wait_vmem<9 * (kRing - 1)>();
    else
      wait_vmem<0>();
    read_slot(slot, int(threadIdx.x & 63), m, V);
    wait_lds();
    if (k + kRing < h.n_layers()) h.template stage<POLICY>(k + kRing, slot);
    s = s + 1 == kRing ? 0 : s + 1;
  }
  __device__ __forceinline__ void end() { wait_vmem<0>(); }
};

// Layer k of a track: from the second layer on, a plane step knows the zero
// z row and column its predecessor left in C.
template <int GEOM, int PREC, class T>
__device__ __forceinline__ uint32_t layer_at(int k, T p[6], T C[21], DirT<T>& d, const T m[3], const T V[6], T target,
                                             T b, T& chi2) {
  if (GEOM == 0 && k > 0) return layer_step<GEOM, PREC, true, T>(p, C, d, m, V, target, b, chi2);
  return layer_step<GEOM, PREC, false, T>(p, C, d, m, V, target, b, chi2);
}

// The layer loop of one track.  Every lane of the wave that runs a track
// calls this together (lanes without one are inactive); the stager's
// wave-level waits rely on that.
// T: the scalar of the state, the hits and the layer table (float, or double
// in the FP64 form).
template <int GEOM, int PREC, class State, class Hits, class Stager, class Ckpt, class T>
__device__ __forceinline__ void run_track(const State& state, const Hits& hits, Stager& stager, const Ckpt& ckpt,
                                          int nl, const T* layer, T b, T& chi2_out, uint32_t& status_out) {
  T p[6], C[21];
  uint32_t flags = state.load(p, C) ? 0u : S_NONFINITE;
  T chi2 = T(0);
  int k = 0;
  if ((Stager::kCooperative || !flags) && nl > 0) {
    DirT<T> d;
    dir_init(p, d);
    T m[3], V[6];
    stager.begin();
    // the first layer is peeled so that the loop body is the plane step that
    // knows C's zero z row
    stager.get(0, m, V);
    ckpt(0, p, C);
    const uint32_t f0 = layer_step<GEOM, PREC, false>(p, C, d, m, V, layer[0], b, chi2);
    if (!flags) flags = f0;
    if constexpr (Stager::kCooperative) {
      // every lane walks all nl layers; the first failure (or a non-finite
      // input) is kept, and the state after it, discarded below, no longer
      // matters
      int fail_at = flags ? 0 : nl;
      for (k = 1; k < nl; ++k) {
        stager.get(k, m, V);
        ckpt(k, p, C);
        const uint32_t f = layer_step<GEOM, PREC, GEOM == 0>(p, C, d, m, V, layer[k], b, chi2);
        if (f && !flags) {
          flags = f;
          fail_at = k;
        }
      }
      k = fail_at;
    } else if constexpr (Ckpt::kFullRows) {
      // every lane walks as many layers as the wave's longest track so that
      // each checkpoint row is written by the whole wave (partially written
      // lines cost a read-modify-write in memory); a lane past its own last
      // layer, or after its failure, computes nothing and stores its state
      int fail_at = flags ? 0 : nl;
      const int nl_w = ckpt.nl_wave;  // the wave's longest track, <= the layer table
      for (k = 1; k < nl_w; ++k) {
        const bool act = !flags && k < nl;
        stager.get(k, m, V);
        ckpt(k, p, C);
        if (act) {
          const uint32_t f = layer_step<GEOM, PREC, GEOM == 0>(p, C, d, m, V, layer[k], b, chi2);
          if (f) {
            flags = f;
            fail_at = k;
          }
        }
      }
      k = fail_at;
    } else if (!flags) {
      for (k = 1; k < nl; ++k) {
        stager.get(k, m, V);
        ckpt(k, p, C);
        const uint32_t f = layer_step<GEOM, PREC, GEOM == 0>(p, C, d, m, V, layer[k], b, chi2);
        if (f) {
          flags = f;
          break;
        }
      }
    }
    stager.end();
  }
  const int done = k;
  if (flags) {
    // recompute the state from before the failing layer
    state.load(p, C);
    chi2 = T(0);
    DirT<T> d;
    dir_init(p, d);
    for (int j = 0; j < done; ++j) {
      T m[3], V[6];
      hits.load(j, m, V);
      layer_at<GEOM, PREC>(j, p, C, d, m, V, layer[j], b, chi2);
    }
  }
  state.store(p, C);
  chi2_out = chi2;
  status_out = flags | (uint32_t(done) << KF_S_LAYERS_SHIFT);
}

}  // namespace kf

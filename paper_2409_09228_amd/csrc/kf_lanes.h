// Per-lane addressing of the track and hit arrays.
//
// Element e of a track (E elements per track and layer) on layer l sits at
//   lane_offset(E) + l * layer_stride(E) + e * es        floats from the base:
//   SoA:      lane_offset = i,                      layer_stride = E*n,  es = n
//   AoSoA-B:  lane_offset = (i/B)*(E*L*B) + i%B,    layer_stride = E*B,  es = B
//   AoS:      lane_offset = i*E,                    layer_stride = n*E,  es = 1
// Only the first term differs between the lanes of a wave, so every access is
// a wave-uniform byte offset plus a per-lane byte offset computed once per
// track.  Arrays below 4 GiB are accessed through buffer resources (base and
// size in scalar registers): the per-lane offset is one 32-bit VGPR, the
// uniform offset a scalar register, and no 64-bit address is formed per
// element; accesses past the array's end read zero and write nothing.  Larger
// arrays (WIDE) use 64-bit global addresses.
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
__host__ __device__ inline int64_t layout_floats(int64_t n, int E, int L, TrackLayout lay) {
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
template <int N, class T = float>
struct __attribute__((packed, aligned(4))) FRec {
  T v[N];
};
template <int N, class T>
__device__ __forceinline__ void ld_rec(const T* p, T* dst) {
  FRec<N, T> r;
  __builtin_memcpy(&r, p, sizeof(r));
#pragma unroll
  for (int i = 0; i < N; ++i) dst[i] = r.v[i];
}
template <int N, class T>
__device__ __forceinline__ void st_rec(T* p, const T* src) {
  FRec<N, T> r;
#pragma unroll
  for (int i = 0; i < N; ++i) r.v[i] = src[i];
  __builtin_memcpy(p, &r, sizeof(r));
}

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void gbl_void;

// Cache-policy bits of an access: 0 the default, kStreamPolicy the
// non-temporal hint (gfx950 NT) for data that is read or written once.
constexpr int kStreamPolicy = 2;
// The policy for arrays a kernel reads or writes once, by layout: element-
// major layouts (SoA, AoSoA) stream; an AoS record is moved by several
// loads that touch the same cache lines, so it keeps the default.
template <int KIND>
__host__ __device__ constexpr int once_policy() {
  return KIND == KF_AOS ? 0 : kStreamPolicy;
}

// Buffer-resource word 3 for untyped 32-bit access on gfx9-family parts.
constexpr int kBufWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const float* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, int(bytes), kBufWord3);
}
template <int POLICY = 0>
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), POLICY));
}
template <int POLICY = 0>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, int(voff), int(soff), POLICY);
}
// Element j of a vector of dwords as a float.  The element is copied to a
// scalar first: a bit cast applied directly to a vector subscript reads
// element 0 with this compiler.
template <class V>
__device__ __forceinline__ float lane_word(const V& v, int j) {
  const unsigned w = v[j];
  return __builtin_bit_cast(float, w);
}
// N consecutive floats of one lane: dwordx4 pieces, then x3/x2/x1 for the rest
template <int N, int POLICY = 0>
__device__ __forceinline__ void buf_ld_rec(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float* dst) {
#pragma unroll
  for (int c = 0; c + 4 <= N; c += 4) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, int(voff), int(soff + 4 * c), POLICY);
#pragma unroll
    for (int j = 0; j < 4; ++j) dst[c + j] = lane_word(v, j);
  }
  constexpr int c = N & ~3;
  if (N - c == 3) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b96(r, int(voff), int(soff + 4 * c), POLICY);
#pragma unroll
    for (int j = 0; j < 3; ++j) dst[c + j] = lane_word(v, j);
  } else if (N - c == 2) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), int(soff + 4 * c), POLICY);
    dst[c] = lane_word(v, 0);
    dst[c + 1] = lane_word(v, 1);
  } else if (N - c == 1) {
    dst[c] = buf_ld<POLICY>(r, voff, soff + 4 * c);
  }
}
template <int N, int POLICY = 0>
__device__ __forceinline__ void buf_st_rec(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, const float* src) {
#pragma unroll
  for (int c = 0; c + 4 <= N; c += 4) {
    __attribute__((ext_vector_type(4))) unsigned v;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = __builtin_bit_cast(unsigned, src[c + j]);
    __builtin_amdgcn_raw_buffer_store_b128(v, r, int(voff), int(soff + 4 * c), POLICY);
  }
  constexpr int c = N & ~3;
  if (N - c == 3) {
    __attribute__((ext_vector_type(3))) unsigned v;
#pragma unroll
    for (int j = 0; j < 3; ++j) v[j] = __builtin_bit_cast(unsigned, src[c + j]);
    __builtin_amdgcn_raw_buffer_store_b96(v, r, int(voff), int(soff + 4 * c), POLICY);
  } else if (N - c == 2) {
    __attribute__((ext_vector_type(2))) unsigned v;
    v[0] = __builtin_bit_cast(unsigned, src[c]);
    v[1] = __builtin_bit_cast(unsigned, src[c + 1]);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, int(voff), int(soff + 4 * c), POLICY);
  } else if (N - c == 1) {
    buf_st<POLICY>(r, voff, soff + 4 * c, src[c]);
  }
}

template <bool WIDE>
struct LaneRef {
  using Off = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
  Off boff;        // byte offset of this lane's element 0, layer 0
  uint32_t bytes;  // size of the array (buffer form)
  template <class T>
  __device__ __forceinline__ const T* at(const T* base, int64_t uni) const {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base + uni) + boff);
  }
  template <class T>
  __device__ __forceinline__ T* at(T* base, int64_t uni) const {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base + uni) + boff);
  }
};

// This lane's reference into an array of E floats per track and layer, Lx
// layers, in `lay` (for arrays whose element count is known only at run
// time; accesses then use Lanes::uni(E, l, e)).
template <int KIND, bool WIDE>
__device__ __forceinline__ LaneRef<WIDE> lane_ref(int64_t i, int64_t n, int E, int Lx, TrackLayout lay) {
  using Off = typename LaneRef<WIDE>::Off;
  LaneRef<WIDE> r;
  if (KIND == KF_AOSOA) {
    const int64_t B = int64_t(1) << lay.shift;
    r.boff = Off(((i >> lay.shift) * E * Lx * B + (i & (B - 1))) * 4);
  } else if (KIND == KF_AOS) {
    r.boff = Off(i * E * 4);
  } else {
    r.boff = Off(i * 4);
  }
  r.bytes = WIDE ? 0u : uint32_t(layout_floats(n, E, Lx, lay) * 4);
  return r;
}

// SZ: bytes per element (4, or 8 for the FP64 form, which addresses with
// 64-bit pointers: the buffer form above moves dwords only).  POL: the cache
// policy of ld_all / ld_first / st_all in the buffer form.
template <int KIND, bool WIDE, int SZ = 4, int POL = 0>
struct Lanes {
  static_assert(SZ == 4 || (SZ == 8 && WIDE), "FP64 arrays use the 64-bit address form");
  LaneRef<WIDE> par, cov, hp, hc, ck;
  int64_t es, n;
  // L: layers of the hit arrays; Lck: slots of the checkpoint array
  __device__ __forceinline__ Lanes(int64_t i, int64_t n_, int L, TrackLayout lay, int Lck = -1) : n(n_) {
    if (Lck < 0) Lck = L;
    using Off = typename LaneRef<WIDE>::Off;
    if (KIND == KF_AOSOA) {
      const int64_t B = int64_t(1) << lay.shift;
      const int64_t blk = i >> lay.shift, lane = i & (B - 1);
      es = B;
      par.boff = Off((blk * 6 * B + lane) * SZ);
      cov.boff = Off((blk * 21 * B + lane) * SZ);
      hp.boff = Off((blk * 3 * L * B + lane) * SZ);
      hc.boff = Off((blk * 6 * L * B + lane) * SZ);
      ck.boff = Off((blk * 27 * Lck * B + lane) * SZ);
    } else if (KIND == KF_AOS) {
      es = 1;
      par.boff = Off(i * 6 * SZ);
      cov.boff = Off(i * 21 * SZ);
      hp.boff = Off(i * 3 * SZ);
      hc.boff = Off(i * 6 * SZ);
      ck.boff = Off(i * 27 * SZ);
    } else {
      es = n;
      par.boff = cov.boff = hp.boff = hc.boff = ck.boff = Off(i * SZ);
    }
    if (!WIDE) {
      par.bytes = uint32_t(layout_floats(n, 6, 1, lay) * 4);
      cov.bytes = uint32_t(layout_floats(n, 21, 1, lay) * 4);
      hp.bytes = uint32_t(layout_floats(n, 3, L, lay) * 4);
      hc.bytes = uint32_t(layout_floats(n, 6, L, lay) * 4);
      ck.bytes = uint32_t(layout_floats(n, 27, Lck, lay) * 4);
    }
  }
  // E consecutive elements of one layer (AoS records) from / to array `base`
  template <int E, class T>
  __device__ __forceinline__ void ld_all(const LaneRef<WIDE>& r, const T* base, int l, T* dst) const {
    static_assert(sizeof(T) == SZ, "element size");
    if constexpr (!WIDE) {
      const __amdgpu_buffer_rsrc_t rs = buf_rsrc(base, r.bytes);
      if (KIND == KF_AOS) {
        buf_ld_rec<E, POL>(rs, uint32_t(r.boff), uint32_t(uni(E, l, 0)) * 4u, dst);
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) dst[e] = buf_ld<POL>(rs, uint32_t(r.boff), uint32_t(uni(E, l, e)) * 4u);
      }
    } else if (KIND == KF_AOS) {
      ld_rec<E>(r.at(base, uni(E, l, 0)), dst);
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) dst[e] = *r.at(base, uni(E, l, e));
    }
  }
  // the first N of the E elements of one layer
  template <int E, int N, class T>
  __device__ __forceinline__ void ld_first(const LaneRef<WIDE>& r, const T* base, int l, T* dst) const {
    static_assert(sizeof(T) == SZ && N <= E, "element size, count");
    if constexpr (!WIDE) {
      const __amdgpu_buffer_rsrc_t rs = buf_rsrc(base, r.bytes);
      if (KIND == KF_AOS) {
        buf_ld_rec<N, POL>(rs, uint32_t(r.boff), uint32_t(uni(E, l, 0)) * 4u, dst);
      } else {
#pragma unroll
        for (int e = 0; e < N; ++e) dst[e] = buf_ld<POL>(rs, uint32_t(r.boff), uint32_t(uni(E, l, e)) * 4u);
      }
    } else if (KIND == KF_AOS) {
      ld_rec<N>(r.at(base, uni(E, l, 0)), dst);
    } else {
#pragma unroll
      for (int e = 0; e < N; ++e) dst[e] = *r.at(base, uni(E, l, e));
    }
  }
  // P: the stores' cache policy (default: the object's)
  template <int E, class T, int P = POL>
  __device__ __forceinline__ void st_all(const LaneRef<WIDE>& r, T* base, int l, const T* src) const {
    static_assert(sizeof(T) == SZ, "element size");
    if constexpr (!WIDE) {
      const __amdgpu_buffer_rsrc_t rs = buf_rsrc(base, r.bytes);
      if (KIND == KF_AOS) {
        buf_st_rec<E, P>(rs, uint32_t(r.boff), uint32_t(uni(E, l, 0)) * 4u, src);
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) buf_st<P>(rs, uint32_t(r.boff), uint32_t(uni(E, l, e)) * 4u, src[e]);
      }
    } else if (KIND == KF_AOS) {
      st_rec<E>(r.at(base, uni(E, l, 0)), src);
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) *r.at(base, uni(E, l, e)) = src[e];
    }
  }
  // Asynchronous copy of the E elements of one layer straight into LDS:
  // element e of lane j lands at lds[e * 64 + j] (lds wave-uniform).  The
  // layer is min(j_uni, the lane's last layer): j_uni is wave-uniform and
  // <= L - 1, last_off the lane's byte offset of its last layer (layer_off).
  // Completion is tracked by the wave's vector-memory counter only; the
  // caller waits before reading.  POLICY: the copies' cache-policy bits.
  template <int E, int POLICY = 0>
  __device__ __forceinline__ void stage(const LaneRef<WIDE>& r, const float* base, int j_uni,
                                        typename LaneRef<WIDE>::Off last_off, float* lds) const {
    using Off = typename LaneRef<WIDE>::Off;
    const int64_t lstride = KIND == KF_AOS ? n * E : int64_t(E) * es;  // floats per layer
    Off off = r.boff + Off(j_uni) * Off(lstride * 4);
    off = off < last_off ? off : last_off;
    if constexpr (!WIDE) {
      const __amdgpu_buffer_rsrc_t rs = buf_rsrc(base, r.bytes);
#pragma unroll
      for (int e = 0; e < E; ++e)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void*)(lds + e * 64), 4, int(off), int(uint32_t(e * es * 4)),
                                                 0, POLICY);
    } else {
      const float* p = reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + off);
#pragma unroll
      for (int e = 0; e < E; ++e)
        __builtin_amdgcn_global_load_lds((gbl_void*)(p + e * es), (lds_void*)(lds + e * 64), 4, 0, POLICY);
    }
  }
  // byte offset of this lane's layer l (element 0) in a per-layer array of E elements
  template <int E>
  __device__ __forceinline__ typename LaneRef<WIDE>::Off layer_off(const LaneRef<WIDE>& r, int l) const {
    using Off = typename LaneRef<WIDE>::Off;
    const int64_t lstride = KIND == KF_AOS ? n * E : int64_t(E) * es;
    return r.boff + Off(l) * Off(lstride * 4);
  }
  // wave-uniform part of the offset of element e (of E) on layer l, in floats
  __device__ __forceinline__ int64_t uni(int E, int l, int e) const {
    const int64_t lstride = KIND == KF_AOS ? n * E : int64_t(E) * es;
    return int64_t(l) * lstride + int64_t(e) * es;
  }
};

}  // namespace kf

// Mixed-geometry, uneven-length batches: one persistent launch.
//
// Planning, on the device, every call (so the whole call can be captured once
// into a hipGraph and replayed):
//   1. clear      zero the bucket counters and the work counters
//   2. count      histogram of tracks over buckets (geometry, layer count);
//                 its last block lays the buckets out in decreasing estimated
//                 cost (layer count, a cylinder layer costing about twice a
//                 plane layer), each rounded up to whole work items of W = 64 *
//                 tracks_per_thread tracks (slots past a bucket's count are
//                 skipped)
//   3. scatter    track indices into their bucket's slots
//   4. run        persistent waves claim items, longest first, and find an
//                 item's bucket by binary search over the item layout; an item
//                 holds tracks of one geometry and one layer count, so a wave
//                 never diverges on either.
// A work item's tracks are gathered by index: their state through the track
// layout, their hits from ragged per-track runs.
#include "kf_batched.h"

#include <mutex>
#include "kf_lanes.h"
#include "kf_track.h"

namespace kf {

__host__ __device__ inline int bucket_of(uint8_t geom, int nl, int max_layers) {
  const int g = geom ? 1 : 0;
  const int l = nl < 0 ? 0 : (nl > max_layers ? max_layers : nl);
  return g * (KF_MAX_LAYERS + 1) + l;
}

// Layers track i runs: n_layers_per_track clamped to [0, L], or 0 when its hit
// rows would fall outside [0, n_hits).
__device__ __forceinline__ bool bad_hits(const BatchedArgs& a, int64_t i, int nl) {
  const int64_t off = a.hit_offset[i];
  return nl > 0 && (off < 0 || off > a.n_hits - nl);
}
__device__ __forceinline__ int track_layers(const BatchedArgs& a, int64_t i) {
  int nl = a.nlay[i];
  nl = nl < 0 ? 0 : (nl > a.L ? a.L : nl);
  return bad_hits(a, i, nl) ? 0 : nl;
}

__global__ void __launch_bounds__(256) kf_plan_clear(BatchedArgs a) {
  for (int b = threadIdx.x; b < KF_NBUCKETS; b += blockDim.x) {
    a.ws.bucket_count[b] = 0;
    a.ws.bucket_cursor[b] = 0;
  }
  if (threadIdx.x < 4) a.ws.counter[threadIdx.x] = 0;
}

// Per-block histograms in LDS, one global atomic per (block, bucket).  The
// last block to finish (a done-counter after a fence) then lays the buckets
// out: in the order given by a.order (decreasing cost), each rounded up to
// whole items of W = 64 * tracks_per_thread slots; it writes every bucket's
// first slot, the first item of every order position, and the item count.
__global__ void __launch_bounds__(256) kf_plan_count(BatchedArgs a) {
  __shared__ int hist[KF_NBUCKETS];
  __shared__ int base_item[KF_NBUCKETS + 1];
  __shared__ bool last;
  for (int b = threadIdx.x; b < KF_NBUCKETS; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += int64_t(gridDim.x) * blockDim.x)
    atomicAdd(&hist[bucket_of(a.geom[i], track_layers(a, i), a.L)], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < KF_NBUCKETS; b += blockDim.x)
    if (hist[b]) atomicAdd(&a.ws.bucket_count[b], hist[b]);
  // The counts are device-scope atomics, performed where every XCD sees them:
  // once this block's have been acknowledged (all counters waited to zero) it
  // may report itself done -- no cache write-back is needed for atomics, and a
  // full fence here (an L2 write-back on this part) costs more than the scan.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(&a.ws.counter[2], 1) == int(gridDim.x) - 1;
  __syncthreads();
  if (!last) return;
  // every block's counts are in; read them at the same place (atomics), in cost order
  for (int j = threadIdx.x; j < KF_NBUCKETS; j += blockDim.x) hist[j] = atomicAdd(&a.ws.bucket_count[a.order[j]], 0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int wsh = a.tpt == 2 ? 7 : 6;  // log2(W)
    const int W = 1 << wsh;
    int items = 0;
    for (int j = 0; j < KF_NBUCKETS; ++j) {
      base_item[j] = items;
      items += (hist[j] + W - 1) >> wsh;
    }
    base_item[KF_NBUCKETS] = items;
    a.ws.counter[1] = items;
  }
  __syncthreads();
  const int W = 64 * a.tpt;
  for (int j = threadIdx.x; j <= KF_NBUCKETS; j += blockDim.x) {
    a.ws.item_base[j] = base_item[j];
    if (j < KF_NBUCKETS) a.ws.bucket_base[a.order[j]] = base_item[j] * W;
  }
}

// Track indices into their bucket's slots: ranks within the block from LDS
// atomics, one global atomic per (block, bucket) to reserve the range.
__global__ void __launch_bounds__(256) kf_plan_scatter(BatchedArgs a) {
  constexpr int kPer = 4;  // tracks per thread
  __shared__ int local[KF_NBUCKETS];
  __shared__ int start[KF_NBUCKETS];
  for (int b = threadIdx.x; b < KF_NBUCKETS; b += blockDim.x) local[b] = 0;
  __syncthreads();
  int bk[kPer], rk[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int64_t i = (int64_t(blockIdx.x) * kPer + u) * blockDim.x + threadIdx.x;
    bk[u] = -1;
    if (i < a.n) {
      bk[u] = bucket_of(a.geom[i], track_layers(a, i), a.L);
      rk[u] = atomicAdd(&local[bk[u]], 1);
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < KF_NBUCKETS; c += blockDim.x)
    start[c] = local[c] ? atomicAdd(&a.ws.bucket_cursor[c], local[c]) : 0;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int64_t i = (int64_t(blockIdx.x) * kPer + u) * blockDim.x + threadIdx.x;
    if (bk[u] >= 0) a.ws.perm[a.ws.bucket_base[bk[u]] + start[bk[u]] + rk[u]] = int32_t(i);
  }
}

// ---------------------------------------------------------------- the run
template <int KIND, bool WIDE>
struct GatherState {
  const BatchedArgs& a;
  const Lanes<KIND, WIDE>& ln;
  bool valid;  // false: a lane without a track of its own, which stores nothing
  __device__ __forceinline__ bool load(float p[6], float C[21]) const {
    ln.template ld_all<6>(ln.par, a.par_in, 0, p);
    ln.template ld_all<21>(ln.cov, a.cov_in, 0, C);
    bool ok = true;
#pragma unroll
    for (int e = 0; e < 6; ++e) ok = ok & fin(p[e]);
#pragma unroll
    for (int e = 0; e < 21; ++e) ok = ok & fin(C[e]);
    return ok;
  }
  __device__ __forceinline__ void store(const float p[6], const float C[21]) const {
    if (!valid) return;
    ln.template st_all<6>(ln.par, a.par_out, 0, p);
    ln.template st_all<21>(ln.cov, a.cov_out, 0, C);
  }
};

// hits of a track: rows hit_offset[t] .. hit_offset[t] + n_layers - 1 of the
// ragged [n_hits][3] and [n_hits][6] arrays (the recompute path)
struct RaggedHits {
  const float* hp;
  const float* hc;
  __device__ __forceinline__ void load(int k, float m[3], float V[6]) const {
    ld_rec<3>(hp + 3 * k, m);
    ld_rec<6>(hc + 6 * k, V);
  }
};

// The ragged hits of a work item, staged through LDS in chunks of kChunk
// layers, double-buffered.  A track's rows for one chunk are contiguous in
// each array (kChunk * 12 and kChunk * 24 bytes), so the wave copies them
// cooperatively: copy g of a chunk moves rows r = 64 g + lane, i.e. layer
// r % kChunk of track r / kChunk, one element per instruction, straight into
// LDS.  Fetching a track's rows for several layers at once uses most of every
// line it touches; one lane reading its own 12- and 24-byte rows a layer at a
// time fetched about five times the bytes it used.
// Buffer: positions [kChunk][3][64] floats, then covariances [kChunk][6][64].
#ifndef KF_CHUNK_LAYERS
#define KF_CHUNK_LAYERS 4
#endif
#ifndef KF_CHUNK_BUFS
#define KF_CHUNK_BUFS 2
#endif
constexpr int kChunk = KF_CHUNK_LAYERS;
constexpr int kChunkBufs = KF_CHUNK_BUFS;  // 2: the next chunk fetched a chunk ahead; 1: a layer ahead
constexpr int kChunkFloats = kChunk * 64 * 9;
constexpr int kChunkLdsFloats = kChunkBufs * kChunkFloats;  // per wave
constexpr int kDmaLdsLimit = 65536;  // bytes of a block's LDS that copies into LDS can address
static_assert(kChunkBufs == 1 || 9 * kChunk < 64, "a chunk's copies must fit the wave's vector-memory counter");
static_assert(kChunkBufs == 1 || kChunkBufs == 2, "one or two chunk buffers");

template <bool WIDE>
struct ChunkRing {
  static constexpr bool kCooperative = true;
  const float* hp;  // array bases
  const float* hc;
  uint32_t hp_bytes, hc_bytes;
  float* buf;   // kChunkLdsFloats of LDS, wave-uniform
  int64_t h0;   // this lane's first row
  int last;     // the item's layer count - 1 (wave-uniform)
  int cnt;      // tracks in this wave's share of the item: lanes 0 .. cnt-1 (wave-uniform)
  __device__ __forceinline__ void issue(int q, float* dst) const {
    const int lane = int(threadIdx.x & 63);
#pragma unroll
    for (int g = 0; g < kChunk; ++g) {
      const int r = g * 64 + lane;
      int j = r / kChunk;
      j = j < cnt ? j : cnt - 1;  // rows of lanes without a track: repeat a valid one
      const int c = r % kChunk;
      const int layer = q * kChunk + c < last ? q * kChunk + c : last;
      float* dp = dst + g * 3 * 64;
      float* dc = dst + kChunk * 3 * 64 + g * 6 * 64;
      if constexpr (!WIDE) {
        const uint32_t row = uint32_t(__shfl(int(h0), j, 64)) + uint32_t(layer);
        const __amdgpu_buffer_rsrc_t rp = buf_rsrc(hp, hp_bytes);
        const __amdgpu_buffer_rsrc_t rc = buf_rsrc(hc, hc_bytes);
#pragma unroll
        for (int e = 0; e < 3; ++e)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rp, (lds_void*)(dp + e * 64), 4, int(row * 12u), e * 4, 0, 0);
#pragma unroll
        for (int e = 0; e < 6; ++e)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rc, (lds_void*)(dc + e * 64), 4, int(row * 24u), e * 4, 0, 0);
      } else {
        const int lo = __shfl(int(uint32_t(uint64_t(h0))), j, 64);
        const int hi = __shfl(int(uint32_t(uint64_t(h0) >> 32)), j, 64);
        const int64_t row = int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo)) + layer;
        const float* sp = hp + row * 3;
        const float* sc = hc + row * 6;
#pragma unroll
        for (int e = 0; e < 3; ++e) __builtin_amdgcn_global_load_lds((gbl_void*)(sp + e), (lds_void*)(dp + e * 64), 4, 0, 0);
#pragma unroll
        for (int e = 0; e < 6; ++e) __builtin_amdgcn_global_load_lds((gbl_void*)(sc + e), (lds_void*)(dc + e * 64), 4, 0, 0);
      }
    }
  }
  __device__ __forceinline__ void begin() { issue(0, buf); }
  __device__ __forceinline__ void get(int k, float m[3], float V[6]) {
    const int q = k / kChunk, c = k % kChunk;
    const float* cur = kChunkBufs == 2 ? buf + (q & 1) * kChunkFloats : buf;
    if (c == 0) {
      if constexpr (kChunkBufs == 2) {
        // the other buffer (chunk q - 1) has been read; refill it with chunk q + 1
        wait_lds();
        if ((q + 1) * kChunk <= last) {
          issue(q + 1, buf + ((q + 1) & 1) * kChunkFloats);
          wait_vmem<9 * kChunk>();
        } else {
          wait_vmem<0>();
        }
      } else {
        wait_vmem<0>();  // chunk q, requested during the chunk before
      }
    }
    const int r = int(threadIdx.x & 63) * kChunk + c;
    const int g = r >> 6, l = r & 63;
#pragma unroll
    for (int e = 0; e < 3; ++e) m[e] = cur[(g * 3 + e) * 64 + l];
#pragma unroll
    for (int e = 0; e < 6; ++e) V[e] = cur[kChunk * 3 * 64 + (g * 6 + e) * 64 + l];
    if constexpr (kChunkBufs == 1) {
      // the chunk's last layer is read: refill the buffer with the next chunk
      if (c == kChunk - 1 && (q + 1) * kChunk <= last) {
        wait_lds();
        issue(q + 1, buf);
      }
    }
  }
  __device__ __forceinline__ void end() { wait_vmem<0>(); }
};

// Every lane of the wave calls this (the hits are copied cooperatively);
// lanes past the item's last track (valid = false) repeat the item's first
// track and store nothing.
template <int PREC, int KIND, bool WIDE>
__device__ __forceinline__ void run_one(const BatchedArgs& a, int64_t t, bool valid, int geom, int nl, int cnt,
                                        float* ring) {
  const Lanes<KIND, WIDE> ln(t, a.n, 1, a.lay);
  const int64_t h0 = a.hit_offset[t];
  const RaggedHits hits{a.hit_pos + h0 * 3, a.hit_cov + h0 * 6};
  ChunkRing<WIDE> stager{a.hit_pos, a.hit_cov, uint32_t(a.n_hits * 12), uint32_t(a.n_hits * 24), ring, h0,
                         nl > 0 ? nl - 1 : 0, cnt};
  const GatherState<KIND, WIDE> state{a, ln, valid};
  float chi2;
  uint32_t status;
  if (geom == 0)
    run_track<0, PREC>(state, hits, stager, NoCkpt{}, nl, a.layer_z, a.b, chi2, status);
  else
    run_track<1, PREC>(state, hits, stager, NoCkpt{}, nl, a.layer_r, a.b, chi2, status);
  if (!valid) return;
  if (nl == 0) {
    int nt = a.nlay[t];
    nt = nt < 0 ? 0 : (nt > a.L ? a.L : nt);
    if (bad_hits(a, t, nt)) status |= KF_S_BAD_HITS;
  }
  if (a.chi2) a.chi2[t] = chi2;
  if (a.status) a.status[t] = int32_t(status);
}

// Every wave loops over work items until the items run out -- which every
// wave reaches, item numbers only grow.  Schedules:
//   KF_SCHED_DYNAMIC  first item = the wave's number, then lane 0 claims the
//                     next one from an atomic counter (broadcast to the wave)
//   KF_SCHED_STATIC   items wave, wave + n_waves, wave + 2 n_waves, ...
//                     (no atomics; the items are already longest-first)
template <int PREC, int KIND, bool WIDE>
__global__ void __launch_bounds__(256) kf_batched_kernel(const BatchedArgs a) {
  extern __shared__ float kf_lds[];
  float* ring = kf_lds + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)) * kChunkLdsFloats;
  __shared__ int item_base[KF_NBUCKETS + 1];  // first item of each order position
  for (int j = threadIdx.x; j <= KF_NBUCKETS; j += blockDim.x) item_base[j] = a.ws.item_base[j];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int W = 64 * a.tpt;
  const int n_waves = int(gridDim.x * (blockDim.x >> 6));
  const int n_items = item_base[KF_NBUCKETS];
  int item = int(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  while (item < n_items) {
    int lo = 0, hi = KF_NBUCKETS - 1;  // the last order position whose first item is <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (item_base[mid] <= item) lo = mid; else hi = mid - 1;
    }
    const int b = a.order[lo];
    const int geom = b / (KF_MAX_LAYERS + 1);
    const int nl = b % (KF_MAX_LAYERS + 1);
    const int64_t slot0 = int64_t(item) * W;
    const int64_t end = int64_t(a.ws.bucket_base[b]) + a.ws.bucket_count[b];  // first slot past the bucket
    for (int u = 0; u < a.tpt; ++u) {
      const int64_t first = slot0 + u * 64;  // slots first .. first + 63 of this pass
      const int cnt = end - first >= 64 ? 64 : int(end - first);
      if (cnt <= 0) break;
      const int64_t slot = first + lane;
      const bool valid = slot < end;
      run_one<PREC, KIND, WIDE>(a, a.ws.perm[valid ? slot : first], valid, geom, nl, cnt, ring);
    }
    if (a.schedule == KF_SCHED_STATIC) {
      item += n_waves;
    } else {
      int next = 0;
      if (lane == 0) next = atomicAdd(&a.ws.counter[0], 1);
      item = n_waves + __shfl(next, 0, 64);
    }
  }
}

// Enough waves to fill every CU at the kernel's occupancy, no more.
template <int PREC, int KIND, bool WIDE>
static hipError_t launch_run(const BatchedArgs& a, int block, hipStream_t s) {
  int dev = 0, n_cu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0)
    return hipErrorInvalidDevice;
  int max_lds = 0;
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return hipErrorInvalidDevice;
  // copies straight into LDS address their destination through the low 16
  // bits of M0: every wave's chunk buffers must lie in the block's first 64 KiB
  if (max_lds > kDmaLdsLimit) max_lds = kDmaLdsLimit;
  const int per_wave = kChunkLdsFloats * int(sizeof(float));
  while (block > 64 && (block / 64) * per_wave > max_lds) block /= 2;  // the chunk buffers must fit a block
  if (per_wave > max_lds) return hipErrorInvalidConfiguration;
  const size_t lds = size_t(block / 64) * per_wave;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kf_batched_kernel<PREC, KIND, WIDE>, block, lds) !=
          hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  const int mult = a.waves_mult > 0 ? a.waves_mult : 1;
  hipLaunchKernelGGL((kf_batched_kernel<PREC, KIND, WIDE>), dim3(unsigned(per_cu * n_cu * mult)), dim3(block), lds, s,
                     a);
  return hipGetLastError();
}

template <int PREC>
static hipError_t launch_kinds(const BatchedArgs& a, int block, bool wide, hipStream_t s) {
  if (a.lay.kind == KF_AOS)
    return wide ? launch_run<PREC, KF_AOS, true>(a, block, s) : launch_run<PREC, KF_AOS, false>(a, block, s);
  if (a.lay.kind == KF_AOSOA)
    return wide ? launch_run<PREC, KF_AOSOA, true>(a, block, s) : launch_run<PREC, KF_AOSOA, false>(a, block, s);
  return wide ? launch_run<PREC, KF_SOA, true>(a, block, s) : launch_run<PREC, KF_SOA, false>(a, block, s);
}

hipError_t launch_batched(const BatchedArgs& a, int prec, int block, hipStream_t s) {
  const int64_t blocks = (a.n + 255) / 256;
  const unsigned g_count = unsigned(blocks < 1 ? 1 : (blocks > 256 ? 256 : blocks));
  const unsigned g_scatter = unsigned((a.n + 1023) / 1024 > 0 ? (a.n + 1023) / 1024 : 1);
  hipLaunchKernelGGL(kf_plan_clear, dim3(1), dim3(256), 0, s, a);
  hipLaunchKernelGGL(kf_plan_count, dim3(g_count), dim3(256), 0, s, a);
  hipLaunchKernelGGL(kf_plan_scatter, dim3(g_scatter), dim3(256), 0, s, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // 64-bit addressing when the state arrays or the ragged covariance rows span 4 GiB
  const bool wide = needs_wide(a.n, 1, a.lay) || a.n_hits * 24 >= (int64_t(1) << 32);
  if (prec == 0) return launch_kinds<PREC_F32>(a, block, wide, s);
  if (prec == 1) return launch_kinds<PREC_F64>(a, block, wide, s);
  return launch_kinds<PREC_F64_JOSEPH>(a, block, wide, s);
}

// Order of buckets by decreasing estimated cost: layers x (2 for cylinders).
void bucket_order(int32_t order[KF_NBUCKETS]) {
  int cost[KF_NBUCKETS];
  for (int b = 0; b < KF_NBUCKETS; ++b) {
    order[b] = b;
    cost[b] = (b % (KF_MAX_LAYERS + 1)) * (b / (KF_MAX_LAYERS + 1) ? 2 : 1);
  }
  // insertion sort, stable: equal costs keep plane buckets first
  for (int i = 1; i < KF_NBUCKETS; ++i) {
    const int v = order[i];
    int j = i - 1;
    while (j >= 0 && cost[order[j]] < cost[v]) {
      order[j + 1] = order[j];
      --j;
    }
    order[j + 1] = v;
  }
}

}  // namespace kf

namespace kf {

static int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

// most slots: every bucket padded to whole 128-track items
static int64_t max_slots(int64_t n) { return n + int64_t(KF_NBUCKETS + 1) * 128; }

int64_t batched_workspace_bytes(int64_t n) {
  return align256(4 * (4 * KF_NBUCKETS + 5)) + align256(4 * max_slots(n));
}

// The planning workspace of kf_propagate_update_batched_noalloc: a fixed
// device array, one per device, sized for KF_NOALLOC_MAX_TRACKS tracks
// (about 4 MiB), held until the process ends.  In host code its name is a
// host-side stand-in, not a device address: host code uses only the
// address that hipGetSymbolAddress returns for the current device.
constexpr int64_t kScratchBytes = (((4 * (4 * KF_NBUCKETS + 5)) + 255) & ~int64_t(255)) +
                                  ((4 * (KF_NOALLOC_MAX_TRACKS + int64_t(KF_NBUCKETS + 1) * 128) + 255) & ~int64_t(255));
static __device__ __align__(256) char scratch[kScratchBytes];

hipError_t noalloc_scratch(int dev, void** ptr, int64_t* bytes) {
  static std::mutex mu;
  static void* addr[64];
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = kScratchBytes;
  return hipSuccess;
}

bool batched_carve(void* ws, int64_t bytes, int64_t n, BatchedWorkspace* out) {
  if (!ws || bytes < batched_workspace_bytes(n)) return false;
  char* p = static_cast<char*>(ws);
  int32_t* head = reinterpret_cast<int32_t*>(p);
  out->bucket_count = head;
  out->bucket_cursor = head + KF_NBUCKETS;
  out->bucket_base = head + 2 * KF_NBUCKETS;
  out->counter = head + 3 * KF_NBUCKETS;
  out->item_base = head + 3 * KF_NBUCKETS + 4;
  p += align256(4 * (4 * KF_NBUCKETS + 5));
  out->perm = reinterpret_cast<int32_t*>(p);
  return true;
}

}  // namespace kf

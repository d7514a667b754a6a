// Host-resident form of the step: chunks of tracks stream through the GPU on
// several HIP streams, so the copies of one chunk overlap the kernel of
// another -- the time the paper measures with its transfers included.
//
// Per chunk, on stream (chunk mod n_streams): host-to-device copies of the
// chunk's state and hits, the step kernel on the chunk's device buffers (the
// same launcher and kernels as the device-resident calls), device-to-host
// copies of its results.  Every array keeps its layout; a chunk of c tracks
// is itself an array of c tracks in that layout:
//   SoA      row (l, e) of the chunk = c floats of row (l, e) of the whole
//            array: one 2D copy (rows of c floats, source pitch n floats)
//   AoS      layer l of the chunk = c*E floats of layer l: one 2D copy
//   AoSoA-B  whole blocks of B tracks (chunks are multiples of B): one copy
// The device buffers and streams of the last configuration are kept per
// device and reused; kf_host_release frees them.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "kf_host.h"
#include "kf_lanes.h"

namespace kf {

namespace {

struct StreamSet {
  hipStream_t s = nullptr;
  float *par = nullptr, *cov = nullptr, *hp = nullptr, *hc = nullptr;
  float *par_out = nullptr, *cov_out = nullptr, *chi2 = nullptr;
  int32_t *status = nullptr, *nlay = nullptr;
};

struct DeviceCache {
  int64_t chunk = 0;  // tracks per chunk the buffers hold
  int32_t L = 0;
  TrackLayout lay{-1, 0};
  std::vector<StreamSet> sets;
};

std::mutex g_mu;
DeviceCache g_cache[64];

void free_set(StreamSet& st) {
  float* fs[] = {st.par, st.cov, st.hp, st.hc, st.par_out, st.cov_out, st.chi2};
  for (float* p : fs)
    if (p) (void)hipFree(p);
  if (st.status) (void)hipFree(st.status);
  if (st.nlay) (void)hipFree(st.nlay);
  if (st.s) (void)hipStreamDestroy(st.s);
  st = StreamSet{};
}

void free_cache(DeviceCache& c) {
  for (StreamSet& st : c.sets) free_set(st);
  c = DeviceCache{};
}

template <class T>
hipError_t alloc(T** p, int64_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), size_t(count > 0 ? count : 1) * sizeof(T));
}

hipError_t ensure(DeviceCache& c, int64_t chunk, int32_t L, TrackLayout lay, int n_streams) {
  if (c.chunk >= chunk && c.L >= L && c.lay.kind == lay.kind && c.lay.shift == lay.shift &&
      int(c.sets.size()) >= n_streams)
    return hipSuccess;
  free_cache(c);
  c.chunk = chunk;
  c.L = L;
  c.lay = lay;
  c.sets.resize(size_t(n_streams));
  const int Lh = L > 0 ? L : 1;
  for (StreamSet& st : c.sets) {
    hipError_t e = hipStreamCreateWithFlags(&st.s, hipStreamNonBlocking);
    if (e == hipSuccess) e = alloc(&st.par, layout_floats(chunk, 6, 1, lay));
    if (e == hipSuccess) e = alloc(&st.cov, layout_floats(chunk, 21, 1, lay));
    if (e == hipSuccess) e = alloc(&st.hp, layout_floats(chunk, 3, Lh, lay));
    if (e == hipSuccess) e = alloc(&st.hc, layout_floats(chunk, 6, Lh, lay));
    if (e == hipSuccess) e = alloc(&st.par_out, layout_floats(chunk, 6, 1, lay));
    if (e == hipSuccess) e = alloc(&st.cov_out, layout_floats(chunk, 21, 1, lay));
    if (e == hipSuccess) e = alloc(&st.chi2, chunk);
    if (e == hipSuccess) e = alloc(&st.status, chunk);
    if (e == hipSuccess) e = alloc(&st.nlay, chunk);
    if (e != hipSuccess) {
      free_cache(c);
      return e;
    }
  }
  return hipSuccess;
}

// Copy the chunk [t0, t0 + c) of an array of E elements and Lx layers between
// the whole host array (n tracks) and a chunk buffer (c tracks), both in `lay`.
hipError_t copy_chunk(float* dev, float* host, int E, int Lx, int64_t n, int64_t t0, int64_t c, TrackLayout lay,
                      bool to_device, hipStream_t s) {
  const hipMemcpyKind kind = to_device ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost;
  const size_t f = sizeof(float);
  if (lay.kind == KF_SOA) {
    float* h = host + t0;
    return to_device ? hipMemcpy2DAsync(dev, size_t(c) * f, h, size_t(n) * f, size_t(c) * f, size_t(Lx) * E, kind, s)
                     : hipMemcpy2DAsync(h, size_t(n) * f, dev, size_t(c) * f, size_t(c) * f, size_t(Lx) * E, kind, s);
  }
  if (lay.kind == KF_AOS) {
    float* h = host + t0 * E;
    const size_t w = size_t(c) * E * f, hp = size_t(n) * E * f;
    return to_device ? hipMemcpy2DAsync(dev, w, h, hp, w, size_t(Lx), kind, s)
                     : hipMemcpy2DAsync(h, hp, dev, w, w, size_t(Lx), kind, s);
  }
  const int64_t B = int64_t(1) << lay.shift;  // t0 is a multiple of B; whole blocks
  const int64_t blocks = (c + B - 1) / B;
  float* h = host + (t0 / B) * E * Lx * B;
  const size_t bytes = size_t(blocks * E * Lx * B) * f;
  return to_device ? hipMemcpyAsync(dev, h, bytes, kind, s) : hipMemcpyAsync(h, dev, bytes, kind, s);
}

}  // namespace

hipError_t run_host_pipeline(const HostCall& h, StepArgs base, int geom, int prec, int block, int tpt) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_mu);
  DeviceCache& c = g_cache[dev];
  const TrackLayout lay = base.lay;
  int64_t chunk = h.chunk < h.n ? h.chunk : h.n;
  if (lay.kind == KF_AOSOA) {
    const int64_t B = int64_t(1) << lay.shift;
    chunk = (chunk + B - 1) / B * B;
  }
  e = ensure(c, chunk, base.L, lay, h.n_streams);
  if (e != hipSuccess) return e;
  const int Lh = base.L > 0 ? base.L : 1;
  float* hp = const_cast<float*>(h.hit_pos);
  float* hc = const_cast<float*>(h.hit_cov);
  int64_t i = 0;
  for (int64_t t0 = 0; t0 < h.n; t0 += chunk, ++i) {
    StreamSet& st = c.sets[size_t(i % h.n_streams)];
    const int64_t cn = h.n - t0 < chunk ? h.n - t0 : chunk;
    if (e == hipSuccess) e = copy_chunk(st.par, const_cast<float*>(h.par_in), 6, 1, h.n, t0, cn, lay, true, st.s);
    if (e == hipSuccess) e = copy_chunk(st.cov, const_cast<float*>(h.cov_in), 21, 1, h.n, t0, cn, lay, true, st.s);
    if (e == hipSuccess && base.L > 0) e = copy_chunk(st.hp, hp, 3, Lh, h.n, t0, cn, lay, true, st.s);
    if (e == hipSuccess && base.L > 0) e = copy_chunk(st.hc, hc, 6, Lh, h.n, t0, cn, lay, true, st.s);
    if (e == hipSuccess && h.nlay)
      e = hipMemcpyAsync(st.nlay, h.nlay + t0, size_t(cn) * sizeof(int32_t), hipMemcpyHostToDevice, st.s);
    StepArgs a = base;
    a.par_in = st.par;
    a.cov_in = st.cov;
    a.par_out = st.par_out;
    a.cov_out = st.cov_out;
    a.hit_pos = st.hp;
    a.hit_cov = st.hc;
    a.nlay = h.nlay ? st.nlay : nullptr;
    a.chi2 = h.chi2 ? st.chi2 : nullptr;
    a.status = h.status ? st.status : nullptr;
    a.ckpt = nullptr;
    a.n = cn;
    if (e == hipSuccess) e = launch_step(geom, prec, block, tpt, a, st.s);
    if (e == hipSuccess) e = copy_chunk(st.par_out, h.par_out, 6, 1, h.n, t0, cn, lay, false, st.s);
    if (e == hipSuccess) e = copy_chunk(st.cov_out, h.cov_out, 21, 1, h.n, t0, cn, lay, false, st.s);
    if (e == hipSuccess && h.chi2)
      e = hipMemcpyAsync(h.chi2 + t0, st.chi2, size_t(cn) * sizeof(float), hipMemcpyDeviceToHost, st.s);
    if (e == hipSuccess && h.status)
      e = hipMemcpyAsync(h.status + t0, st.status, size_t(cn) * sizeof(int32_t), hipMemcpyDeviceToHost, st.s);
  }
  // the call returns with every result in host memory (also after an error:
  // nothing may still be writing into the caller's buffers)
  for (int k = 0; k < h.n_streams && k < int(c.sets.size()); ++k) {
    const hipError_t se = hipStreamSynchronize(c.sets[size_t(k)].s);
    if (e == hipSuccess) e = se;
  }
  return e;
}

void release_host_pipeline() {
  std::lock_guard<std::mutex> g(g_mu);
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return;
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return;
  for (int d = 0; d < n && d < 64; ++d) {
    if (g_cache[d].sets.empty()) continue;
    if (hipSetDevice(d) != hipSuccess) continue;
    free_cache(g_cache[d]);
  }
  (void)hipSetDevice(cur);
}

}  // namespace kf

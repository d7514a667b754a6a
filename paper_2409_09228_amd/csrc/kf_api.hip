// C ABI of libkf.so (declared in include/kf.h): argument validation and
// dispatch to the kernel launchers.  Nothing here allocates device memory
// (the host-resident pipeline's chunk buffers live in kf_host.hip).
#include <string.h>

#include <list>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>

#include "kf_batched.h"
#include "kf_host.h"
#include "kf_internal.h"
#include "kf_lanes.h"

namespace {

constexpr double kCLight = 0.00299792458;

bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

bool layout_ok(kf_layout_t lay, kf::TrackLayout* out) {
  if (lay.kind == KF_SOA || lay.kind == KF_AOS) {
    *out = {lay.kind, 0};
    return true;
  }
  if (lay.kind != KF_AOSOA) return false;
  for (int sh = 4; sh <= 8; ++sh)
    if (lay.block == (1 << sh)) {
      *out = {KF_AOSOA, sh};
      return true;
    }
  return false;
}

// The library only ships gfx950 code objects; refuse other devices up front
// instead of failing inside the launch.
kf_status_t device_ok() {
  static std::mutex mu;
  static int known[64];  // 0 unknown, 1 ok, 2 not ok
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return KF_E_DEVICE;
  std::lock_guard<std::mutex> g(mu);
  if (known[dev] == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return KF_E_DEVICE;
    known[dev] = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
  }
  return known[dev] == 1 ? KF_OK : KF_E_DEVICE;
}

// log2 of a checkpoint stride (0 -> 1; 1, 2, 4, .. 64), or -1
int ckpt_shift(int32_t every) {
  if (every == 0) return 0;
  for (int sh = 0; sh <= 6; ++sh)
    if (every == (1 << sh)) return sh;
  return -1;
}

kf_status_t step(int geom, const float* par_in, const float* cov_in, float* par_out, float* cov_out,
                 const float* hit_pos, const float* hit_cov, const float* layers, int32_t n_layers,
                 const int32_t* nlay, int64_t n_tracks, float bz, kf_layout_t layout, uint32_t flags,
                 float* chi2_out, int32_t* status_out, float* ckpt_out, int32_t ckpt_every,
                 const kf_tune_t* tune, void* stream) {
  if (n_tracks < 0 || n_layers < 0 || n_layers > KF_MAX_LAYERS) return KF_E_SHAPE;
  const int ck_shift = ckpt_shift(ckpt_every);
  if (ckpt_out && ck_shift < 0) return KF_E_SHAPE;
  kf::TrackLayout tl;
  if (!layout_ok(layout, &tl)) return KF_E_LAYOUT;
  if (flags & ~uint32_t(KF_F_PRECISION)) return KF_E_FLAGS;
  int block = 256, tpt = 1;
  if (tune) {
    block = tune->block_threads;
    tpt = tune->tracks_per_thread;
    if ((block != 64 && block != 128 && block != 256) || (tpt != 1 && tpt != 2) ||
        (tune->schedule != KF_SCHED_DYNAMIC && tune->schedule != KF_SCHED_STATIC) || tune->waves_mult < 0 ||
        tune->waves_mult > 8)
      return KF_E_FLAGS;
  }
  if (n_tracks == 0) return KF_OK;
  if (!par_in || !cov_in || !par_out || !cov_out) return KF_E_NULL;
  if (n_layers > 0 && (!hit_pos || !hit_cov || !layers)) return KF_E_NULL;
  const void* ptrs[] = {par_in, cov_in, par_out, cov_out, hit_pos, hit_cov, chi2_out, status_out, ckpt_out, nlay};
  for (const void* p : ptrs)
    if (p && !aligned4(p)) return KF_E_ALIGN;
  kf_status_t ds = device_ok();
  if (ds != KF_OK) return ds;

  kf::StepArgs a;
  a.par_in = par_in;
  a.cov_in = cov_in;
  a.par_out = par_out;
  a.cov_out = cov_out;
  a.hit_pos = hit_pos;
  a.hit_cov = hit_cov;
  a.nlay = nlay;
  a.chi2 = chi2_out;
  a.status = status_out;
  a.ckpt = ckpt_out;
  a.n = n_tracks;
  a.L = n_layers;
  a.ck_shift = ckpt_out ? ck_shift : 0;
  a.Lck = ckpt_out ? (n_layers + (1 << ck_shift) - 1) >> ck_shift : n_layers;
  a.lay = tl;
  a.b = float(kCLight * double(bz));
  for (int l = 0; l < KF_MAX_LAYERS; ++l) a.layer[l] = l < n_layers ? layers[l] : 0.0f;
  const int prec = (flags & KF_F_JOSEPH) ? 2 : ((flags & KF_F_FP64_INVERSE) ? 1 : 0);
  hipError_t e = kf::launch_step(geom, prec, block, tpt, a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? KF_OK : KF_E_LAUNCH;
}

kf_status_t step_f64(int geom, const double* par_in, const double* cov_in, double* par_out, double* cov_out,
                     const double* hit_pos, const double* hit_cov, const double* layers, int32_t n_layers,
                     const int32_t* nlay, int64_t n_tracks, double bz, kf_layout_t layout, uint32_t flags,
                     double* chi2_out, int32_t* status_out, const kf_tune_t* tune, void* stream) {
  if (n_tracks < 0 || n_layers < 0 || n_layers > KF_MAX_LAYERS) return KF_E_SHAPE;
  kf::TrackLayout tl;
  if (!layout_ok(layout, &tl)) return KF_E_LAYOUT;
  if (flags & ~uint32_t(KF_F_PRECISION)) return KF_E_FLAGS;
  int block = 256;
  if (tune) {
    block = tune->block_threads;
    if ((block != 64 && block != 128 && block != 256) || (tune->tracks_per_thread != 1 && tune->tracks_per_thread != 2))
      return KF_E_FLAGS;
  }
  if (n_tracks == 0) return KF_OK;
  if (!par_in || !cov_in || !par_out || !cov_out) return KF_E_NULL;
  if (n_layers > 0 && (!hit_pos || !hit_cov || !layers)) return KF_E_NULL;
  const void* ptrs8[] = {par_in, cov_in, par_out, cov_out, hit_pos, hit_cov, chi2_out};
  for (const void* p : ptrs8)
    if (p && (reinterpret_cast<uintptr_t>(p) & 7u)) return KF_E_ALIGN;
  if ((status_out && !aligned4(status_out)) || (nlay && !aligned4(nlay))) return KF_E_ALIGN;
  kf_status_t ds = device_ok();
  if (ds != KF_OK) return ds;
  kf::StepArgsT<double> a;
  memset(&a, 0, sizeof(a));
  a.par_in = par_in;
  a.cov_in = cov_in;
  a.par_out = par_out;
  a.cov_out = cov_out;
  a.hit_pos = hit_pos;
  a.hit_cov = hit_cov;
  a.nlay = nlay;
  a.chi2 = chi2_out;
  a.status = status_out;
  a.n = n_tracks;
  a.L = n_layers;
  a.Lck = n_layers;
  a.lay = tl;
  a.b = kCLight * bz;
  for (int l = 0; l < KF_MAX_LAYERS; ++l) a.layer[l] = l < n_layers ? layers[l] : 0.0;
  const int prec = (flags & KF_F_JOSEPH) ? 2 : 0;
  hipError_t e = kf::launch_step_f64(geom, prec, block, a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? KF_OK : KF_E_LAUNCH;
}

kf_status_t pack_common(const float* src, float* dst, int32_t n_elem, int32_t n_layers, int64_t n,
                        kf_layout_t layout, void* stream, bool to_layout) {
  if (n_elem <= 0 || n_layers <= 0 || n < 0) return KF_E_SHAPE;
  kf::TrackLayout tl;
  if (!layout_ok(layout, &tl)) return KF_E_LAYOUT;
  if (n == 0) return KF_OK;
  if (!src || !dst) return KF_E_NULL;
  if (!aligned4(src) || !aligned4(dst)) return KF_E_ALIGN;
  kf_status_t ds = device_ok();
  if (ds != KF_OK) return ds;
  hipError_t e = kf::launch_pack(src, dst, n_elem, n_layers, n, tl, to_layout, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? KF_OK : KF_E_LAUNCH;
}

// ------------------------------------------------------------ graph cache
// Executable graphs of whole batched calls, keyed by every argument of the
// call (pointers, sizes, tables, precision, launch shape) and the device.
// Least recently used entries are destroyed beyond kMaxGraphs.
constexpr size_t kMaxGraphs = 32;

struct GraphCache {
  std::mutex mu;
  std::list<std::pair<std::string, hipGraphExec_t>> lru;  // front = most recent
  std::unordered_map<std::string, std::list<std::pair<std::string, hipGraphExec_t>>::iterator> index;
  hipStream_t capture[64] = {};
};

GraphCache& graphs() {
  static GraphCache* g = new GraphCache();  // never destroyed: no HIP calls at exit
  return *g;
}

kf_status_t batched_via_graph(const kf::BatchedArgs& a, int prec, int block, int dev, hipStream_t stream) {
  std::string key(reinterpret_cast<const char*>(&a), sizeof(a));
  key.append(reinterpret_cast<const char*>(&prec), sizeof(prec));
  key.append(reinterpret_cast<const char*>(&block), sizeof(block));
  key.append(reinterpret_cast<const char*>(&dev), sizeof(dev));
  GraphCache& gc = graphs();
  std::lock_guard<std::mutex> g(gc.mu);
  hipGraphExec_t exec = nullptr;
  auto it = gc.index.find(key);
  if (it != gc.index.end()) {
    gc.lru.splice(gc.lru.begin(), gc.lru, it->second);
    exec = it->second->second;
  } else {
    if (!gc.capture[dev] && hipStreamCreateWithFlags(&gc.capture[dev], hipStreamNonBlocking) != hipSuccess)
      return KF_E_LAUNCH;
    hipStream_t cs = gc.capture[dev];
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return KF_E_LAUNCH;
    const hipError_t le = kf::launch_batched(a, prec, block, cs);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(cs, &graph);
    if (le != hipSuccess || ce != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return KF_E_LAUNCH;
    }
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ie != hipSuccess) return KF_E_LAUNCH;
    gc.lru.emplace_front(key, exec);
    gc.index[key] = gc.lru.begin();
    while (gc.lru.size() > kMaxGraphs) {
      hipGraphExecDestroy(gc.lru.back().second);
      gc.index.erase(gc.lru.back().first);
      gc.lru.pop_back();
    }
  }
  return hipGraphLaunch(exec, stream) == hipSuccess ? KF_OK : KF_E_LAUNCH;
}

}  // namespace

extern "C" {

kf_status_t kf_chi2_backward(int32_t geometry, const float* par_in, const float* cov_in, const float* hit_pos,
                             const float* hit_cov, const float* layers, int32_t n_layers, int64_t n_tracks,
                             float bz_tesla, kf_layout_t layout, const int32_t* status_fwd, const float* ckpt,
                             int32_t ckpt_every, const float* grad_chi2, float* grad_hit_pos, float* grad_par_in,
                             float* grad_cov_in, const kf_tune_t* tune, void* stream) {
  if (geometry != 0 && geometry != 1) return KF_E_SHAPE;
  if (n_tracks < 0 || n_layers < 0 || n_layers > KF_MAX_LAYERS) return KF_E_SHAPE;
  const int ck_shift = ckpt_shift(ckpt_every);
  if (ckpt && ck_shift < 0) return KF_E_SHAPE;
  kf::TrackLayout tl;
  if (!layout_ok(layout, &tl)) return KF_E_LAYOUT;
  int block = 256;
  if (tune) {
    block = tune->block_threads;
    if (block != 64 && block != 128 && block != 256) return KF_E_FLAGS;
  }
  if (n_tracks == 0) return KF_OK;
  if (!par_in || !cov_in || !status_fwd || !grad_chi2 || !grad_par_in) return KF_E_NULL;
  if (n_layers > 0 && (!hit_pos || !hit_cov || !layers || !grad_hit_pos)) return KF_E_NULL;
  const void* ptrs[] = {par_in, cov_in, hit_pos, hit_cov, status_fwd, ckpt, grad_chi2, grad_hit_pos, grad_par_in,
                        grad_cov_in};
  for (const void* p : ptrs)
    if (p && !aligned4(p)) return KF_E_ALIGN;
  kf_status_t ds = device_ok();
  if (ds != KF_OK) return ds;
  kf::AdjointArgs a;
  a.par_in = par_in;
  a.cov_in = cov_in;
  a.hit_pos = hit_pos;
  a.hit_cov = hit_cov;
  a.ckpt = ckpt;
  a.status = status_fwd;
  a.grad_chi2 = grad_chi2;
  a.grad_hit = grad_hit_pos;
  a.grad_par = grad_par_in;
  a.grad_cov = grad_cov_in;
  a.n = n_tracks;
  a.L = n_layers;
  a.ck_shift = ckpt ? ck_shift : 0;
  a.Lck = ckpt ? (n_layers + (1 << ck_shift) - 1) >> ck_shift : n_layers;
  a.lay = tl;
  a.b = float(kCLight * double(bz_tesla));
  for (int l = 0; l < KF_MAX_LAYERS; ++l) a.layer[l] = l < n_layers ? layers[l] : 0.0f;
  const hipError_t e = kf::launch_adjoint(geometry, block, a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? KF_OK : KF_E_LAUNCH;
}

kf_status_t kf_chi2_backward_z(const float* par_in, const float* cov_in, const float* hit_pos,
                               const float* hit_cov, const float* layer_z, int32_t n_layers, int64_t n_tracks,
                               float bz_tesla, kf_layout_t layout, const int32_t* status_fwd, const float* ckpt,
                               int32_t ckpt_every, const float* grad_chi2, float* grad_hit_pos,
                               float* grad_par_in, float* grad_cov_in, const kf_tune_t* tune, void* stream) {
  return kf_chi2_backward(0, par_in, cov_in, hit_pos, hit_cov, layer_z, n_layers, n_tracks, bz_tesla, layout,
                          status_fwd, ckpt, ckpt_every, grad_chi2, grad_hit_pos, grad_par_in, grad_cov_in, tune,
                          stream);
}

kf_status_t kf_smooth(int32_t geometry, const float* ckpt, const float* par_out, const float* cov_out,
                      const int32_t* status, const float* layers, int32_t n_layers, int64_t n_tracks, float bz_tesla,
                      kf_layout_t layout, float* smoothed, const kf_tune_t* tune, void* stream) {
  if (geometry != 0 && geometry != 1) return KF_E_SHAPE;
  if (n_tracks < 0 || n_layers < 0 || n_layers > KF_MAX_LAYERS) return KF_E_SHAPE;
  kf::TrackLayout tl;
  if (!layout_ok(layout, &tl)) return KF_E_LAYOUT;
  int block = 256;
  if (tune) {
    block = tune->block_threads;
    if (block != 64 && block != 128 && block != 256) return KF_E_FLAGS;
  }
  if (n_tracks == 0 || n_layers == 0) return KF_OK;
  if (!ckpt || !par_out || !cov_out || !status || !layers || !smoothed) return KF_E_NULL;
  const void* ptrs[] = {ckpt, par_out, cov_out, status, smoothed};
  for (const void* p : ptrs)
    if (!aligned4(p)) return KF_E_ALIGN;
  kf_status_t ds = device_ok();
  if (ds != KF_OK) return ds;
  kf::SmoothArgs a;
  a.ckpt = ckpt;
  a.par = par_out;
  a.cov = cov_out;
  a.status = status;
  a.smoothed = smoothed;
  a.n = n_tracks;
  a.L = n_layers;
  a.lay = tl;
  a.b = float(kCLight * double(bz_tesla));
  for (int l = 0; l < KF_MAX_LAYERS; ++l) a.layer[l] = l < n_layers ? layers[l] : 0.0f;
  const hipError_t e = kf::launch_smooth(geometry, block, a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? KF_OK : KF_E_LAUNCH;
}

kf_status_t kf_propagate_gate_update(int32_t geometry, const float* par_in, const float* cov_in, float* par_out,
                                     float* cov_out, const float* cand_pos, const float* cand_cov, int32_t n_cand,
                                     float chi2_gate, const float* layers, int32_t n_layers,
                                     const int32_t* n_layers_per_track, int64_t n_tracks, float bz_tesla,
                                     kf_layout_t layout, uint32_t flags, float* chi2_out, int32_t* status_out,
                                     int32_t* chosen_out, const kf_tune_t* tune, void* stream) {
  if (geometry != 0 && geometry != 1) return KF_E_SHAPE;
  if (n_tracks < 0 || n_layers < 0 || n_layers > KF_MAX_LAYERS) return KF_E_SHAPE;
  if (n_cand < 1 || n_cand > KF_MAX_CANDIDATES || chi2_gate != chi2_gate) return KF_E_SHAPE;
  kf::TrackLayout tl;
  if (!layout_ok(layout, &tl)) return KF_E_LAYOUT;
  if (flags & ~uint32_t(KF_F_PRECISION)) return KF_E_FLAGS;
  const int prec = (flags & KF_F_JOSEPH) ? 2 : ((flags & KF_F_FP64_INVERSE) ? 1 : 0);
  int block = 256;
  if (tune) {
    block = tune->block_threads;
    if (block != 64 && block != 128 && block != 256) return KF_E_FLAGS;
  }
  if (n_tracks == 0) return KF_OK;
  if (!par_in || !cov_in || !par_out || !cov_out) return KF_E_NULL;
  if (n_layers > 0 && (!cand_pos || !cand_cov || !layers)) return KF_E_NULL;
  const void* ptrs[] = {par_in, cov_in, par_out, cov_out, cand_pos, cand_cov, n_layers_per_track, chi2_out,
                        status_out, chosen_out};
  for (const void* p : ptrs)
    if (p && !aligned4(p)) return KF_E_ALIGN;
  kf_status_t ds = device_ok();
  if (ds != KF_OK) return ds;
  kf::GateArgs a;
  a.par_in = par_in;
  a.cov_in = cov_in;
  a.par_out = par_out;
  a.cov_out = cov_out;
  a.cand_pos = cand_pos;
  a.cand_cov = cand_cov;
  a.nlay = n_layers_per_track;
  a.chi2 = chi2_out;
  a.status = status_out;
  a.chosen = chosen_out;
  a.n = n_tracks;
  a.L = n_layers;
  a.M = n_cand;
  a.lay = tl;
  a.b = float(kCLight * double(bz_tesla));
  a.gate = chi2_gate;
  for (int l = 0; l < KF_MAX_LAYERS; ++l) a.layer[l] = l < n_layers ? layers[l] : 0.0f;
  const hipError_t e = kf::launch_gate(geometry, prec, block, a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? KF_OK : KF_E_LAUNCH;
}

int64_t kf_checkpoint_floats(int64_t n_tracks, int32_t n_layers, int32_t ckpt_every, kf_layout_t layout) {
  kf::TrackLayout tl;
  const int sh = ckpt_shift(ckpt_every);
  if (n_tracks < 0 || n_layers <= 0 || sh < 0 || !layout_ok(layout, &tl)) return 0;
  return kf::layout_floats(n_tracks, 27, (n_layers + (1 << sh) - 1) >> sh, tl);
}

kf_status_t kf_propagate_update_z_f64(const double* par_in, const double* cov_in, double* par_out, double* cov_out,
                                      const double* hit_pos, const double* hit_cov, const double* layer_z,
                                      int32_t n_layers, const int32_t* n_layers_per_track, int64_t n_tracks,
                                      double bz_tesla, kf_layout_t layout, uint32_t flags, double* chi2_out,
                                      int32_t* status_out, const kf_tune_t* tune, void* stream) {
  return step_f64(0, par_in, cov_in, par_out, cov_out, hit_pos, hit_cov, layer_z, n_layers, n_layers_per_track,
                  n_tracks, bz_tesla, layout, flags, chi2_out, status_out, tune, stream);
}

kf_status_t kf_propagate_update_r_f64(const double* par_in, const double* cov_in, double* par_out, double* cov_out,
                                      const double* hit_pos, const double* hit_cov, const double* layer_r,
                                      int32_t n_layers, const int32_t* n_layers_per_track, int64_t n_tracks,
                                      double bz_tesla, kf_layout_t layout, uint32_t flags, double* chi2_out,
                                      int32_t* status_out, const kf_tune_t* tune, void* stream) {
  return step_f64(1, par_in, cov_in, par_out, cov_out, hit_pos, hit_cov, layer_r, n_layers, n_layers_per_track,
                  n_tracks, bz_tesla, layout, flags, chi2_out, status_out, tune, stream);
}

kf_status_t kf_propagate_update_host(int32_t geometry, const float* par_in, const float* cov_in, float* par_out,
                                     float* cov_out, const float* hit_pos, const float* hit_cov, const float* layers,
                                     int32_t n_layers, const int32_t* n_layers_per_track, int64_t n_tracks,
                                     float bz_tesla, kf_layout_t layout, uint32_t flags, float* chi2_out,
                                     int32_t* status_out, int64_t chunk_tracks, int32_t n_streams,
                                     const kf_tune_t* tune) {
  if (geometry != 0 && geometry != 1) return KF_E_SHAPE;
  if (n_tracks < 0 || n_layers < 0 || n_layers > KF_MAX_LAYERS || chunk_tracks < 0 || n_streams < 0 ||
      n_streams > 8)
    return KF_E_SHAPE;
  kf::TrackLayout tl;
  if (!layout_ok(layout, &tl)) return KF_E_LAYOUT;
  if (flags & ~uint32_t(KF_F_PRECISION)) return KF_E_FLAGS;
  int block = 256, tpt = 1;
  if (tune) {
    block = tune->block_threads;
    tpt = tune->tracks_per_thread;
    if ((block != 64 && block != 128 && block != 256) || (tpt != 1 && tpt != 2)) return KF_E_FLAGS;
  }
  if (n_tracks == 0) return KF_OK;
  if (!par_in || !cov_in || !par_out || !cov_out) return KF_E_NULL;
  if (n_layers > 0 && (!hit_pos || !hit_cov || !layers)) return KF_E_NULL;
  const void* ptrs[] = {par_in, cov_in, par_out, cov_out, hit_pos, hit_cov, chi2_out, status_out, n_layers_per_track};
  for (const void* p : ptrs)
    if (p && !aligned4(p)) return KF_E_ALIGN;
  kf_status_t ds = device_ok();
  if (ds != KF_OK) return ds;
  kf::StepArgs a;
  memset(&a, 0, sizeof(a));
  a.L = n_layers;
  a.lay = tl;
  a.ck_shift = 0;
  a.Lck = n_layers;
  a.b = float(kCLight * double(bz_tesla));
  for (int l = 0; l < KF_MAX_LAYERS; ++l) a.layer[l] = l < n_layers ? layers[l] : 0.0f;
  kf::HostCall h;
  h.par_in = par_in;
  h.cov_in = cov_in;
  h.par_out = par_out;
  h.cov_out = cov_out;
  h.hit_pos = hit_pos;
  h.hit_cov = hit_cov;
  h.nlay = n_layers_per_track;
  h.chi2 = chi2_out;
  h.status = status_out;
  h.n = n_tracks;
  h.chunk = chunk_tracks > 0 ? chunk_tracks : (int64_t(1) << 17);
  h.n_streams = n_streams > 0 ? n_streams : 3;
  const int prec = (flags & KF_F_JOSEPH) ? 2 : ((flags & KF_F_FP64_INVERSE) ? 1 : 0);
  const hipError_t e = kf::run_host_pipeline(h, a, geometry, prec, block, tpt);
  return e == hipSuccess ? KF_OK : KF_E_LAUNCH;
}

void kf_host_release(void) { kf::release_host_pipeline(); }

int64_t kf_batched_workspace_size(int64_t n_tracks) {
  return n_tracks < 0 ? 0 : kf::batched_workspace_bytes(n_tracks);
}

}  // extern "C"

namespace {

// Everything kf_propagate_update_batched checks and sets up except the
// workspace: the argument checks in the order the header states, the launch
// shape, and the kernel arguments (the bytes of `a` key the graph cache, so
// it is cleared first).  Returns KF_OK with *a, *prec, *block filled, or the
// error; *empty is set when there is nothing to enqueue.
kf_status_t batched_prepare(const float* par_in, const float* cov_in, float* par_out, float* cov_out,
                            const float* hit_pos, const float* hit_cov, const int64_t* hit_offset, int64_t n_hits,
                            const uint8_t* geom, const int32_t* n_layers_per_track, const float* layer_z,
                            const float* layer_r, int32_t max_layers, int64_t n_tracks, float bz_tesla,
                            kf_layout_t layout, uint32_t flags, float* chi2_out, int32_t* status_out,
                            const kf_tune_t* tune, kf::BatchedArgs* a, int* prec, int* block_out, bool* empty) {
  *empty = false;
  if (n_tracks < 0 || n_tracks > KF_BATCHED_MAX_TRACKS || max_layers < 0 || max_layers > KF_MAX_LAYERS ||
      n_hits < 0)
    return KF_E_SHAPE;
  kf::TrackLayout tl;
  if (!layout_ok(layout, &tl)) return KF_E_LAYOUT;
  if (flags & ~uint32_t(KF_F_PRECISION | KF_F_NO_GRAPH)) return KF_E_FLAGS;
  // default shape: the one measured fastest on a mixed uneven batch (static
  // round-robin over a grid of twice the resident 128-thread blocks)
  int block = 128, tpt = 1, sched = KF_SCHED_STATIC, mult = 2;
  if (tune) {
    block = tune->block_threads;
    tpt = tune->tracks_per_thread;
    sched = tune->schedule;
    mult = tune->waves_mult;
    if ((block != 64 && block != 128 && block != 256) || (tpt != 1 && tpt != 2) ||
        (sched != KF_SCHED_DYNAMIC && sched != KF_SCHED_STATIC) || mult < 0 || mult > 8)
      return KF_E_FLAGS;
    if (mult == 0) mult = 1;
  }
  if (n_tracks == 0) {
    *empty = true;
    return KF_OK;
  }
  if (!par_in || !cov_in || !par_out || !cov_out || !geom || !n_layers_per_track || !hit_offset) return KF_E_NULL;
  if (max_layers > 0 && (!hit_pos || !hit_cov || !layer_z || !layer_r)) return KF_E_NULL;
  const void* ptrs[] = {par_in, cov_in, par_out, cov_out, hit_pos, hit_cov, chi2_out, status_out, n_layers_per_track};
  for (const void* p : ptrs)
    if (p && !aligned4(p)) return KF_E_ALIGN;
  if (reinterpret_cast<uintptr_t>(hit_offset) & 7u) return KF_E_ALIGN;
  memset(a, 0, sizeof(*a));
  a->par_in = par_in;
  a->cov_in = cov_in;
  a->par_out = par_out;
  a->cov_out = cov_out;
  a->hit_pos = hit_pos;
  a->hit_cov = hit_cov;
  a->hit_offset = hit_offset;
  a->n_hits = n_hits;
  a->geom = geom;
  a->nlay = n_layers_per_track;
  a->chi2 = chi2_out;
  a->status = status_out;
  a->n = n_tracks;
  a->L = max_layers;
  a->tpt = tpt;
  a->schedule = sched;
  a->waves_mult = mult;
  a->lay = tl;
  a->b = float(kCLight * double(bz_tesla));
  kf::bucket_order(a->order);
  for (int l = 0; l < max_layers; ++l) {
    a->layer_z[l] = layer_z[l];
    a->layer_r[l] = layer_r[l];
  }
  *prec = (flags & KF_F_JOSEPH) ? 2 : ((flags & KF_F_FP64_INVERSE) ? 1 : 0);
  *block_out = block;
  return KF_OK;
}

}  // namespace

extern "C" {

kf_status_t kf_propagate_update_batched(
    const float* par_in, const float* cov_in, float* par_out, float* cov_out, const float* hit_pos,
    const float* hit_cov, const int64_t* hit_offset, int64_t n_hits, const uint8_t* geom,
    const int32_t* n_layers_per_track,
    const float* layer_z, const float* layer_r, int32_t max_layers, int64_t n_tracks, float bz_tesla,
    kf_layout_t layout, uint32_t flags, float* chi2_out, int32_t* status_out, void* workspace,
    int64_t workspace_bytes, const kf_tune_t* tune, void* stream) {
  kf::BatchedArgs a;
  int prec = 0, block = 0;
  bool empty = false;
  const kf_status_t ps = batched_prepare(par_in, cov_in, par_out, cov_out, hit_pos, hit_cov, hit_offset, n_hits, geom,
                                         n_layers_per_track, layer_z, layer_r, max_layers, n_tracks, bz_tesla, layout,
                                         flags, chi2_out, status_out, tune, &a, &prec, &block, &empty);
  if (ps != KF_OK || empty) return ps;
  if (reinterpret_cast<uintptr_t>(workspace) & 7u) return KF_E_ALIGN;
  if (!kf::batched_carve(workspace, workspace_bytes, n_tracks, &a.ws)) return KF_E_WORKSPACE;
  kf_status_t ds = device_ok();
  if (ds != KF_OK) return ds;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (flags & KF_F_NO_GRAPH) {
    const hipError_t e = kf::launch_batched(a, prec, block, st);
    return e == hipSuccess ? KF_OK : KF_E_LAUNCH;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return KF_E_DEVICE;
  return batched_via_graph(a, prec, block, dev, st);
}

kf_status_t kf_propagate_update_batched_noalloc(
    const float* par_in, const float* cov_in, float* par_out, float* cov_out, const float* hit_pos,
    const float* hit_cov, const int64_t* hit_offset, int64_t n_hits, const uint8_t* geom,
    const int32_t* n_layers_per_track, const float* layer_z, const float* layer_r, int32_t max_layers,
    int64_t n_tracks, float bz_tesla, kf_layout_t layout, uint32_t flags, float* chi2_out, int32_t* status_out,
    const kf_tune_t* tune, void* stream) {
  kf::BatchedArgs a;
  int prec = 0, block = 0;
  bool empty = false;
  const kf_status_t ps = batched_prepare(par_in, cov_in, par_out, cov_out, hit_pos, hit_cov, hit_offset, n_hits, geom,
                                         n_layers_per_track, layer_z, layer_r, max_layers, n_tracks, bz_tesla, layout,
                                         flags, chi2_out, status_out, tune, &a, &prec, &block, &empty);
  if (ps != KF_OK || empty) return ps;
  if (n_tracks > KF_NOALLOC_MAX_TRACKS) return KF_E_WORKSPACE;
  kf_status_t ds = device_ok();
  if (ds != KF_OK) return ds;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return KF_E_DEVICE;
  void* scratch = nullptr;
  int64_t scratch_bytes = 0;
  if (kf::noalloc_scratch(dev, &scratch, &scratch_bytes) != hipSuccess) return KF_E_DEVICE;
  if (!kf::batched_carve(scratch, scratch_bytes, n_tracks, &a.ws)) return KF_E_WORKSPACE;
  // enqueued directly: no graph is built (that would allocate); a caller
  // capturing this stream gets the four kernels as nodes of its own graph
  const hipError_t e = kf::launch_batched(a, prec, block, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? KF_OK : KF_E_LAUNCH;
}

void kf_batched_release(void) {
  GraphCache& gc = graphs();
  std::lock_guard<std::mutex> g(gc.mu);
  for (auto& e : gc.lru) hipGraphExecDestroy(e.second);
  gc.lru.clear();
  gc.index.clear();
}

kf_status_t kf_propagate_update_z(const float* par_in, const float* cov_in, float* par_out, float* cov_out,
                                  const float* hit_pos, const float* hit_cov, const float* layer_z,
                                  int32_t n_layers, const int32_t* n_layers_per_track, int64_t n_tracks,
                                  float bz_tesla, kf_layout_t layout, uint32_t flags, float* chi2_out,
                                  int32_t* status_out, float* ckpt_out, int32_t ckpt_every, const kf_tune_t* tune,
                                  void* stream) {
  return step(0, par_in, cov_in, par_out, cov_out, hit_pos, hit_cov, layer_z, n_layers, n_layers_per_track,
              n_tracks, bz_tesla, layout, flags, chi2_out, status_out, ckpt_out, ckpt_every, tune, stream);
}

kf_status_t kf_propagate_update_r(const float* par_in, const float* cov_in, float* par_out, float* cov_out,
                                  const float* hit_pos, const float* hit_cov, const float* layer_r,
                                  int32_t n_layers, const int32_t* n_layers_per_track, int64_t n_tracks,
                                  float bz_tesla, kf_layout_t layout, uint32_t flags, float* chi2_out,
                                  int32_t* status_out, float* ckpt_out, int32_t ckpt_every, const kf_tune_t* tune,
                                  void* stream) {
  return step(1, par_in, cov_in, par_out, cov_out, hit_pos, hit_cov, layer_r, n_layers, n_layers_per_track,
              n_tracks, bz_tesla, layout, flags, chi2_out, status_out, ckpt_out, ckpt_every, tune, stream);
}

kf_status_t kf_pack(const float* src_soa, float* dst, int32_t n_elem, int32_t n_layers_or_1, int64_t n_tracks,
                    kf_layout_t layout, void* stream) {
  return pack_common(src_soa, dst, n_elem, n_layers_or_1, n_tracks, layout, stream, true);
}

kf_status_t kf_unpack(const float* src, float* dst_soa, int32_t n_elem, int32_t n_layers_or_1, int64_t n_tracks,
                      kf_layout_t layout, void* stream) {
  return pack_common(src, dst_soa, n_elem, n_layers_or_1, n_tracks, layout, stream, false);
}

int64_t kf_array_floats(int32_t n_elem, int32_t n_layers_or_1, int64_t n_tracks, kf_layout_t layout) {
  kf::TrackLayout tl;
  if (n_elem <= 0 || n_layers_or_1 <= 0 || n_tracks < 0 || !layout_ok(layout, &tl)) return 0;
  return kf::layout_floats(n_tracks, n_elem, n_layers_or_1, tl);
}

const char* kf_status_string(kf_status_t s) {
  switch (s) {
    case KF_OK: return "ok";
    case KF_E_NULL: return "a required pointer is NULL";
    case KF_E_SHAPE: return "invalid sizes";
    case KF_E_LAYOUT: return "unknown layout or block width";
    case KF_E_ALIGN: return "pointer not 4-byte aligned";
    case KF_E_DEVICE: return "no gfx950 device current";
    case KF_E_LAUNCH: return "kernel launch failed";
    case KF_E_WORKSPACE: return "workspace missing or too small";
    case KF_E_FLAGS: return "unknown flags or tuning values";
    case KF_E_UNSUPPORTED: return "not supported by the library";
  }
  return "unknown status";
}

int kf_abi_version(void) { return KF_ABI_VERSION; }

}  // extern "C"

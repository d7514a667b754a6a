// C ABI of libkf.so (declared in include/kf.h): argument validation and
// dispatch to the kernel launchers.  Nothing here allocates device memory.
#include <string.h>

#include <mutex>

#include "kf_internal.h"

namespace {

constexpr double kCLight = 0.00299792458;

bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

bool layout_ok(kf_layout_t lay, kf::TrackLayout* out) {
  if (lay.kind == KF_SOA) {
    *out = {0, 0};
    return true;
  }
  if (lay.kind != KF_AOSOA) return false;
  for (int sh = 4; sh <= 8; ++sh)
    if (lay.block == (1 << sh)) {
      *out = {1, sh};
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

kf_status_t step(int geom, const float* par_in, const float* cov_in, float* par_out, float* cov_out,
                 const float* hit_pos, const float* hit_cov, const float* layers, int32_t n_layers,
                 const int32_t* nlay, int64_t n_tracks, float bz, kf_layout_t layout, uint32_t flags,
                 float* chi2_out, int32_t* status_out, float* ckpt_out, const kf_tune_t* tune,
                 void* stream) {
  if (n_tracks < 0 || n_layers < 0 || n_layers > KF_MAX_LAYERS) return KF_E_SHAPE;
  kf::TrackLayout tl;
  if (!layout_ok(layout, &tl)) return KF_E_LAYOUT;
  if (flags & ~uint32_t(KF_F_PRECISION)) return KF_E_FLAGS;
  int block = 256, tpt = 1;
  if (tune) {
    block = tune->block_threads;
    tpt = tune->tracks_per_thread;
    if ((block != 64 && block != 128 && block != 256) || (tpt != 1 && tpt != 2)) return KF_E_FLAGS;
  }
  if (geom == 1 && ckpt_out) return KF_E_UNSUPPORTED;
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
  a.lay = tl;
  a.b = float(kCLight * double(bz));
  for (int l = 0; l < KF_MAX_LAYERS; ++l) a.layer[l] = l < n_layers ? layers[l] : 0.0f;
  const int prec = (flags & KF_F_JOSEPH) ? 2 : ((flags & KF_F_FP64_INVERSE) ? 1 : 0);
  hipError_t e = kf::launch_step(geom, prec, block, tpt, a, static_cast<hipStream_t>(stream));
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

}  // namespace

extern "C" {

kf_status_t kf_propagate_update_z(const float* par_in, const float* cov_in, float* par_out, float* cov_out,
                                  const float* hit_pos, const float* hit_cov, const float* layer_z,
                                  int32_t n_layers, const int32_t* n_layers_per_track, int64_t n_tracks,
                                  float bz_tesla, kf_layout_t layout, uint32_t flags, float* chi2_out,
                                  int32_t* status_out, float* ckpt_out, const kf_tune_t* tune, void* stream) {
  return step(0, par_in, cov_in, par_out, cov_out, hit_pos, hit_cov, layer_z, n_layers, n_layers_per_track,
              n_tracks, bz_tesla, layout, flags, chi2_out, status_out, ckpt_out, tune, stream);
}

kf_status_t kf_propagate_update_r(const float* par_in, const float* cov_in, float* par_out, float* cov_out,
                                  const float* hit_pos, const float* hit_cov, const float* layer_r,
                                  int32_t n_layers, const int32_t* n_layers_per_track, int64_t n_tracks,
                                  float bz_tesla, kf_layout_t layout, uint32_t flags, float* chi2_out,
                                  int32_t* status_out, float* ckpt_out, const kf_tune_t* tune, void* stream) {
  return step(1, par_in, cov_in, par_out, cov_out, hit_pos, hit_cov, layer_r, n_layers, n_layers_per_track,
              n_tracks, bz_tesla, layout, flags, chi2_out, status_out, ckpt_out, tune, stream);
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
  if (!tl.aos) return int64_t(n_elem) * n_layers_or_1 * n_tracks;
  const int64_t B = int64_t(1) << tl.shift;
  return ((n_tracks + B - 1) / B) * B * n_elem * n_layers_or_1;
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
    case KF_E_UNSUPPORTED: return "not supported by this build";
  }
  return "unknown status";
}

int kf_abi_version(void) { return KF_ABI_VERSION; }

}  // extern "C"

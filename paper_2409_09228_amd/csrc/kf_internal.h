// Internal host-side interface between the C ABI (kf_api.hip) and the kernel
// launchers.  Not installed; the public interface is include/kf.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kf.h"

namespace kf {

// Physical layout of a launch's track arrays (see kf_lanes.h).
struct TrackLayout {
  int32_t kind;  // KF_SOA, KF_AOSOA or KF_AOS
  int32_t shift; // log2(B) for AoSoA
};

// One plain step call; T is the scalar of every array, of the field constant
// and of the layer table (float, or double in the FP64 form).
template <class T>
struct StepArgsT {
  using Scalar = T;
  const T* par_in;
  const T* cov_in;
  T* par_out;
  T* cov_out;
  const T* hit_pos;
  const T* hit_cov;
  const int32_t* nlay;
  T* chi2;
  int32_t* status;
  T* ckpt;
  int64_t n;
  int32_t L;
  int32_t ck_shift;  // log2 of the checkpoint stride
  int32_t Lck;       // checkpoint slots per track: ceil(L / stride)
  TrackLayout lay;
  T b;  // 0.00299792458 * Bz
  T layer[KF_MAX_LAYERS];
};
using StepArgs = StepArgsT<float>;

struct AdjointArgs {
  const float* par_in;
  const float* cov_in;
  const float* hit_pos;
  const float* hit_cov;
  const float* ckpt;       // entering states of every stride-th layer, or NULL: recompute
  const int32_t* status;   // the forward's status words
  const float* grad_chi2;  // dL/dchi2_i
  float* grad_hit;         // dL/dm, per layer
  float* grad_par;         // dL/dp0
  float* grad_cov;         // dL/dC0 or NULL
  int64_t n;
  int32_t L;
  int32_t ck_shift;        // log2 of the checkpoint stride
  int32_t Lck;             // checkpoint slots per track
  TrackLayout lay;
  float b;
  float layer[KF_MAX_LAYERS];
};

hipError_t launch_adjoint(int geom, int block, const AdjointArgs& a, hipStream_t s);

// Smoother over the layers the filter applied (kf_smooth.hip).
struct SmoothArgs {
  const float* ckpt;      // the filter's per-layer checkpoints (stride 1): slot k = state entering layer k
  const float* par;       // the filter's output: the state after its last layer
  const float* cov;
  const int32_t* status;  // the filter's status words (layers applied in bits 16..31)
  float* smoothed;        // slot k = smoothed state on layer k (may be ckpt itself)
  int64_t n;
  int32_t L;
  TrackLayout lay;
  float b;
  float layer[KF_MAX_LAYERS];
};

hipError_t launch_smooth(int geom, int block, const SmoothArgs& a, hipStream_t s);

// Filter with hit selection among n_cand candidates per layer (kf_gate.hip).
struct GateArgs {
  const float* par_in;
  const float* cov_in;
  float* par_out;
  float* cov_out;
  const float* cand_pos;  // per layer 3 * M floats per track, in `lay`
  const float* cand_cov;  // per layer 6 * M floats per track, in `lay`
  const int32_t* nlay;
  float* chi2;
  int32_t* status;
  int32_t* chosen;        // [L][n] or NULL
  int64_t n;
  int32_t L;
  int32_t M;
  TrackLayout lay;
  float b;
  float gate;
  float layer[KF_MAX_LAYERS];
};

hipError_t launch_gate(int geom, int prec, int block, const GateArgs& a, hipStream_t s);

// precision variant: 0 FP32, 1 FP64 gain + plain covariance, 2 FP64 gain + Joseph
hipError_t launch_step(int geom, int prec, int block, int tpt, const StepArgs& a, hipStream_t s);
// The FP64 form: FP64 arrays, FP64 arithmetic throughout (prec 0 plain update,
// 2 Joseph update)
hipError_t launch_step_f64(int geom, int prec, int block, const StepArgsT<double>& a, hipStream_t s);

hipError_t launch_pack(const float* src, float* dst, int32_t E, int32_t L, int64_t n, TrackLayout lay,
                       bool to_layout, hipStream_t s);

}  // namespace kf

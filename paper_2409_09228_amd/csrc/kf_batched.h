// Internal interface of the mixed-geometry, uneven-length batched form.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kf_internal.h"

#define KF_NBUCKETS (2 * (KF_MAX_LAYERS + 1))

namespace kf {

// Views into the caller's workspace.
struct BatchedWorkspace {
  int32_t* bucket_count;   // [KF_NBUCKETS] tracks per bucket
  int32_t* bucket_cursor;  // [KF_NBUCKETS] scatter cursors
  int32_t* bucket_base;    // [KF_NBUCKETS] first slot of each bucket
  int32_t* counter;        // [4]: next item, number of items, count blocks done
  int32_t* item_base;      // [KF_NBUCKETS + 1] first item of each bucket order position
  int32_t* perm;           // [max slots] track index per slot
};

struct BatchedArgs {
  const float* par_in;
  const float* cov_in;
  float* par_out;
  float* cov_out;
  const float* hit_pos;
  const float* hit_cov;
  const int64_t* hit_offset;
  int64_t n_hits;
  const uint8_t* geom;
  const int32_t* nlay;
  float* chi2;
  int32_t* status;
  BatchedWorkspace ws;
  int64_t n;
  int32_t L;    // layer tables' length (max layers per track)
  int32_t tpt;  // tracks per lane per work item
  int32_t schedule;    // KF_SCHED_DYNAMIC or KF_SCHED_STATIC
  int32_t waves_mult;  // grid = waves_mult x (blocks that fit at once)
  TrackLayout lay;
  float b;
  int32_t order[KF_NBUCKETS];
  float layer_z[KF_MAX_LAYERS];
  float layer_r[KF_MAX_LAYERS];
};

// Workspace bytes for n tracks (any tracks_per_thread in {1, 2}).
int64_t batched_workspace_bytes(int64_t n);
// Carve the workspace; false if it is too small.
bool batched_carve(void* ws, int64_t bytes, int64_t n, BatchedWorkspace* out);
void bucket_order(int32_t order[KF_NBUCKETS]);
// Enqueue the three planning kernels and the persistent run.
hipError_t launch_batched(const BatchedArgs& a, int prec, int block, hipStream_t s);
// Device address and size of the fixed planning workspace of
// kf_propagate_update_batched_noalloc on device `dev` (the current device):
// looked up once per device, then kept.
hipError_t noalloc_scratch(int dev, void** ptr, int64_t* bytes);

}  // namespace kf

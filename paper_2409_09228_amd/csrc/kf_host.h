// Internal interface of the host-resident pipeline (kf_host.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kf_internal.h"

namespace kf {

// Host arrays of one kf_propagate_update_host call (the whole sample).
struct HostCall {
  const float* par_in;
  const float* cov_in;
  float* par_out;
  float* cov_out;
  const float* hit_pos;
  const float* hit_cov;
  const int32_t* nlay;  // or NULL
  float* chi2;          // or NULL
  int32_t* status;      // or NULL
  int64_t n;
  int64_t chunk;        // tracks per chunk (>= 1)
  int n_streams;        // 1 .. 8
};

// Runs the chunks; `base` carries everything of the step but the pointers
// and the track count.  Blocks until every result is in host memory.
hipError_t run_host_pipeline(const HostCall& h, StepArgs base, int geom, int prec, int block, int tpt);
void release_host_pipeline();

}  // namespace kf

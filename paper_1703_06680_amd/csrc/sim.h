// Random-walk step of a resident simulation (sim.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ddm.h"

namespace ddm {

struct WalkArgs {
  float *upd_lo, *upd_hi;
  int64_t n;
  float *sub_lo, *sub_hi;
  int64_t m;
  int d;
  float side, sigma;
  uint64_t seed;
  uint32_t step;  // the step being taken (1 for the first)
};

// Enqueues one step: region r (updates 0 .. n-1, then subscriptions
// n .. n+m-1) moves on axis k by sigma * z(r, k, step) and hi = lo + side.
hipError_t launch_walk(const WalkArgs &w, hipStream_t s);

}  // namespace ddm

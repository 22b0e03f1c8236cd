// Device-side pieces of the bucketed path shared by its kernels
// (bucket_path.hip) and by the resident-simulation kernels (resident.hip):
// the bucket map, the boxes, the other-axis quantisation and the offsets
// through which the sweep finds each bucket's records.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace ddm {

struct BucketParams {
  float vmin;        // bucket map of the swept axis' lower coordinate
  float scale;
  uint32_t nb;
  uint32_t valid;
  float qmin[2];     // 16-bit quantisation of the other axes (pre-filter)
  float qscale[2];
};

// bucket(x) = clamp(floor((x - vmin) * scale), 0, nb - 1): monotone
// non-decreasing in x, so a region whose lower coordinate falls in a later
// bucket starts strictly after every region of an earlier one.
__device__ __forceinline__ uint32_t bucket_of(float x, float vmin, float scale, uint32_t nb) {
  float t = (x - vmin) * scale;
  t = fminf(fmaxf(t, 0.0f), (float)(nb - 1));
  return (uint32_t)t;
}

template <int D>
struct Box {
  float lo[D];
  float hi[D];
};

// Error bits and emptiness of one box.  A half-open box with lo == hi on
// some axis is empty; a closed one never is (lo == hi is a point).
template <int D>
__device__ __forceinline__ uint32_t box_errors(const Box<D> &b, bool &empty, uint32_t closed) {
  uint32_t err = 0;
  empty = false;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float l = b.lo[k], h = b.hi[k];
    if (l != l || h != h) err |= kErrNaN;
    if (l > h) err |= kErrOrder;
    if (l == h && !closed) empty = true;
  }
  return err;
}

// Conservative quantisation of a coordinate of another axis onto 16 bits by
// the monotone map t = clamp((x - qmin) * qscale, 0, 65535): lower bounds
// round down, upper bounds round up, so two boxes that overlap on that axis
// also overlap after quantisation.  Quantised bounds only serve the
// sweep's pre-filter; survivors are tested on the exact coordinates.
__device__ __forceinline__ uint32_t quant_lo(float x, float qmin, float qs) {
  float t = (x - qmin) * qs;
  t = fminf(fmaxf(t, 0.0f), 65535.0f);
  return (uint32_t)t;
}

__device__ __forceinline__ uint32_t quant_hi(float x, float qmin, float qs) {
  float t = (x - qmin) * qs;
  t = fminf(fmaxf(t, 0.0f), 65535.0f);
  return (uint32_t)ceilf(t);
}

// Word 3 of a region record: the quantised bounds of the other axes.  d = 2:
// the 16-bit lower | upper << 16 of axis 1; d >= 3: 7-bit bounds of axes 1
// and 2 (the 16-bit ones scaled by 2^-9, lower rounded down, upper rounded
// up and capped at 127) lo1 | hi1 << 8 | lo2 << 16 | hi2 << 24; 0 for d = 1.
template <int D>
__device__ __forceinline__ uint32_t qword_of(const Box<D> &b, const BucketParams &p) {
  if (D == 2) {
    return quant_lo(b.lo[1 % D], p.qmin[0], p.qscale[0]) |
           (quant_hi(b.hi[1 % D], p.qmin[0], p.qscale[0]) << 16);
  }
  if (D >= 3) {
    uint32_t w = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const uint32_t l7 = quant_lo(b.lo[(1 + c) % D], p.qmin[c], p.qscale[c]) >> 9;
      const uint32_t h7 = min(127u, (quant_hi(b.hi[(1 + c) % D], p.qmin[c], p.qscale[c]) + 511u) >> 9);
      w |= (l7 | (h7 << 8)) << (16 * c);
    }
    return w;
  }
  return 0u;
}

// Where the sweep finds bucket j's records and boundary-state entries.
//
// Packed layout (a matching call): the one prefix sum over [bucket sizes |
// boundary-state sizes | 0] (2 nb + 1 entries, buckets numbered over all
// instances) gives S[j], the first record slot of bucket j, S[nb], the
// number of records, and S[nb + j] - S[nb], the first boundary-state entry
// of bucket j (j <= nb).  Block k's first slot in bucket j is S[j] plus the
// block-major prefix written by bk_colscan_kernel.
//
// Slab layout (a resident simulation, cnt non-null): bucket j owns the
// fixed slots [j * cap, (j + 1) * cap) of which the first cnt[j] hold
// records, and [j * bs_slab, (j + 1) * bs_slab) of the boundary-state
// records, of which the first bs_cnt[j] are filled (a count above bs_slab
// means some did not fit).
struct Offsets {
  const uint32_t *S;
  uint32_t nb;  // buckets over all instances
  const uint32_t *cnt = nullptr, *bs_cnt = nullptr;
  uint32_t cap = 0, bs_slab = 0;
  __device__ uint32_t bs_begin(uint32_t j) const { return S[nb + j] - S[nb]; }
};

}  // namespace ddm

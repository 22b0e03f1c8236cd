// Bucketed sort-based matching: the sweep runs per bucket entirely in LDS.
//
// Regions are distributed into buckets by a monotone non-decreasing function
// of the swept axis' lower coordinate, so the buckets, taken in order, are
// consecutive segments of the sorted endpoint list (the segments T_p of the
// paper's Algorithm 5).  Each bucket is sorted and swept by one workgroup in
// LDS; the regions of earlier buckets that are still active when a bucket
// starts (SubSet[p] and UpdSet[p] of Algorithms 5 and 6) are delivered to it
// as a boundary-state list built by a span count, a prefix sum and a fill.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace ddm {

struct BucketLayout {
  uint32_t nb;          // number of buckets
  uint32_t nblk;        // blocks of the count and scatter passes
  uint32_t gpb;         // groups of four rows per count/scatter block
  uint32_t bs_cap;      // capacity of the boundary-state record buffer
  int rec_words;        // 32-bit words per region record
  size_t bytes;         // workspace bytes for all buffers below
  // byte offsets inside the bucket workspace
  size_t params, sample_part, counts, transposed, offsets, block_offsets, scan_tmp, bs_cur, rec,
      bs_rec;
};

// Largest number of buckets the count/scatter passes handle (LDS-resident
// per-bucket counters).
constexpr uint32_t kMaxBuckets = 16384;

bool bucket_path_supported(int d, int64_t n, int64_t m);
BucketLayout bucket_layout(int64_t n, int64_t m, int d);

struct BucketArgs {
  const float *ulo, *uhi, *slo, *shi;
  uint32_t n, m;
  int d;
  void *ws;  // base of the bucket workspace (BucketLayout offsets apply)
  BucketLayout L;
  Header *hdr;
};

// Enqueue sampling, counting (with input validation), prefix sums and the
// scatter of region records into buckets.
hipError_t bucket_prepare(const BucketArgs &a, hipStream_t s);

// Enqueue the per-bucket sweep.  mode 0: total only; 1: total and per-update
// counts (per_update zeroed beforehand); 2: write pairs at pair_off[u] plus a
// per-update cursor (zeroed beforehand).
hipError_t bucket_sweep(const BucketArgs &a, int mode, int32_t *per_update,
                        const unsigned long long *pair_off, uint32_t *cursor, uint32_t *out_u,
                        uint32_t *out_s, unsigned long long *total, hipStream_t s);

}  // namespace ddm

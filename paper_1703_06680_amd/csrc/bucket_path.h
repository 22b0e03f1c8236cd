// Bucketed sort-based matching: the sweep runs per bucket entirely in LDS.
//
// Regions are distributed into buckets by a monotone non-decreasing function
// of the swept axis' lower coordinate, so the buckets, taken in order, are
// consecutive segments of the sorted endpoint list (the segments T_p of the
// paper's Algorithm 5).  Each bucket is sorted and swept by one workgroup in
// LDS; the regions of earlier buckets that are still active when a bucket
// starts (SubSet[p] and UpdSet[p] of Algorithms 5 and 6) are delivered to it
// as a boundary-state list built by a span count, a prefix sum and a fill.
// For d >= 2 the plan may also cut every such segment (a column) into rows
// by axis 1's lower coordinate: boxes reaching later rows of their column are
// copied there as records, and a pair is counted only in the row of the
// larger of its two axis-1 lower bounds, so that each is counted once.
//
// One launch sequence serves a batch of independent instances stored back to
// back: every instance has its own buckets, count/scatter blocks and sample
// blocks, all numbered globally, and a single call is a batch of one.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "common.h"

namespace ddm {

// d = 1 pair emission by rows (see bucket_sweep): each bucket update's pairs
// found in its bucket are gathered by one wave, ordered in LDS and written
// as a finished row; rows that also get pairs from later buckets are left,
// ordered, in the staging array for a final row sort.
constexpr uint32_t kRowStage = 256;    // longest row the emitting waves can hold
constexpr uint32_t kBsSubCap = 512;    // boundary-state subscriptions per bucket held in LDS
struct RowEmit {
  const int32_t *cnt;  // per-update pair counts (null: emission pair by pair)
  uint32_t *ids;       // CSR output (subscription ids), or null
  int32_t *pairs;      // pair-list output [K][2], or null
  uint32_t *flag;      // set to 1 if some bucket could not emit by rows
};

// Launch-shape parameters of the bucketed path.
struct BucketTuning {
  uint32_t target = 1536;         // mean records per bucket (at most 3/4 of the capacity)
  uint32_t sweep_threads = 512;   // 256, 512 or 1024 threads per sweep workgroup
  uint32_t groups_per_thread = 1; // count/scatter: groups of four rows per thread (minimum)
  uint32_t max_blocks = 256;      // count/scatter blocks per instance at most
};

// Largest d of the bucketed path (the pre-filter quantises axes 1 and 2; the
// exact test reads every other axis).
constexpr int kBucketMaxDims = 8;

// Records per bucket the sweep holds in LDS: kBucketCap for sweep
// workgroups of 256 or 512 threads, kBigBucketCap for 1024.
constexpr uint32_t kBucketCap = 2048;
constexpr uint32_t kBigBucketCap = 4096;
// Largest number of buckets of one instance (LDS-resident per-bucket counters
// of the count and scatter passes).
constexpr uint32_t kMaxBuckets = 16384;

// One instance: its own row arrays (float32 [n][d] / [m][d]); closed != 0
// matches closed intervals [lo, hi] instead of half-open [lo, hi).
struct InstSpec {
  const float *ulo, *uhi, *slo, *shi;
  int64_t n, m;
  uint32_t closed = 0;
};

// Per-instance launch plan, in device memory for batches of more than one.
struct InstPlan {
  const float *ulo, *uhi, *slo, *shi;  // the instance's rows
  uint32_t u0, n, s0, m;     // first output row of its updates / subscriptions, counts
  uint32_t gu, g;            // groups of up to four rows: of updates, of both kinds
  uint32_t blk0, nblk, gpb;  // count/scatter blocks (first, number) and groups per block
  uint32_t b0, nb;           // buckets (first, number)
  uint32_t cell0;            // first cell of the instance's nblk x nb count matrix
  uint32_t smp0, nsmp;       // sample blocks
  uint32_t vec;              // rows may be read with 16-byte loads
  uint32_t closed;           // 1: closed intervals (records hold enc(hi) + 1)
  uint32_t d;                // dimensions (floats per row)
};

inline uint32_t bucket_cap(const BucketTuning &t) {
  return t.sweep_threads == 1024 ? kBigBucketCap : kBucketCap;
}

// Host copy of the per-instance plans, contiguous: a batch of one is held
// inline (a single call touches no heap), larger batches on the heap.
class PlanList {
 public:
  void resize(size_t count) {
    count_ = count;
    many_.assign(count > 1 ? count : 0, InstPlan{});
  }
  size_t size() const { return count_; }
  InstPlan *data() { return count_ > 1 ? many_.data() : &one_; }
  const InstPlan *data() const { return count_ > 1 ? many_.data() : &one_; }
  InstPlan &operator[](size_t i) { return data()[i]; }
  const InstPlan &operator[](size_t i) const { return data()[i]; }

 private:
  InstPlan one_{};
  std::vector<InstPlan> many_;
  size_t count_ = 0;
};

struct BucketLayout {
  uint32_t B;                          // instances
  uint32_t nb, nblk, nsmp;             // totals over the instances
  uint32_t max_nb;                     // most buckets of one instance
  uint32_t nb_split;                   // room for buckets after a split (one instance)
  uint32_t n_total, m_total;           // updates, subscriptions over the instances
  uint32_t bs_cap;                     // capacity of the boundary-state record buffer
  uint32_t rec_cap;                    // capacity of the record buffer (even)
  int rec_words;                       // 32-bit words per region record
  BucketTuning tune;
  size_t cells;                        // count-matrix cells over the instances
  size_t bytes;                        // workspace bytes for all buffers below
  // byte offsets inside the bucket workspace
  size_t params, sample_part, sample_pts, counts, totals, offsets, block_offsets, scan_tmp, bs_cur,
      rec, bs_rec, heavy, split, plan, maps, hits;
  PlanList inst;                       // host copy of the per-instance plan
};

// Instances in order; output rows (per-update counts, pair rows) number the
// updates and the subscriptions of all instances consecutively.  Only the
// sizes are read by bucket_path_supported; the layout records the pointers.
bool bucket_path_supported(int d, const InstSpec *inst, int64_t B, const BucketTuning &t);
BucketLayout bucket_layout(const InstSpec *inst, int64_t B, int d, const BucketTuning &t);
// Single instance of n updates and m subscriptions with the default tuning.
bool bucket_path_supported(int d, int64_t n, int64_t m);
BucketLayout bucket_layout(const float *ulo, const float *uhi, int64_t n, const float *slo,
                           const float *shi, int64_t m, int d, bool closed = false);

struct BucketArgs {
  int d;
  void *ws;  // base of the bucket workspace (BucketLayout offsets apply)
  const BucketLayout *L;
  Header *hdr;
  unsigned long long *inst_total;  // per-instance pair counts [B], or null
  int32_t *zero;                   // cleared by bucket_prepare ([zero_count]), or null
  uint32_t zero_count;
  // d = 1 pair mode: per update, its pairs found in its own bucket ([n],
  // written by the count sweep, read by the emitting sweep), or null
  uint32_t *own = nullptr;
  RowEmit rows{};  // d = 1 emitting sweep by rows (rows.cnt non-null), with own
};

// Copies the per-instance plan to the workspace and expands the block,
// sample, tile and bucket to instance maps (batches of more than one; no-op
// otherwise).  The plan stays valid until the workspace is reused.  If
// ``pinned`` is given (page-locked host memory of plan_bytes(L) bytes), the
// plan is staged there and the copy does not block the host; the caller
// keeps it untouched until the stream has passed the copy.
size_t plan_bytes(const BucketLayout &L);
hipError_t bucket_upload_plan(const BucketArgs &a, hipStream_t s, void *pinned = nullptr);

// Enqueue sampling, counting (with input validation), prefix sums and the
// scatter of region records into buckets.  It clears the header, the
// per-instance totals and a.zero itself (so the outputs need no clearing
// beforehand).
hipError_t bucket_prepare(const BucketArgs &a, hipStream_t s);

// The swept axis of later bucketed calls (process-wide): -1 lets every
// instance's plan choose the axis with the fewest expected 1-D candidates
// (the default); k >= 0 sweeps input axis k (axis 0 where k >= d).
void set_sweep_axis(int axis);
int sweep_axis();

// Splitting overfull buckets (one instance, slabs).  When an attempt fails
// only because some buckets hold more records than a sweep workgroup can
// (Header::pad[1] == kSplittable), bucket_split() enqueues the split plan:
// every overfull column becomes several consecutive buckets under a map that
// stays monotone, and Header::split_nb receives the new bucket count (0: no
// split is possible; the caller falls back).  With split_layout(L, split_nb)
// as the layout, bucket_prepare_split() then enqueues the count, offsets and
// scatter of the split map, and bucket_sweep() the sweep, as for a first
// attempt; the map, the validation and the cleared outputs of the first
// attempt are reused.
hipError_t bucket_split(const BucketArgs &a, hipStream_t s);
BucketLayout split_layout(const BucketLayout &L, uint32_t nb);
hipError_t bucket_prepare_split(const BucketArgs &a, hipStream_t s);

// Enqueue the per-bucket sweep.  mode 0: totals only; 1: totals and
// per-update counts (per_update zeroed beforehand, indexed by the update's
// row in the concatenated arrays); 2: write pairs (row of the update, row of
// the subscription) at pair_off[u] plus a per-update cursor (zeroed
// beforehand).  In mode 2, if ``gate`` is not null and *gate is 0 on the
// device, the launch writes nothing (the pairs did not fit their buffer).
// A mode-2 sweep visits only the buckets in which the mode-1 sweep before it
// found pairs, so that one must be made with ``mark`` (which marks them).
hipError_t bucket_sweep(const BucketArgs &a, int mode, int32_t *per_update,
                        const unsigned long long *pair_off, uint32_t *cursor, uint32_t *out_u,
                        uint32_t *out_s, unsigned long long *total, hipStream_t s,
                        const uint32_t *gate = nullptr, bool mark = false);

// Slab layout of one instance for a resident simulation (resident.hip):
// bucket j's regions at slots [j * cap, j * cap + cnt[j]) of ids (region
// index, updates first), lo and hi (float [slots][d], row-major); empty
// regions in the extra slab nb.  Requires cap == kBucketCap.
struct SlabBuild {
  uint32_t *ids;
  float *lo, *hi;
  uint32_t *cnt;       // [nb + 1]
  uint32_t cap;
  uint32_t *overflow;  // set to nonzero if some slab could not hold its regions
};

// Enqueues sampling, the bucket map, validation and counting (as
// bucket_prepare, into a.hdr), then the slab fill.  a describes a batch of
// one with at least one bucket.
hipError_t bucket_build_slabs(const BucketArgs &a, const SlabBuild &sb, hipStream_t s);

// Count-mode sweep of slab-resident buckets.  rec / bs_rec hold the records
// of bucket j at [j * cap, j * cap + cnt[j]) and its boundary-state records
// at [j * bs_slab, j * bs_slab + bs_cnt[j]).  A record's region field is the
// slot g of the region's coordinates in lo / hi (float [slots][d]) for an
// update, nv + g for a subscription.  Pairs are added to hdr->total; a
// bucket that does not fit sets hdr->pad[0].
struct SlabSweep {
  const uint32_t *rec, *bs_rec, *cnt, *bs_cnt;
  uint32_t cap, bs_slab, nb, nv;
  const float *lo, *hi;
  Header *hdr;
  int d;
};
hipError_t bucket_sweep_slabs(const SlabSweep &w, hipStream_t s);

}  // namespace ddm

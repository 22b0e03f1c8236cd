// Internal interface of the batched path (batch.hip): a validated,
// laid-out batch that can be enqueued without blocking the host and
// finished later (used by the serving runtime).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/ddm.h"
#include "bucket_path.h"

namespace ddm {

// Byte offsets of the batch workspace.
struct BatchLayout {
  size_t hdr, offs, gate, cnt, off, cur, ps, scan_tmp, region;
  BucketLayout bk;
  size_t total;
};

struct Batch {
  std::vector<InstSpec> spec;
  std::vector<int64_t> uoff, soff;  // first output row of each instance's updates / subscriptions
  int64_t B;
  int d, mode;      // output mode (without DDM_CLOSED)
  uint32_t closed;  // closed intervals
  void *ws;
  size_t ws_bytes;
  uint64_t *counts;
  int32_t *per_update, *pairs;
  int64_t *pair_off;
  int64_t cap;
  bool bucketed;  // the batch fits the bucketed plan
  BatchLayout L;
  int match_mode() const { return mode | (closed ? DDM_CLOSED : 0); }  // as ddm_match takes it
};

// Validates a batch given as instances (output rows follow the instance
// order) and fills c; no device work.
int make_batch(Batch &c, std::vector<InstSpec> spec, int d, int mode, void *ws, size_t ws_bytes,
               const ddm_tuning *tuning, uint64_t *counts, int32_t *per_update, int32_t *pairs,
               int64_t *pair_off, int64_t cap);

// Workspace for these instances under one tuning (or, if null, under the
// default and every autotuner candidate), fallback included.
size_t workspace_for(const std::vector<InstSpec> &spec, int d, int mode, int64_t cap,
                     const ddm_tuning *tuning);

// Page-locked staging that batch_begin() needs to run without blocking.
size_t batch_staging_bytes(const Batch &c);

// Uploads the plan and enqueues every launch on s.  With pinned staging it
// returns without waiting (the staging stays untouched until the stream has
// passed it); without, it waits for the stream.  DDM_E_UNSUPPORTED if the
// batch does not fit the bucketed plan (batch_finish() then runs it
// instance by instance).
int batch_begin(const Batch &c, hipStream_t s, void *pinned);

// Waits for s, reads the outcome, runs the per-instance fallback if needed
// (then *fell_back, if given, is set: outputs were rewritten after the
// stream's own work).
int batch_finish(const Batch &c, hipStream_t s, uint64_t *total_host, bool *fell_back = nullptr);

}  // namespace ddm

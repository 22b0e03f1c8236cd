// Launchers of the device-wide sort-based matching kernels
// (match_global.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace ddm {

struct SweepArgs {
  const uint32_t *skey;    // sorted lower keys [count]
  const uint32_t *sidx;    // region index of each sorted lower endpoint
  const uint32_t *s_khi;   // upper key of each sorted region
  const float *s_other;    // [2*dm1][stride] other-axis lo/hi in sorted order
  size_t stride;
  uint32_t count;          // non-empty regions
  uint32_t n;              // number of updates (regions < n are updates)
  int dm1;                 // number of other axes (d - 1)
  uint32_t closed;         // 1: closed intervals (s_khi holds enc(hi) + 1)
  int32_t *per_update;     // mode 1: per-update counts (zeroed beforehand)
  const unsigned long long *offsets;  // mode 2: first pair slot of each update
  uint32_t *cursor;        // mode 2: per-update running slot (zeroed)
  uint32_t *out_u, *out_s; // mode 2: pair staging
  unsigned long long *total;
};

constexpr unsigned kKeysMaxBlocks = 8192;
unsigned keys_grid(size_t regions);
// Validates and encodes; per-block partials (<= kKeysMaxBlocks uint4) are
// folded into hdr->err / nonempty / kmin / kmax by a one-block kernel.
// closed = 1: closed intervals (no empty boxes; khi = enc(hi) + 1).
void launch_keys(const float *ulo, const float *uhi, uint32_t n, const float *slo,
                 const float *shi, uint32_t m, int d, int axis, uint32_t closed, uint32_t *klo,
                 uint32_t *khi, uint4 *partial, Header *hdr, hipStream_t s);
void launch_gather(const uint32_t *sidx, uint32_t count, const uint32_t *khi, const float *ulo,
                   const float *uhi, uint32_t n, const float *slo, const float *shi, int d,
                   int axis, uint32_t *s_khi, float *s_other, size_t stride, hipStream_t s);
void launch_sweep(int mode, const SweepArgs &a, hipStream_t s);
void launch_interleave(const uint32_t *u, const uint32_t *sidx, int32_t *out, size_t count,
                       hipStream_t s);
// Rows of at most kRowMax pairs are ordered by launch_row_sort.
constexpr uint32_t kRowMax = 2048;
// Orders each row u (cnt[u] subscription ids at in[off[u] ..)) by id into
// ids[off[u] ..) (CSR), or, with pairs non-null, into pairs rows
// (u, id) at off[u] .. (int32 [K][2]).  Every row must hold distinct ids and
// at most kRowMax of them.  With ``done``, rows with done[u] == cnt[u] are
// skipped (already written in order).
void launch_row_sort(const unsigned long long *off, const int32_t *cnt, const uint32_t *in,
                     uint32_t n, uint32_t *ids, int32_t *pairs, hipStream_t s,
                     const uint32_t *done = nullptr);

}  // namespace ddm

// Calls the library makes on itself.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace ddm {

// ddm_match() for the library's own nested calls (batch fallbacks, resident
// repairs, the per-request server policy, per-axis counts): the same result,
// without replacing the calling thread's ddm_last_path() record.
int match_quiet(const float *upd_lo, const float *upd_hi, int64_t n, const float *sub_lo,
                const float *sub_hi, int64_t m, int d, int mode, void *workspace, size_t ws_bytes,
                void *stream, uint64_t *count_host, int32_t *per_update, int32_t *pairs,
                int64_t pair_capacity);

}  // namespace ddm

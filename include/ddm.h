/*
 * ddm.h -- C interface of libddm, sort-based region matching for Data
 * Distribution Management on AMD Instinct MI355X (gfx950).
 *
 * The operation is the matching problem of Marzolla & D'Angelo, "Parallel
 * Sort-Based Matching for Data Distribution Management on Shared-Memory
 * Multiprocessors" (DS-RT 2017), Sec. 3: given n update regions U_i and m
 * subscription regions S_j, each an axis-parallel box in d dimensions, report
 * every pair (i, j) whose boxes intersect.  Boxes are half-open on every axis,
 * [lo_k, hi_k), so boxes that only touch do not match, and a box with
 * lo_k == hi_k on some axis is empty and matches nothing.  The reduction of d
 * axes to one (AND of the 1-D tests, Sec. 3 after Algorithm 1) and the
 * sort-then-sweep structure of Algorithm 4 are what the library computes.
 *
 * Conventions shared by every entry point
 *   - ids are 0-based positions in the input arrays; a pair is written as
 *     (update id, subscription id), int32 each;
 *   - pairs come out in lexicographic (update id, subscription id) order,
 *     without duplicates; the count is exactly the number of pairs;
 *   - coordinates are float32 and are only ever compared (never combined), so
 *     results are exact; -0.0 equals +0.0; +-Inf are allowed; NaN or
 *     lo_k > hi_k on any axis is an input error;
 *   - every pointer named "device" must point to memory of the current HIP
 *     device; the caller owns every buffer, the library never allocates or
 *     frees caller memory and keeps no pointer after a call returns;
 *   - all GPU work is enqueued on the caller's stream (a hipStream_t passed as
 *     void*, NULL for the default stream); a call is not re-entrant on the
 *     same workspace;
 *   - no exception crosses this interface; every call returns a DDM_* code.
 */
#ifndef DDM_H
#define DDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define DDM_OK 0
#define DDM_E_INVAL (-1)     /* bad argument, NaN coordinate, lo > hi        */
#define DDM_E_CAPACITY (-2)  /* pair buffer too small; *count_host = K      */
#define DDM_E_WORKSPACE (-3) /* workspace smaller than ddm_workspace_bytes() */
#define DDM_E_DEVICE (-4)    /* a HIP runtime call failed                    */
#define DDM_E_UNSUPPORTED (-5) /* valid request outside the supported range   */

/* Output modes (exactly one). */
#define DDM_COUNT 0      /* total number of intersecting pairs                */
#define DDM_PER_UPDATE 1 /* total + per-update match counts                  */
#define DDM_PAIRS 2      /* total + per-update counts (optional) + pair list  */

/* Limits: n + m must be below 2^31 (ids and sorted positions are 32-bit) and
 * 1 <= d <= DDM_MAX_DIMS. */
#define DDM_MAX_DIMS 16

/*
 * Size in bytes of the device workspace that ddm_match() needs for these
 * sizes and this mode.  For DDM_PAIRS the workspace also holds the pair
 * staging and ordering buffers for up to pair_capacity pairs (ignored in the
 * other modes).  Returns 0 for arguments ddm_match() would reject.
 */
size_t ddm_workspace_bytes(int64_t n, int64_t m, int d, int mode, int64_t pair_capacity);

/*
 * Sort-based matching of n update boxes against m subscription boxes
 * (Sec. 3 problem statement; Algorithm 4 with the per-axis AND of Sec. 3).
 *
 *   upd_lo, upd_hi  device, float32 [n][d] row-major: lower / upper corner of
 *                   update i on axis k at [i*d + k]
 *   sub_lo, sub_hi  device, float32 [m][d] row-major, same layout
 *   n, m            number of update / subscription boxes (>= 0)
 *   d               number of axes (1 .. DDM_MAX_DIMS)
 *   mode            DDM_COUNT, DDM_PER_UPDATE or DDM_PAIRS
 *   workspace       device, at least ddm_workspace_bytes(n, m, d, mode,
 *                   pair_capacity) bytes, 256-byte aligned; contents on entry
 *                   are ignored and on return undefined
 *   ws_bytes        size of workspace
 *   stream          hipStream_t as void*, or NULL
 *   count_host      host, out: the total number of pairs K (required)
 *   per_update      device, out, int32 [n]: matches per update; required for
 *                   DDM_PER_UPDATE, optional (NULL) for DDM_PAIRS, ignored for
 *                   DDM_COUNT
 *   pairs           device, out, int32 [pair_capacity][2]: the pairs in
 *                   lexicographic order; DDM_PAIRS only
 *   pair_capacity   rows available in pairs
 *
 * The call returns after the result is complete on the device and
 * *count_host is set (it synchronises with the stream).  Errors: DDM_E_INVAL
 * for bad sizes, NULL pointers where data is needed, or (detected on the
 * device) a NaN coordinate or lo > hi, in which case no output is defined;
 * DDM_E_WORKSPACE if ws_bytes is too small (nothing is launched);
 * DDM_E_CAPACITY if K > pair_capacity: *count_host is set to K, per_update
 * (if given) is complete and pairs is untouched, so the caller can retry with
 * a larger buffer; DDM_E_DEVICE if the HIP runtime reports an error.
 */
int ddm_match(const float *upd_lo, const float *upd_hi, int64_t n,
              const float *sub_lo, const float *sub_hi, int64_t m,
              int d, int mode, void *workspace, size_t ws_bytes, void *stream,
              uint64_t *count_host, int32_t *per_update,
              int32_t *pairs, int64_t pair_capacity);

/* Human-readable text for a DDM_* return code (static storage). */
const char *ddm_strerror(int code);

/*
 * Implementation selection (process-global, for tests and benchmarks).
 * Both implementations compute the same result (the pairs of Sec. 3, swept
 * as in Algorithm 4):
 *   DDM_PATH_BUCKETED  regions are partitioned by their axis-0 lower
 *                      coordinate into buckets (consecutive segments of the
 *                      sorted endpoint list, as in Algorithm 5); each bucket
 *                      is sorted and swept in on-chip memory, starting from
 *                      the regions of earlier buckets still active at its
 *                      start (the boundary state of Algorithm 6); available
 *                      for d <= 3;
 *   DDM_PATH_GLOBAL    a device-wide sort of the lower endpoints and a sweep
 *                      over device memory; any d.
 * DDM_PATH_AUTO (default) uses the bucketed path where available and falls
 * back to the global one when a bucket or the boundary state does not fit.
 * A forced DDM_PATH_BUCKETED call returns DDM_E_UNSUPPORTED instead of
 * falling back.  ddm_set_path() returns DDM_E_INVAL for an unknown value;
 * ddm_last_path() reports the path that produced the last successful result
 * of ddm_match() on any thread (0 if none).
 */
#define DDM_PATH_AUTO 0
#define DDM_PATH_BUCKETED 1
#define DDM_PATH_GLOBAL 2
int ddm_set_path(int path);
int ddm_last_path(void);

/*
 * Per-phase GPU timing (diagnostic; not part of the method).
 *
 * ddm_profile(1) clears the totals and starts recording: every later call of
 * this library brackets each kernel phase with HIP events on the caller's
 * stream and, once the call has synchronised, adds the elapsed time of each
 * phase to a running total.  ddm_profile(0) stops recording.  The recorder is
 * process-global and not thread-safe; it adds one event record per phase.
 *
 * ddm_profile_report() writes the totals as a JSON object
 * {"phase": {"ms": total_milliseconds, "launches": n}, ...} into buf (host,
 * len bytes, NUL-terminated).  Returns DDM_OK, or, if buf is NULL or too
 * small, the number of bytes needed.
 */
int ddm_profile(int enable);
int ddm_profile_report(char *buf, size_t len);

#ifdef __cplusplus
}
#endif

#endif /* DDM_H */

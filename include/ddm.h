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
 * lo_k == hi_k on some axis is empty and matches nothing -- unless the mode
 * carries DDM_CLOSED (below): then boxes are closed, [lo_k, hi_k], as in the
 * tests of Algorithm 1, touching boxes match and lo_k == hi_k is a point that
 * matches every box containing it.  The reduction of d
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
#define DDM_E_SCRATCH (-6)   /* ddm_match_noalloc(): request beyond its array  */

/* Output modes (exactly one). */
#define DDM_COUNT 0      /* total number of intersecting pairs                */
#define DDM_PER_UPDATE 1 /* total + per-update match counts                  */
#define DDM_PAIRS 2      /* total + per-update counts (optional) + pair list  */

/* Interval flag, OR-ed into the mode of ddm_workspace_bytes, ddm_match, the
 * batched calls and the graph calls: closed boxes [lo_k, hi_k] on every axis
 * (Algorithm 1's tests: lo <= hi' and lo' <= hi).  Without it boxes are
 * half-open.  The serving runtime and ddm_dim_counts are half-open only. */
#define DDM_CLOSED 16

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
 *   mode            DDM_COUNT, DDM_PER_UPDATE or DDM_PAIRS, optionally
 *                   | DDM_CLOSED
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

/*
 * The same matching with the result as compressed rows (CSR), the form an
 * event router consumes: update i's matching subscriptions are
 * sub_ids[row_off[i] .. row_off[i+1]), in ascending order.  This is the pair
 * list of DDM_PAIRS without its first column (the pairs of the problem
 * statement of Sec. 3, grouped by update).
 *
 *   flags      0 or DDM_CLOSED
 *   workspace  at least ddm_workspace_bytes(n, m, d, DDM_PAIRS | flags,
 *              capacity) bytes, 256-byte aligned
 *   row_off    device, out, int64 [n + 1] (required): row_off[0] = 0,
 *              row_off[n] = K
 *   sub_ids    device, out, int32 [capacity] (required if capacity > 0)
 *   capacity   entries available in sub_ids
 *
 * Other arguments and errors as for ddm_match().  If K > capacity the call
 * returns DDM_E_CAPACITY with *count_host = K and row_off complete (sub_ids
 * untouched), so the caller can size sub_ids and retry.
 */
int ddm_match_csr(const float *upd_lo, const float *upd_hi, int64_t n,
                  const float *sub_lo, const float *sub_hi, int64_t m,
                  int d, int flags, void *workspace, size_t ws_bytes, void *stream,
                  uint64_t *count_host, int64_t *row_off, int32_t *sub_ids,
                  int64_t capacity);

/*
 * For callers that cannot allocate memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it):
 * ddm_match() without a workspace argument.  The workspace is a static
 * device array of DDM_NOALLOC_SCRATCH_BYTES inside the library; each device
 * the library runs on holds its own copy from the first call on it until
 * the process ends.  The call allocates nothing (no device, page-locked or
 * graph memory; no profiling events) and never captures or replays a graph.
 *
 *   arguments   as for ddm_match(), minus workspace and ws_bytes; inputs and
 *               outputs are still the caller's device buffers
 *
 * Errors: as ddm_match(); DDM_E_SCRATCH, before anything touches the GPU,
 * if ddm_workspace_bytes(n, m, d, mode, pair_capacity) exceeds
 * DDM_NOALLOC_SCRATCH_BYTES (64 MiB: n + m up to about 2.0e6 boxes for
 * d = 2, 1.6e6 for d = 3, in count or per-update mode); DDM_E_UNSUPPORTED while ddm_profile(1) is on or
 * on a device numbered 64 or above.  Sharing: every call on a device uses
 * that device's one array, which keeps the last call's contents (each call
 * clears what it needs).  Calls of one process on one device take turns (a
 * lock held until the call has synchronised); work that bypasses this
 * entry point and touches the array would race with them.
 */
#define DDM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int ddm_match_noalloc(const float *upd_lo, const float *upd_hi, int64_t n,
                      const float *sub_lo, const float *sub_hi, int64_t m,
                      int d, int mode, void *stream, uint64_t *count_host,
                      int32_t *per_update, int32_t *pairs, int64_t pair_capacity);

/*
 * Per-axis 1-D candidate counts (diagnostic).  counts_host[k] (host, [d])
 * receives K_1D(k): the number of (update, subscription) pairs whose
 * intervals on axis k intersect, counted among the boxes that are non-empty
 * on every axis -- the pairs a sweep along axis k would examine before the
 * other axes filter them (Sec. 3, the reduction of d axes to one after
 * Algorithm 1; the d = 1 count of Algorithm 4 on each axis).  Arguments as
 * for ddm_match(); the workspace is ddm_dim_counts_workspace_bytes() bytes.
 * Synchronises with the stream.  Errors as ddm_match() in DDM_COUNT mode.
 */
size_t ddm_dim_counts_workspace_bytes(int64_t n, int64_t m, int d);
int ddm_dim_counts(const float *upd_lo, const float *upd_hi, int64_t n,
                   const float *sub_lo, const float *sub_hi, int64_t m, int d,
                   void *workspace, size_t ws_bytes, void *stream, uint64_t *counts_host);

/* ------------------------------------------------------------------------
 * Batches of independent instances.
 *
 * B instances of the problem above (Sec. 3) are stored back to back: instance
 * b has the update rows [upd_off[b], upd_off[b+1]) of upd_lo / upd_hi and the
 * subscription rows [sub_off[b], sub_off[b+1]) of sub_lo / sub_hi.  upd_off
 * and sub_off are HOST arrays of B + 1 int64 offsets, starting at 0 and
 * non-decreasing; instances may be empty.  Every instance is matched on its
 * own, exactly as ddm_match() would match it; ids in the outputs are local to
 * the instance (0-based within its rows).  All instances share one launch
 * sequence: every kernel covers the buckets, blocks and pairs of the whole
 * batch, which is what makes small instances cheap.  The outputs:
 *
 *   counts      device, out, uint64 [B]: pairs of each instance (required)
 *   per_update  device, out, int32 [upd_off[B]]: matches of every update, at
 *               its row; required for DDM_PER_UPDATE, optional for DDM_PAIRS
 *   pairs       device, out, int32 [pair_capacity][2]: instance b's pairs at
 *               rows [pair_off[b], pair_off[b+1]), each instance's in
 *               lexicographic order; DDM_PAIRS only
 *   pair_off    device, out, int64 [B + 1]; DDM_PAIRS only (set also when the
 *               pairs do not fit, so the caller learns the size it needs)
 *
 * Totals over the batch must stay below 2^31 updates + subscriptions and
 * pair_capacity below 2^31.
 * ------------------------------------------------------------------------ */

/* Launch-shape parameters of the batched path (see ddm_batch_autotune). */
typedef struct ddm_tuning {
  int32_t target;            /* mean regions per bucket, 64 .. 1536           */
  int32_t sweep_threads;     /* threads of a sweep workgroup: 256 or 512      */
  int32_t groups_per_thread; /* count/scatter: groups of 4 rows per thread    */
  int32_t max_blocks;        /* count/scatter workgroups per instance at most */
} ddm_tuning;

/* The tuning used when none is given. */
void ddm_default_tuning(ddm_tuning *out);

/*
 * Workspace bytes that ddm_match_batched() and ddm_batch_graph_create() need
 * for this batch under the given tuning, or, if tuning is NULL, under the
 * default tuning and every candidate of ddm_batch_autotune() (so that one
 * workspace serves the autotuner), in both cases including what the
 * per-instance fallback needs.  Returns 0 for arguments the calls would
 * reject.  A call given a tuning whose need exceeds ws_bytes returns
 * DDM_E_WORKSPACE.
 */
size_t ddm_batch_workspace_bytes(const int64_t *upd_off, const int64_t *sub_off, int64_t B, int d,
                                 int mode, int64_t pair_capacity, const ddm_tuning *tuning);

/*
 * Matches every instance of the batch (arguments as described above; the
 * other arguments as for ddm_match()).  tuning may be NULL (default).  The
 * call synchronises with the stream and sets *total_host (required) to the
 * sum of counts.  Errors: as ddm_match(); DDM_E_CAPACITY if the pairs of all
 * instances exceed pair_capacity (counts, per_update and pair_off are then
 * complete, pairs untouched).  When a bucket of some instance overflows its
 * on-chip buffer, or d > 8, the instances are matched one by one with the
 * device-wide path instead (same results).
 */
int ddm_match_batched(const float *upd_lo, const float *upd_hi, const int64_t *upd_off,
                      const float *sub_lo, const float *sub_hi, const int64_t *sub_off,
                      int64_t B, int d, int mode, void *workspace, size_t ws_bytes, void *stream,
                      const ddm_tuning *tuning, uint64_t *counts, uint64_t *total_host,
                      int32_t *per_update, int32_t *pairs, int64_t *pair_off,
                      int64_t pair_capacity);

/*
 * The same for instances held in separate arrays: inst[b] gives instance b's
 * device row arrays (float32 [n][d] / [m][d]) and sizes.  Output rows
 * (per_update, pair_off) number the updates of all instances consecutively
 * in instance order, exactly as if the instances were stored back to back;
 * ids in pairs are local to the instance.  Errors as ddm_match_batched().
 */
typedef struct ddm_instance {
  const float *upd_lo, *upd_hi;
  const float *sub_lo, *sub_hi;
  int64_t n, m;
} ddm_instance;
size_t ddm_multi_workspace_bytes(const ddm_instance *inst, int64_t B, int d, int mode,
                                 int64_t pair_capacity, const ddm_tuning *tuning);
int ddm_match_multi(const ddm_instance *inst, int64_t B, int d, int mode, void *workspace,
                    size_t ws_bytes, void *stream, const ddm_tuning *tuning, uint64_t *counts,
                    uint64_t *total_host, int32_t *per_update, int32_t *pairs,
                    int64_t *pair_off, int64_t pair_capacity);

/*
 * The batch as one captured HIP graph.  ddm_batch_graph_create() validates
 * the arguments, writes the batch plan into the workspace and captures every
 * launch of ddm_match_batched() (from zeroing the outputs to the ordered
 * pairs) into a graph, with the pointers and sizes given here; the buffers
 * must stay valid and the workspace reserved for the graph until it is
 * destroyed.  ddm_batch_graph_launch() enqueues one replay on a stream and
 * returns at once; the input arrays may be rewritten between replays (same
 * sizes).  ddm_batch_graph_result() waits for the stream, sets *total_host
 * and returns what ddm_match_batched() would return for that replay (running
 * the per-instance fallback itself if a bucket overflowed).  tuning may be
 * NULL (default).  Errors of create: as ddm_match_batched() for the
 * arguments, DDM_E_UNSUPPORTED if d > 8 or the batch does not fit the
 * bucketed plan, DDM_E_DEVICE if capture fails.
 */
typedef struct ddm_batch_graph ddm_batch_graph;
int ddm_batch_graph_create(const float *upd_lo, const float *upd_hi, const int64_t *upd_off,
                           const float *sub_lo, const float *sub_hi, const int64_t *sub_off,
                           int64_t B, int d, int mode, void *workspace, size_t ws_bytes,
                           const ddm_tuning *tuning, uint64_t *counts, int32_t *per_update,
                           int32_t *pairs, int64_t *pair_off, int64_t pair_capacity,
                           ddm_batch_graph **out);
int ddm_batch_graph_launch(ddm_batch_graph *g, void *stream);
int ddm_batch_graph_result(ddm_batch_graph *g, void *stream, uint64_t *total_host);
int ddm_batch_graph_destroy(ddm_batch_graph *g);

/*
 * Autotuner: times one replay of the batch's graph for every candidate
 * tuning (bucket target 768 / 1024 / 1536, sweep workgroups of 256 / 512
 * threads, 1 or 4 groups per count/scatter thread), checks that all
 * candidates produce the same counts, and writes the fastest to *best and
 * its replay time in milliseconds to *best_ms (optional).  Arguments as for
 * ddm_batch_graph_create(); the outputs hold the last candidate's result.
 */
int ddm_batch_autotune(const float *upd_lo, const float *upd_hi, const int64_t *upd_off,
                       const float *sub_lo, const float *sub_hi, const int64_t *sub_off,
                       int64_t B, int d, int mode, void *workspace, size_t ws_bytes, void *stream,
                       uint64_t *counts, int32_t *per_update, int32_t *pairs, int64_t *pair_off,
                       int64_t pair_capacity, ddm_tuning *best, double *best_ms);

/* ------------------------------------------------------------------------
 * Serving: resident simulations, one matching request per time step.
 *
 * A simulation's regions (device float32 arrays, owned by the caller, updated
 * in place) stay in device memory for its whole life.  A request for
 * simulation j takes one random-walk step of j's regions and then counts the
 * intersecting pairs of the moved regions (DDM_COUNT semantics).
 *
 * ddm_sim_step() enqueues one step on a stream: region r (updates are
 * regions 0 .. n-1, subscriptions n .. n+m-1) moves its lower corner on axis
 * k by sigma * z and its upper corner is reset to lo + side (IEEE float32
 * operations, each rounded to nearest), where z is the sum of twelve uniforms
 * minus six; the uniforms are the twelve 32-bit words (each shifted right by
 * 8) of Philox4x32-10 at counters (r, k, step, 0..2) under the 64-bit key
 * seed, so the motion is reproducible bit for bit by any implementation of
 * that generator.  step numbers the step being taken (1 for the first).
 * ------------------------------------------------------------------------ */
int ddm_sim_step(float *upd_lo, float *upd_hi, int64_t n, float *sub_lo, float *sub_hi,
                 int64_t m, int d, float side, float sigma, uint64_t seed, uint32_t step,
                 void *stream);

/* ------------------------------------------------------------------------
 * Resident simulations matched incrementally.
 *
 * The dynamic matching problem the paper names as its next step (Sec. 6;
 * regions that move between matching requests, solved for serial SBM by
 * the work cited in Sec. 2): a simulation whose regions move a little
 * between two requests keeps its sorted state instead of sorting again.  Here the state is the bucket order of the
 * bucketed path (the segments of Algorithm 5): the library keeps the
 * regions themselves in device memory, grouped by bucket in fixed-capacity
 * slabs, and a step moves them in place, moves the few that leave their
 * bucket to their new one, rebuilds the boundary state of Algorithm 6 and
 * sweeps every bucket (Algorithm 4).  Motion and result are exactly those of
 * ddm_sim_step() followed by ddm_match(DDM_COUNT) on the same rows: the
 * count is the number of intersecting pairs of half-open boxes.  When the
 * slabs cannot hold a step's outcome, that step is counted by ddm_match()
 * and the slabs are rebuilt; a simulation that keeps overflowing, or whose
 * regions do not fit the slabs (a bucket with more than 2048 regions, more
 * than 512 regions active at a bucket boundary), is matched by ddm_match()
 * instead, and the slabs are tried again every 64 steps; d > 3 is always
 * matched by ddm_match().
 *
 * ddm_resident_bytes() gives the device state size for n updates and m
 * subscriptions in d dimensions (0 for invalid sizes).
 *
 * ddm_resident_create() copies the regions in (device rows as in
 * ddm_match(); the caller's arrays are not referenced afterwards),
 * validates them and builds the slabs in state (device, 256-byte aligned,
 * owned by the caller, at least ddm_resident_bytes(); the library keeps a
 * pointer to it until ddm_resident_destroy()).  side, sigma and seed define
 * the motion as for ddm_sim_step() (side finite and >= 0, |sigma| <= 1e30).
 * It synchronises with the stream.  Errors: DDM_E_INVAL for bad arguments,
 * NaN or lo > hi; DDM_E_WORKSPACE if state_bytes is too small.  The handle
 * holds a HIP event and 256 bytes of page-locked host memory of its own.
 *
 * ddm_resident_step() enqueues step number step (>= 1; the caller numbers
 * steps as for ddm_sim_step()) and its count on the stream without blocking;
 * ddm_resident_finish() waits for it and reports the count in *count (host).
 * Every step must be finished before the next one is enqueued (DDM_E_INVAL
 * otherwise).  finish() may run repair work on the stream of the step and
 * synchronise with it.
 *
 * ddm_resident_export() writes the current corners in region order to
 * device rows of the caller (as ddm_sim_step()'s arrays) and synchronises.
 * ------------------------------------------------------------------------ */
typedef struct ddm_resident ddm_resident;

typedef struct ddm_resident_info {
  int64_t steps;        /* steps finished                                    */
  int64_t rebuilds;     /* slab rebuilds after a slab or the mover list filled */
  int64_t full_matches; /* steps counted by ddm_match() instead of the slabs */
  int64_t movers;       /* regions that changed bucket in the last step      */
  int32_t buckets;      /* buckets of the slab layout (0 in full-match mode) */
  int32_t full_mode;    /* 1: every step is matched by ddm_match()           */
} ddm_resident_info;

size_t ddm_resident_bytes(int64_t n, int64_t m, int d);
int ddm_resident_create(void *state, size_t state_bytes, const float *upd_lo,
                        const float *upd_hi, int64_t n, const float *sub_lo,
                        const float *sub_hi, int64_t m, int d, float side, float sigma,
                        uint64_t seed, void *stream, ddm_resident **out);
int ddm_resident_step(ddm_resident *r, uint32_t step, void *stream);
int ddm_resident_finish(ddm_resident *r, uint64_t *count);
int ddm_resident_export(ddm_resident *r, float *upd_lo, float *upd_hi, float *sub_lo,
                        float *sub_hi, void *stream);
int ddm_resident_get_info(const ddm_resident *r, ddm_resident_info *out);
int ddm_resident_destroy(ddm_resident *r);

/* Scheduling policies of a server. */
#define DDM_SERVE_BATCHED 0 /* continuous batching over several streams       */
#define DDM_SERVE_PLAIN 1   /* one request at a time, in arrival order, with
                               ddm_match(): the per-request baseline          */
#define DDM_SERVE_INCREMENTAL 2 /* continuous scheduling over several streams of
                               resident simulations (ddm_resident_*): each
                               simulation's state lives in the arena from its
                               registration on; the caller's arrays keep the
                               registered state until ddm_server_export()     */

typedef struct ddm_serve_stats {
  double wall_s;           /* first arrival slot to last completion           */
  int64_t launches;        /* matching launches (groups) issued               */
  double mean_batch;       /* requests per launch                             */
  double peak_arena_bytes; /* most arena bytes in use at once                 */
} ddm_serve_stats;

/*
 * Creates a server on the current device.  arena (device, arena_bytes,
 * 256-byte aligned, owned by the caller) is the HBM budget from which every
 * request's workspace is carved; requests are admitted only while their
 * workspace fits.  slots (1 .. 16): groups in flight at once, each on its own
 * stream (default priority); max_batch (1 .. 4096): requests matched by one
 * launch at most.  The plain policy uses one slot and groups of one.  The
 * server allocates a few small buffers of its own (per-slot counts, page-
 * locked staging), freed by ddm_server_destroy().
 */
typedef struct ddm_server ddm_server;
int ddm_server_create(void *arena, size_t arena_bytes, int policy, int slots, int max_batch,
                      ddm_server **out);

/* Registers a simulation (arguments as ddm_sim_step(); every simulation of a
 * server has the same d).  DDM_E_WORKSPACE if one request of it alone would
 * not fit the arena. */
int ddm_server_add_sim(ddm_server *s, float *upd_lo, float *upd_hi, int64_t n, float *sub_lo,
                       float *sub_hi, int64_t m, int d, float side, float sigma, uint64_t seed,
                       int32_t *sim_id);

/*
 * Serves count requests open-loop: request i (for simulation sim[i]) arrives
 * arrival_s[i] seconds after the start (host monotonic clock) and is released
 * to the scheduler then; each simulation's requests are served in arrival
 * order, so its k-th request always matches its state after k steps (steps
 * continue across calls).  Returns when every request has completed.  Out
 * (host, [count]): counts[i], the pairs of request i; steps[i], the step it
 * matched; latency_s[i], completion minus arrival.  stats may be NULL.
 * Errors: DDM_E_INVAL for bad arguments; the first error of a request
 * otherwise (its count is then 0).
 */
int ddm_server_run(ddm_server *s, const int32_t *sim, const double *arrival_s, int64_t count,
                   uint64_t *counts, uint32_t *steps, double *latency_s, ddm_serve_stats *stats);
/* Writes simulation sim_id's current state into the arrays it was
 * registered with (DDM_SERVE_INCREMENTAL; a no-op for the other policies,
 * whose steps update those arrays in place).  Synchronises. */
int ddm_server_export(ddm_server *s, int32_t sim_id);
int ddm_server_destroy(ddm_server *s);

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
 *                      start (the boundary state of Algorithm 6); for d >= 2
 *                      the buckets may also be cut into rows by axis 1
 *                      (boxes reaching later rows are copied there, and a
 *                      pair is counted in the row of its larger axis-1
 *                      lower bound), which the plan chooses from a sample
 *                      when it shortens the sweep; available
 *                      for d <= 8 (a pre-filter on axes 1 and 2, the exact
 *                      test on every axis);
 *   DDM_PATH_GLOBAL    a device-wide sort of the lower endpoints and a sweep
 *                      over device memory; any d.
 * DDM_PATH_AUTO (default) uses the bucketed path where available and falls
 * back to the global one when a bucket or the boundary state does not fit.
 * A forced DDM_PATH_BUCKETED call returns DDM_E_UNSUPPORTED instead of
 * falling back.  ddm_set_path() returns DDM_E_INVAL for an unknown value;
 * ddm_last_path() reports the path that served the calling thread's last
 * ddm_match(), ddm_match_csr() or ddm_match_noalloc() call (0 if that call
 * produced no result); the library's own nested calls (batch fallbacks,
 * resident repairs, the server, per-axis counts) leave it unchanged.  The
 * path request applies to every thread; both are safe to use concurrently.
 */
#define DDM_PATH_AUTO 0
#define DDM_PATH_BUCKETED 1
#define DDM_PATH_GLOBAL 2
int ddm_set_path(int path);
int ddm_last_path(void);

/*
 * The swept axis of the bucketed path (process-global, for tests and
 * benchmarks).  Any axis gives the same pairs (Sec. 3: the d-dimensional
 * test is the AND of the 1-D ones), but the work of a sweep grows with the
 * 1-D candidates of its axis.  axis = -1 (default): every instance's plan
 * sweeps the input axis with the fewest expected 1-D candidates estimated
 * from its sample (mean extent over the range of lower bounds), unless that
 * is not under half of axis 0's; axis = k (0 <= k < DDM_MAX_DIMS) sweeps
 * axis k (axis 0 for instances with d <= k).  The device-wide path and
 * resident simulations always sweep axis 0.  Returns DDM_E_INVAL for other
 * values.
 */
int ddm_set_sweep_axis(int axis);

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

/*
 * Achievable-bandwidth reference (diagnostic; not part of the method): a
 * plain device copy of ``bytes`` (a multiple of 16, both pointers device
 * memory aligned to 16 bytes) from src to dst with 16-byte loads and
 * stores, run once to warm up and then reps times on the stream; *ms_out
 * (host) receives the mean time of one copy in milliseconds.  The copy
 * moves 2 * bytes through HBM.  Synchronises; creates and destroys two HIP
 * events.  Errors: DDM_E_INVAL for bad arguments, DDM_E_DEVICE.
 */
int ddm_copy_probe(void *dst, const void *src, size_t bytes, int reps, void *stream,
                   double *ms_out);

#ifdef __cplusplus
}
#endif

#endif /* DDM_H */

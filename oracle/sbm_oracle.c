/*
 * Serial CPU oracle for region matching in Data Distribution Management.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU path.
 *
 * Follows Marzolla & D'Angelo, "Parallel Sort-Based Matching for Data
 * Distribution Management on Shared-Memory Multiprocessors" (DS-RT 2017):
 *
 *   - problem statement: report every (subscription, update) pair whose
 *     d-dimensional axis-parallel rectangles intersect (Sec. 3, first
 *     paragraph);
 *   - reduction from d dimensions to one: two rectangles overlap iff every
 *     1-D projection overlaps, i.e. the logical AND of Algorithm 1 over the
 *     d axes (Sec. 3, after Algorithm 1);
 *   - Algorithm 2 (BruteForce-1D), generalised to d axes with that AND;
 *   - Algorithm 4 (Sort-Based-Matching-1D) on axis 0, with the other d-1
 *     axes tested for every 1-D pair it reports.
 *
 * Readings taken where the paper is silent or inconsistent (each one is
 * pinned by a test against the plain definition):
 *   R1  intervals are half-open [lo, hi): an interval is active at t when
 *       lo <= t < hi (Sec. 3.4 defines "active" this way); Algorithm 1's
 *       closed test is therefore applied in its strict form lo < hi'.
 *   R2  endpoints with equal coordinates sort upper-before-lower, then
 *       update-before-subscription, then by id (the paper only asks for
 *       "non-decreasing order"); only the first rule changes the result.
 *   R3  an interval with lo == hi on any axis is empty, matches nothing and
 *       is dropped before the sweep (the paper never mentions empties).
 *   R4  lo > hi or a NaN coordinate is an input error (no result).
 *   R5  ids are 0-based; pairs are reported as (update id, subscription id)
 *       and returned in lexicographic order (the paper's L is an unordered
 *       set).
 *   R6  the closed reading, selected by the *_closed entry points, takes
 *       Algorithm 1's tests as printed: intervals [lo, hi], overlap iff
 *       lo <= hi' and lo' <= hi.  Then no interval is empty (lo == hi is a
 *       point), and endpoints with equal coordinates sort lower-before-upper
 *       (then kind, then id), so that an interval whose lower endpoint
 *       equals another's upper one is still active when that upper endpoint
 *       is swept.
 *
 * Coordinates are float32 on input and are only ever compared; each one is
 * widened to double (exact) before any comparison.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_INVAL (-1)
#define OR_E_CAPACITY (-2)
#define OR_E_NOMEM (-5)
#define OR_E_INTERNAL (-6)

#define KIND_UPD 0
#define KIND_SUB 1
#define TYPE_UPPER 0
#define TYPE_LOWER 1

/* One element of the endpoint list T of Algorithm 4. */
typedef struct {
    double coord;
    int type;   /* TYPE_UPPER or TYPE_LOWER */
    int rank;   /* tie order of the type: R2 (half-open) or R6 (closed) */
    int kind;   /* KIND_UPD or KIND_SUB */
    int64_t id; /* 0-based index inside its own set */
} Endpoint;

/* The interval reading of a call: R1-R3 (half-open) or R6 (closed). */
typedef struct {
    int closed;
} Reading;

/* Tie rank of an endpoint type: uppers first when half-open (R2), lowers
 * first when closed (R6). */
static int type_rank(const Reading *rd, int type)
{
    if (rd->closed) return type == TYPE_LOWER ? 0 : 1;
    return type == TYPE_UPPER ? 0 : 1;
}

/* a < b for half-open intervals, a <= b for closed ones (R1 / R6). */
static int before(const Reading *rd, double a, double b)
{
    return rd->closed ? a <= b : a < b;
}

/* Output sink shared by the brute force and the sweep. */
typedef struct {
    uint64_t count;
    int32_t *per_update; /* [n] or NULL */
    int32_t *pairs;      /* [cap][2] or NULL */
    int64_t cap;
} Sink;

static void report(Sink *s, int64_t upd, int64_t sub)
{
    if (s->per_update) s->per_update[upd] += 1;
    if (s->pairs && (int64_t)s->count < s->cap) {
        s->pairs[2 * s->count] = (int32_t)upd;
        s->pairs[2 * s->count + 1] = (int32_t)sub;
    }
    s->count += 1;
}

/* R4: every coordinate must be a number and lo <= hi on every axis. */
static int validate(const float *lo, const float *hi, int64_t cnt, int d)
{
    for (int64_t i = 0; i < cnt; ++i) {
        for (int k = 0; k < d; ++k) {
            double l = lo[i * d + k], h = hi[i * d + k];
            if (isnan(l) || isnan(h)) return OR_E_INVAL;
            if (l > h) return OR_E_INVAL;
        }
    }
    return OR_OK;
}

/* R3: empty on any axis means the region is empty; R6: never when closed. */
static int is_empty(const Reading *rd, const float *lo, const float *hi, int64_t i, int d)
{
    if (rd->closed) return 0;
    for (int k = 0; k < d; ++k)
        if ((double)lo[i * d + k] == (double)hi[i * d + k]) return 1;
    return 0;
}

/* Algorithm 1 for axis k, in the reading of the call (R1 or R6). */
static int intersect_1d(const Reading *rd, const float *alo, const float *ahi, int64_t a,
                        const float *blo, const float *bhi, int64_t b,
                        int d, int k)
{
    double a_low = alo[a * d + k], a_high = ahi[a * d + k];
    double b_low = blo[b * d + k], b_high = bhi[b * d + k];
    return before(rd, a_low, b_high) && before(rd, b_low, a_high);
}

/* The AND over the remaining axes 1..d-1 (axis 0 is the swept one). */
static int intersect_other_axes(const Reading *rd, const float *ulo, const float *uhi, int64_t u,
                                const float *slo, const float *shi, int64_t s,
                                int d)
{
    for (int k = 1; k < d; ++k)
        if (!intersect_1d(rd, ulo, uhi, u, slo, shi, s, d, k)) return 0;
    return 1;
}

static int cmp_pair(const void *a, const void *b)
{
    const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
    return 0;
}

static int finish(Sink *s, int want_pairs)
{
    if (want_pairs) {
        if ((int64_t)s->count > s->cap) return OR_E_CAPACITY;
        qsort(s->pairs, (size_t)s->count, 2 * sizeof(int32_t), cmp_pair);
    }
    return OR_OK;
}

static int check_args(int64_t n, int64_t m, int d, const float *ulo,
                      const float *uhi, const float *slo, const float *shi)
{
    if (n < 0 || m < 0 || d < 1) return OR_E_INVAL;
    if ((n > 0 && (!ulo || !uhi)) || (m > 0 && (!slo || !shi))) return OR_E_INVAL;
    if (validate(ulo, uhi, n, d) != OR_OK) return OR_E_INVAL;
    if (validate(slo, shi, m, d) != OR_OK) return OR_E_INVAL;
    return OR_OK;
}

/*
 * Algorithm 2 (BruteForce-1D) generalised to d axes: test all n*m pairs.
 * The per-pair test is the plain definition of a non-empty intersection of
 * two half-open boxes, max(lo) < min(hi) on every axis, which is false for
 * any empty region without a separate rule; for closed boxes (R6) it is
 * max(lo) <= min(hi).
 */
static int bruteforce(const Reading *rd, const float *ulo, const float *uhi, int64_t n,
                      const float *slo, const float *shi, int64_t m, int d,
                      uint64_t *count, int32_t *per_update, int32_t *pairs,
                      int64_t pair_cap)
{
    int rc = check_args(n, m, d, ulo, uhi, slo, shi);
    if (rc != OR_OK) return rc;
    Sink s = {0, per_update, pairs, pairs ? pair_cap : 0};
    if (per_update) memset(per_update, 0, (size_t)n * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            int hit = 1;
            for (int k = 0; k < d && hit; ++k) {
                double lo_max = fmax((double)ulo[i * d + k], (double)slo[j * d + k]);
                double hi_min = fmin((double)uhi[i * d + k], (double)shi[j * d + k]);
                hit = before(rd, lo_max, hi_min);
            }
            if (hit) report(&s, i, j);
        }
    }
    if (count) *count = s.count;
    return finish(&s, pairs != NULL);
}

/* R2: coordinate, then upper before lower (lower before upper under R6),
 * then update before subscription, then id.  The order is total, so qsort's
 * instability does not matter. */
static int cmp_endpoint(const void *a, const void *b)
{
    const Endpoint *x = (const Endpoint *)a, *y = (const Endpoint *)b;
    if (x->coord < y->coord) return -1;
    if (x->coord > y->coord) return 1;
    if (x->rank != y->rank) return x->rank < y->rank ? -1 : 1;
    if (x->kind != y->kind) return x->kind < y->kind ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return 0;
}

/* Step 2 of Algorithm 4: the lower and upper endpoint on axis 0 of every
 * region that is not empty (R3), into T; returns the number written. */
static int64_t fill_endpoints(const Reading *rd, const float *ulo, const float *uhi, int64_t n,
                              const float *slo, const float *shi, int64_t m, int d, Endpoint *T)
{
    const int rl = type_rank(rd, TYPE_LOWER), ru = type_rank(rd, TYPE_UPPER);
    int64_t t = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (is_empty(rd, ulo, uhi, i, d)) continue;
        T[t++] = (Endpoint){(double)ulo[i * d], TYPE_LOWER, rl, KIND_UPD, i};
        T[t++] = (Endpoint){(double)uhi[i * d], TYPE_UPPER, ru, KIND_UPD, i};
    }
    for (int64_t j = 0; j < m; ++j) {
        if (is_empty(rd, slo, shi, j, d)) continue;
        T[t++] = (Endpoint){(double)slo[j * d], TYPE_LOWER, rl, KIND_SUB, j};
        T[t++] = (Endpoint){(double)shi[j * d], TYPE_UPPER, ru, KIND_SUB, j};
    }
    return t;
}

/* SubSet / UpdSet of Algorithm 4: an unordered set of ids with O(1)
 * insertion and removal (dense array plus id -> slot index). */
typedef struct {
    int64_t *items;
    int64_t *slot;
    int64_t size;
} IdSet;

static int idset_init(IdSet *s, int64_t universe)
{
    s->size = 0;
    s->items = (int64_t *)malloc((size_t)(universe > 0 ? universe : 1) * sizeof(int64_t));
    s->slot = (int64_t *)malloc((size_t)(universe > 0 ? universe : 1) * sizeof(int64_t));
    if (!s->items || !s->slot) return OR_E_NOMEM;
    for (int64_t i = 0; i < universe; ++i) s->slot[i] = -1; /* not a member */
    return OR_OK;
}

static void idset_free(IdSet *s)
{
    free(s->items);
    free(s->slot);
}

/* Insertion of a member or removal of a non-member cannot happen when every
 * region's lower endpoint precedes its upper one in T; both are reported as
 * an internal error instead of corrupting the set. */
static int idset_insert(IdSet *s, int64_t id)
{
    if (s->slot[id] >= 0) return OR_E_INTERNAL;
    s->slot[id] = s->size;
    s->items[s->size++] = id;
    return OR_OK;
}

static int idset_erase(IdSet *s, int64_t id)
{
    int64_t at = s->slot[id];
    if (at < 0) return OR_E_INTERNAL;
    int64_t last = s->items[--s->size];
    s->items[at] = last;
    s->slot[last] = at;
    s->slot[id] = -1;
    return OR_OK;
}

/*
 * Algorithm 4 (Sort-Based-Matching-1D) on axis 0 with the remaining axes
 * tested per reported pair.
 *
 *   1. validate (R4) and drop empty regions (R3);
 *   2. insert the lower and the upper endpoint of every region into T;
 *   3. sort T (order R2);
 *   4. sweep T: a lower endpoint inserts its region into SubSet or UpdSet;
 *      an upper endpoint removes it and pairs it with every member of the
 *      other set (the pairs whose other axes also overlap are reported);
 *   5. return the pairs in lexicographic order (R5).
 */
static int sbm(const Reading *rd, const float *ulo, const float *uhi, int64_t n,
               const float *slo, const float *shi, int64_t m, int d,
               uint64_t *count, int32_t *per_update, int32_t *pairs,
               int64_t pair_cap)
{
    int rc = check_args(n, m, d, ulo, uhi, slo, shi);
    if (rc != OR_OK) return rc;

    int64_t total = 2 * (n + m);
    Endpoint *T = (Endpoint *)malloc((size_t)(total > 0 ? total : 1) * sizeof(Endpoint));
    if (!T) return OR_E_NOMEM;

    /* step 2: endpoints of the non-empty regions */
    int64_t t = fill_endpoints(rd, ulo, uhi, n, slo, shi, m, d, T);

    /* step 3 */
    qsort(T, (size_t)t, sizeof(Endpoint), cmp_endpoint);

    IdSet SubSet, UpdSet;
    if (idset_init(&SubSet, m) != OR_OK || idset_init(&UpdSet, n) != OR_OK) {
        free(T);
        idset_free(&SubSet);
        idset_free(&UpdSet);
        return OR_E_NOMEM;
    }

    Sink s = {0, per_update, pairs, pairs ? pair_cap : 0};
    if (per_update) memset(per_update, 0, (size_t)n * sizeof(int32_t));

    /* step 4 */
    rc = OR_OK;
    for (int64_t q = 0; q < t && rc == OR_OK; ++q) {
        const Endpoint *e = &T[q];
        if (e->kind == KIND_SUB) {
            if (e->type == TYPE_LOWER) {
                rc = idset_insert(&SubSet, e->id);
            } else {
                rc = idset_erase(&SubSet, e->id);
                for (int64_t a = 0; a < UpdSet.size; ++a) {
                    int64_t u = UpdSet.items[a];
                    if (intersect_other_axes(rd, ulo, uhi, u, slo, shi, e->id, d))
                        report(&s, u, e->id);
                }
            }
        } else {
            if (e->type == TYPE_LOWER) {
                rc = idset_insert(&UpdSet, e->id);
            } else {
                rc = idset_erase(&UpdSet, e->id);
                for (int64_t a = 0; a < SubSet.size; ++a) {
                    int64_t sb = SubSet.items[a];
                    if (intersect_other_axes(rd, ulo, uhi, e->id, slo, shi, sb, d))
                        report(&s, e->id, sb);
                }
            }
        }
    }

    free(T);
    idset_free(&SubSet);
    idset_free(&UpdSet);
    if (rc != OR_OK) return rc;
    if (count) *count = s.count;
    /* step 5 */
    return finish(&s, pairs != NULL);
}

/* Public entry points: half-open (R1-R3) and closed (R6) readings. */
int oracle_bruteforce(const float *ulo, const float *uhi, int64_t n,
                      const float *slo, const float *shi, int64_t m, int d,
                      uint64_t *count, int32_t *per_update, int32_t *pairs,
                      int64_t pair_cap)
{
    const Reading rd = {0};
    return bruteforce(&rd, ulo, uhi, n, slo, shi, m, d, count, per_update, pairs, pair_cap);
}

int oracle_bruteforce_closed(const float *ulo, const float *uhi, int64_t n,
                             const float *slo, const float *shi, int64_t m, int d,
                             uint64_t *count, int32_t *per_update, int32_t *pairs,
                             int64_t pair_cap)
{
    const Reading rd = {1};
    return bruteforce(&rd, ulo, uhi, n, slo, shi, m, d, count, per_update, pairs, pair_cap);
}

int oracle_sbm(const float *ulo, const float *uhi, int64_t n,
               const float *slo, const float *shi, int64_t m, int d,
               uint64_t *count, int32_t *per_update, int32_t *pairs,
               int64_t pair_cap)
{
    const Reading rd = {0};
    return sbm(&rd, ulo, uhi, n, slo, shi, m, d, count, per_update, pairs, pair_cap);
}

int oracle_sbm_closed(const float *ulo, const float *uhi, int64_t n,
                      const float *slo, const float *shi, int64_t m, int d,
                      uint64_t *count, int32_t *per_update, int32_t *pairs,
                      int64_t pair_cap)
{
    const Reading rd = {1};
    return sbm(&rd, ulo, uhi, n, slo, shi, m, d, count, per_update, pairs, pair_cap);
}

/*
 * The serial SubSet / UpdSet of Algorithm 4 right after a given number of
 * endpoints of the sorted list T have been swept, for several cut points at
 * once.  Used by the tests of the segment-boundary state (Algorithm 5 is
 * equivalent to Algorithm 4 iff segment p starts from exactly this state).
 *
 * cuts[c] (non-decreasing) is a number of endpoints of the sorted T of the
 * non-empty regions; state_kind/state_id receive, for every cut, the members
 * of both sets (kind 0 = update, 1 = subscription) in ascending (kind, id)
 * order, concatenated; offsets[c] .. offsets[c+1] delimit cut c.  Returns the
 * total number of members written, or a negative error.
 */
static int cmp_member(const void *a, const void *b)
{
    const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
    return 0;
}

int64_t oracle_sweep_state(const float *ulo, const float *uhi, int64_t n,
                           const float *slo, const float *shi, int64_t m,
                           int d, const int64_t *cuts, int64_t ncuts,
                           int64_t *offsets, int32_t *state_kind,
                           int64_t *state_id, int64_t state_cap)
{
    int rc = check_args(n, m, d, ulo, uhi, slo, shi);
    if (rc != OR_OK) return rc;
    int64_t total = 2 * (n + m);
    Endpoint *T = (Endpoint *)malloc((size_t)(total > 0 ? total : 1) * sizeof(Endpoint));
    if (!T) return OR_E_NOMEM;
    const Reading half_open = {0};
    int64_t t = fill_endpoints(&half_open, ulo, uhi, n, slo, shi, m, d, T);
    qsort(T, (size_t)t, sizeof(Endpoint), cmp_endpoint);

    IdSet SubSet, UpdSet;
    if (idset_init(&SubSet, m) != OR_OK || idset_init(&UpdSet, n) != OR_OK) {
        free(T);
        idset_free(&SubSet);
        idset_free(&UpdSet);
        return OR_E_NOMEM;
    }
    int64_t written = 0, q = 0;
    int64_t *tmp = (int64_t *)malloc((size_t)((n + m) > 0 ? (n + m) : 1) * 2 * sizeof(int64_t));
    if (!tmp) {
        free(T);
        idset_free(&SubSet);
        idset_free(&UpdSet);
        return OR_E_NOMEM;
    }
    for (int64_t c = 0; c < ncuts; ++c) {
        int64_t stop = cuts[c] < t ? cuts[c] : t;
        for (; q < stop; ++q) {
            const Endpoint *e = &T[q];
            IdSet *set = e->kind == KIND_SUB ? &SubSet : &UpdSet;
            int r2 = e->type == TYPE_LOWER ? idset_insert(set, e->id) : idset_erase(set, e->id);
            if (r2 != OR_OK) {
                free(tmp);
                free(T);
                idset_free(&SubSet);
                idset_free(&UpdSet);
                return r2;
            }
        }
        int64_t k = 0;
        for (int64_t a = 0; a < UpdSet.size; ++a) { tmp[2 * k] = KIND_UPD; tmp[2 * k + 1] = UpdSet.items[a]; ++k; }
        for (int64_t a = 0; a < SubSet.size; ++a) { tmp[2 * k] = KIND_SUB; tmp[2 * k + 1] = SubSet.items[a]; ++k; }
        qsort(tmp, (size_t)k, 2 * sizeof(int64_t), cmp_member);
        offsets[c] = written;
        for (int64_t a = 0; a < k; ++a) {
            if (written < state_cap) {
                state_kind[written] = (int32_t)tmp[2 * a];
                state_id[written] = tmp[2 * a + 1];
            }
            ++written;
        }
    }
    offsets[ncuts] = written;
    free(tmp);
    free(T);
    idset_free(&SubSet);
    idset_free(&UpdSet);
    return written > state_cap ? OR_E_CAPACITY : written;
}

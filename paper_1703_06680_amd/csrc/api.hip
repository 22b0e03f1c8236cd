// C interface of libddm (declared in include/ddm.h).
//
// Two implementations of the same matching sit behind ddm_match():
//   - the bucketed path (bucket_path.hip): regions are partitioned by their
//     swept-axis lower coordinate into buckets that are sorted and swept in
//     LDS, with each bucket's boundary state delivered from the earlier ones;
//     used when d <= 8 and the bucket count fits, and every bucket and the
//     boundary state fit their buffers;
//   - the device-wide path (match_global.hip): a global radix sort of the
//     lower keys, a gather of the other axes into sorted order and a forward
//     sweep over device memory; it has no size limit beyond 2^31 regions and
//     is the fallback when a bucket overflows.
// Both produce identical results; ddm_set_path() can force one of them.
#include <string.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/ddm.h"
#include "internal.h"
#include "bucket_path.h"
#include "common.h"
#include "match_global.h"
#include "primitives.h"
#include "profile.h"

namespace ddm {
namespace {

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// The implementation requested (process-wide) and the one that produced the
// calling thread's last result; the library's own nested calls (batches,
// resident simulations, the server, per-axis counts) leave the latter alone.
std::atomic<int> g_path_request{DDM_PATH_AUTO};
thread_local int t_last_path = 0;

// Byte offsets of every workspace buffer.  The buffers of the two paths share
// one region (only one path runs at a time).
struct Layout {
  size_t hdr, partial;
  size_t cnt, off, cur, own, pu, ps, pu2, ps2, scan_tmp, pair_sort_tmp;  // pair mode
  size_t region;
  // device-wide path, relative to region
  size_t klo, khi, vals_a, keys_b, vals_b, sort_tmp, s_khi, s_other, global_bytes;
  bool bucket_ok;
  BucketLayout B;
  size_t total;
};

// The pointers only enter the bucketed plan (null when only sizes matter).
Layout make_layout(int64_t n, int64_t m, int d, int mode, int64_t cap,
                   const float *ulo = nullptr, const float *uhi = nullptr,
                   const float *slo = nullptr, const float *shi = nullptr,
                   bool closed = false) {
  Layout L{};
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t o = at;
    at += align256(bytes);
    return o;
  };
  L.hdr = take(sizeof(Header));
  L.partial = take(kKeysMaxBlocks * sizeof(uint4));
  if (mode == DDM_PAIRS) {
    const size_t c = (size_t)(cap > 0 ? cap : 0);
    L.cnt = take((size_t)n * sizeof(int32_t));
    L.off = take((size_t)n * sizeof(unsigned long long));
    L.cur = take((size_t)n * sizeof(uint32_t));
    L.own = take((size_t)n * sizeof(uint32_t));
    L.pu = take(c * sizeof(uint32_t));
    L.ps = take(c * sizeof(uint32_t));
    L.pu2 = take(c * sizeof(uint32_t));
    L.ps2 = take(c * sizeof(uint32_t));
    L.scan_tmp = take(scan_temp_bytes((size_t)n));
    L.pair_sort_tmp = take(radix_sort_temp_bytes((uint32_t)(c ? c : 1)));
  }
  L.region = at;
  // device-wide path
  size_t g = 0;
  auto gtake = [&](size_t bytes) {
    size_t o = g;
    g += align256(bytes);
    return o;
  };
  const size_t N = (size_t)(n + m);
  const size_t u4 = N * sizeof(uint32_t);
  L.klo = gtake(u4);
  L.khi = gtake(u4);
  L.vals_a = gtake(u4);
  L.keys_b = gtake(u4);
  L.vals_b = gtake(u4);
  L.sort_tmp = gtake(radix_sort_temp_bytes((uint32_t)N));
  L.s_khi = gtake(u4);
  L.s_other = gtake((size_t)2 * (d - 1) * u4);
  L.global_bytes = g;
  // bucketed path
  L.bucket_ok = bucket_path_supported(d, n, m);
  size_t region_bytes = g;
  if (L.bucket_ok) {
    L.B = bucket_layout(ulo, uhi, n, slo, shi, m, d, closed);
    if (L.B.bytes > region_bytes) region_bytes = L.B.bytes;
  }
  L.total = L.region + align256(region_bytes);
  return L;
}

// Splits a mode argument into the output mode and the interval flag; false
// for unknown bits.
bool split_mode(int mode, int *out, bool *closed) {
  *closed = (mode & DDM_CLOSED) != 0;
  *out = mode & ~DDM_CLOSED;
  return *out == DDM_COUNT || *out == DDM_PER_UPDATE || *out == DDM_PAIRS;
}

bool sizes_ok(int64_t n, int64_t m, int d, int mode) {
  if (n < 0 || m < 0) return false;
  if (n + m >= (int64_t(1) << 31)) return false;
  if (d < 1 || d > DDM_MAX_DIMS) return false;
  if (mode != DDM_COUNT && mode != DDM_PER_UPDATE && mode != DDM_PAIRS) return false;
  return true;
}

int bit_length(uint32_t x) { return x ? 32 - __builtin_clz(x) : 0; }

#define DDM_HIP(call)                              \
  do {                                             \
    if ((call) != hipSuccess) return DDM_E_DEVICE; \
  } while (0)

constexpr int kFallback = 1;  // internal: the bucketed path asks for the other one
constexpr int kSplit = 2;     // internal: a replayed attempt overflowed buckets that can be split

template <typename T>
T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// Sorts (u, s) pair staging buffers lexicographically: stable by s, then
// stable by u.  Returns the buffers holding the result.
hipError_t order_pairs(uint32_t *pu, uint32_t *ps, uint32_t *pu2, uint32_t *ps2, uint32_t K,
                       int64_t n, int64_t m, void *tmp, hipStream_t s, uint32_t **res_u,
                       uint32_t **res_s) {
  KeyTransform raw{0, 0, 0};
  int in_b = 0;
  hipError_t e = radix_sort_pairs(ps, pu, ps2, pu2, K, bit_length((uint32_t)(m > 0 ? m - 1 : 0)),
                                  false, raw, tmp, s, &in_b);
  if (e != hipSuccess) return e;
  uint32_t *sk = in_b ? ps2 : ps, *sv = in_b ? pu2 : pu;  // keys = s, vals = u
  uint32_t *ok = in_b ? ps : ps2, *ov = in_b ? pu : pu2;  // free pair of buffers
  e = radix_sort_pairs(sv, sk, ok, ov, K, bit_length((uint32_t)(n > 0 ? n - 1 : 0)), false, raw,
                       tmp, s, &in_b);
  if (e != hipSuccess) return e;
  *res_u = in_b ? ok : sv;
  *res_s = in_b ? ov : sk;
  return hipSuccess;
}

struct Call {
  const float *ulo, *uhi, *slo, *shi;
  int64_t n, m;
  int d, mode;    // output mode (without DDM_CLOSED)
  uint32_t closed;
  void *ws;
  Layout L;
  hipStream_t s;
  uint64_t *count_host;
  int32_t *per_update;
  int32_t *pairs;
  int64_t cap;
  Header *hdr;
  int32_t *cnt;  // per-update counts (caller's or workspace), pair/per-update modes
  // CSR output instead of the pair list (pair mode): row offsets [n + 1] and
  // subscription ids [cap], or null
  int64_t *csr_off;
  int32_t *csr_ids;
};

// CSR output of a call with no pairs: every row empty.
int csr_zero(const Call &c) {
  if (!c.csr_off) return DDM_OK;
  DDM_HIP(fill_u64(reinterpret_cast<unsigned long long *>(c.csr_off), 0ull, (size_t)c.n + 1, c.s));
  DDM_HIP(hipStreamSynchronize(c.s));
  return DDM_OK;
}

int reset_outputs(const Call &c) {
  DDM_HIP(hipMemsetAsync(c.hdr, 0, sizeof(Header), c.s));
  DDM_HIP(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(&c.hdr->kmin), 0xFFFFFFFFu, 1, c.s));
  if (c.mode != DDM_COUNT && c.n > 0)
    DDM_HIP(hipMemsetAsync(c.cnt, 0, (size_t)c.n * sizeof(int32_t), c.s));
  return DDM_OK;
}

// Pair list from per-update counts already in c.cnt and K pairs: offsets,
// the emitting sweep (``emit``), lexicographic ordering into c.pairs (or,
// for CSR output, the offsets into c.csr_off and the ordered subscription
// ids into c.csr_ids; the offsets are written even when K exceeds the
// capacity).
template <typename Emit>
int finish_pairs(const Call &c, unsigned long long K, Emit emit, bool bucketed) {
  const Layout &L = c.L;
  unsigned long long *off = c.csr_off ? reinterpret_cast<unsigned long long *>(c.csr_off)
                                      : at<unsigned long long>(c.ws, L.off);
  // offsets, and the longest row into hdr->aux[1]
  auto offsets = [&]() -> int {
    DDM_HIP(fill_u64(&c.hdr->aux[1], 0ull, 1, c.s));
    prof::mark(c.s, "pairs.scan");
    DDM_HIP(exclusive_scan_widen(reinterpret_cast<const uint32_t *>(c.cnt), (size_t)c.n, off,
                                 (size_t)c.n, at<void>(c.ws, L.scan_tmp), c.s, &c.hdr->aux[1]));
    return DDM_OK;
  };
  if (c.csr_off) {
    const int rc = offsets();
    if (rc != DDM_OK) return rc;
    DDM_HIP(fill_u64(off + c.n, K, 1, c.s));  // row_off[n] = K
    if ((int64_t)K > c.cap || K == 0) {
      prof::end(c.s);
      DDM_HIP(hipStreamSynchronize(c.s));
      prof::flush();
      return (int64_t)K > c.cap ? DDM_E_CAPACITY : DDM_OK;
    }
  }
  if ((int64_t)K > c.cap) return DDM_E_CAPACITY;
  if (K >= (1ull << 32)) return DDM_E_UNSUPPORTED;  // pair staging uses 32-bit positions
  uint32_t *cur = at<uint32_t>(c.ws, L.cur);
  uint32_t *pu = at<uint32_t>(c.ws, L.pu), *ps = at<uint32_t>(c.ws, L.ps);
  uint32_t *pu2 = at<uint32_t>(c.ws, L.pu2), *ps2 = at<uint32_t>(c.ws, L.ps2);
  if (!c.csr_off) {
    const int rc = offsets();
    if (rc != DDM_OK) return rc;
  }
  // rows of at most kRowMax pairs are ordered one by one, in LDS; otherwise
  // the pairs are sorted device-wide by (update, subscription)
  unsigned long long longest = 0;
  DDM_HIP(hipMemcpyAsync(&longest, &c.hdr->aux[1], sizeof(longest), hipMemcpyDeviceToHost, c.s));
  DDM_HIP(hipStreamSynchronize(c.s));
  const bool by_rows = longest <= kRowMax;
  uint32_t *ids_out = reinterpret_cast<uint32_t *>(c.csr_ids);
  int32_t *pairs_out = c.csr_ids ? nullptr : c.pairs;
  prof::mark(c.s, "pairs.memset");
  DDM_HIP(hipMemsetAsync(cur, 0, (size_t)c.n * sizeof(uint32_t), c.s));
  // d = 1 on the bucketed path: the emitting sweep writes whole ordered rows
  // (those of updates with no pairs in later buckets finished in place)
  bool rows_done = false;
  if (by_rows && bucketed && c.d == 1 && longest <= kRowStage) {
    uint32_t *flag = reinterpret_cast<uint32_t *>(&c.hdr->aux[2]);
    DDM_HIP(fill_u32(flag, 0u, 1, c.s));
    const RowEmit re{c.cnt, ids_out, pairs_out, flag};
    DDM_HIP(emit(off, cur, nullptr, ps, &re));
    uint32_t failed = 0;
    DDM_HIP(hipMemcpyAsync(&failed, flag, sizeof(failed), hipMemcpyDeviceToHost, c.s));
    DDM_HIP(hipStreamSynchronize(c.s));
    if (!failed) {
      launch_row_sort(off, c.cnt, ps, (uint32_t)c.n, ids_out, pairs_out, c.s,
                      at<uint32_t>(c.ws, L.own));
      rows_done = true;
    } else {  // some bucket could not: emit pair by pair from scratch
      DDM_HIP(hipMemsetAsync(cur, 0, (size_t)c.n * sizeof(uint32_t), c.s));
    }
  }
  if (rows_done) {
  } else if (by_rows) {
    DDM_HIP(emit(off, cur, nullptr, ps, nullptr));
    launch_row_sort(off, c.cnt, ps, (uint32_t)c.n, ids_out, pairs_out, c.s);
  } else {
    DDM_HIP(emit(off, cur, pu, ps, nullptr));
    uint32_t *ru = nullptr, *rs = nullptr;
    DDM_HIP(order_pairs(pu, ps, pu2, ps2, (uint32_t)K, c.n, c.m,
                        at<void>(c.ws, L.pair_sort_tmp), c.s, &ru, &rs));
    if (c.csr_ids) {
      prof::mark(c.s, "pairs.csr");
      DDM_HIP(hipMemcpyAsync(c.csr_ids, rs, (size_t)K * sizeof(uint32_t),
                             hipMemcpyDeviceToDevice, c.s));
    } else {
      launch_interleave(ru, rs, c.pairs, (size_t)K, c.s);
    }
  }
  DDM_HIP(hipGetLastError());
  prof::end(c.s);
  DDM_HIP(hipStreamSynchronize(c.s));
  prof::flush();
  return DDM_OK;
}

// ------------------------------------------------------- bucketed path
// ``replayed``: the first attempt already ran (a replayed graph) and failed
// with splittable buckets; only the split attempt is made.
int run_bucketed(const Call &c, bool replayed = false) {
  BucketArgs a{};
  a.d = c.d;
  a.ws = at<void>(c.ws, c.L.region);
  a.L = &c.L.B;
  a.hdr = c.hdr;
  a.inst_total = nullptr;
  a.zero = c.mode != DDM_COUNT && c.n > 0 ? c.cnt : nullptr;  // cleared by the count pass
  a.zero_count = (uint32_t)c.n;
  // d = 1 pairs: the count pass records each update's own-bucket pairs, so
  // that the emitting pass needs device-wide cursors only for the rest
  a.own = c.mode == DDM_PAIRS && c.d == 1 ? at<uint32_t>(c.ws, c.L.own) : nullptr;
  const int count_mode = c.mode == DDM_COUNT ? 0 : 1;
  Header h{};
  auto header = [&]() -> int {
    prof::end(c.s);
    DDM_HIP(hipMemcpyAsync(&h, c.hdr, sizeof(Header), hipMemcpyDeviceToHost, c.s));
    DDM_HIP(hipStreamSynchronize(c.s));
    prof::flush();
    return DDM_OK;
  };
  if (!replayed) {
    DDM_HIP(bucket_prepare(a, c.s));
    DDM_HIP(bucket_sweep(a, count_mode, c.cnt, nullptr, nullptr, nullptr, nullptr,
                         &c.hdr->total, c.s, nullptr, c.mode == DDM_PAIRS));
  }
  int rc = header();
  if (rc != DDM_OK) return rc;
  if (h.err) return DDM_E_INVAL;
  // buckets that held more records than a sweep workgroup can: split them
  // (their totals are known now) and count, scatter and sweep again
  BucketLayout split;
  if (h.pad[0] && h.pad[1] == kSplittable && c.L.B.nb_split > c.L.B.nb) {
    DDM_HIP(bucket_split(a, c.s));
    rc = header();
    if (rc != DDM_OK) return rc;
    if (h.split_nb == 0) return kFallback;
    split = split_layout(c.L.B, h.split_nb);
    a.L = &split;
    DDM_HIP(bucket_prepare_split(a, c.s));
    DDM_HIP(bucket_sweep(a, count_mode, c.cnt, nullptr, nullptr, nullptr, nullptr,
                         &c.hdr->total, c.s, nullptr, c.mode == DDM_PAIRS));
    rc = header();
    if (rc != DDM_OK) return rc;
  }
  if (h.pad[0]) return kFallback;
  *c.count_host = h.total;
  if (c.mode != DDM_PAIRS || (h.total == 0 && !c.csr_off)) return DDM_OK;
  return finish_pairs(
      c, h.total,
      [&](unsigned long long *off, uint32_t *cur, uint32_t *pu, uint32_t *ps, const RowEmit *rows) {
        BucketArgs e = a;
        if (rows) e.rows = *rows;
        return bucket_sweep(e, 2, nullptr, off, cur, pu, ps, &c.hdr->aux[0], c.s);
      },
      true);
}

// ---------------------------------------------------- device-wide path
int run_global(const Call &c) {
  const Layout &L = c.L;
  const uint32_t un = (uint32_t)c.n, um = (uint32_t)c.m, N = un + um;
  void *R = at<void>(c.ws, L.region);
  int rc = reset_outputs(c);
  if (rc != DDM_OK) return rc;

  // 1. validate, encode, empties
  uint32_t *klo = at<uint32_t>(R, L.klo);
  uint32_t *khi = at<uint32_t>(R, L.khi);
  const int axis = 0;
  launch_keys(c.ulo, c.uhi, un, c.slo, c.shi, um, c.d, axis, c.closed, klo, khi,
              at<uint4>(c.ws, L.partial), c.hdr, c.s);
  DDM_HIP(hipGetLastError());
  Header h{};
  prof::end(c.s);
  DDM_HIP(hipMemcpyAsync(&h, c.hdr, sizeof(Header), hipMemcpyDeviceToHost, c.s));
  DDM_HIP(hipStreamSynchronize(c.s));
  prof::flush();
  if (h.err) return DDM_E_INVAL;
  const uint32_t nne = h.nonempty;
  if (nne == 0 || c.n == 0 || c.m == 0) return csr_zero(c);  // counts already zeroed

  // 2. radix sort of the lower keys (range-reduced; empties last)
  const bool has_empty = nne < N;
  const uint32_t range = h.kmax - h.kmin;
  KeyTransform xf{1u, h.kmin, range + 1u};
  const int bits = bit_length(has_empty ? range + 1u : range);
  uint32_t *vals_a = at<uint32_t>(R, L.vals_a);
  uint32_t *keys_b = at<uint32_t>(R, L.keys_b);
  uint32_t *vals_b = at<uint32_t>(R, L.vals_b);
  int in_b = 0;
  DDM_HIP(radix_sort_pairs(klo, vals_a, keys_b, vals_b, N, bits, true, xf,
                           at<void>(R, L.sort_tmp), c.s, &in_b));
  const uint32_t *skey = in_b ? keys_b : klo;
  const uint32_t *sidx = in_b ? vals_b : vals_a;

  // 3. other axes in sorted order
  uint32_t *s_khi = at<uint32_t>(R, L.s_khi);
  float *s_other = at<float>(R, L.s_other);
  launch_gather(sidx, nne, khi, c.ulo, c.uhi, un, c.slo, c.shi, c.d, axis, s_khi, s_other, N, c.s);
  DDM_HIP(hipGetLastError());

  // 4. the sweep
  SweepArgs a{};
  a.skey = skey;
  a.sidx = sidx;
  a.s_khi = s_khi;
  a.s_other = s_other;
  a.stride = N;
  a.count = nne;
  a.n = un;
  a.dm1 = c.d - 1;
  a.closed = c.closed;
  a.per_update = c.cnt;
  a.total = &c.hdr->total;
  launch_sweep(c.mode != DDM_COUNT ? 1 : 0, a, c.s);
  DDM_HIP(hipGetLastError());
  unsigned long long K = 0;
  prof::end(c.s);
  DDM_HIP(hipMemcpyAsync(&K, &c.hdr->total, sizeof(K), hipMemcpyDeviceToHost, c.s));
  DDM_HIP(hipStreamSynchronize(c.s));
  prof::flush();
  *c.count_host = K;
  if (c.mode != DDM_PAIRS || (K == 0 && !c.csr_off)) return DDM_OK;
  return finish_pairs(c, K, [&](unsigned long long *off, uint32_t *cur, uint32_t *pu,
                                uint32_t *ps, const RowEmit *) {
    SweepArgs e = a;
    e.offsets = off;
    e.cursor = cur;
    e.out_u = pu;
    e.out_s = ps;
    e.total = &c.hdr->aux[0];
    launch_sweep(2, e, c.s);
    return hipGetLastError();
  }, false);
}

// ------------------------------------------------- repeated single calls
//
// A count or per-update call on the bucketed path needs no host decision
// between its launches, so when the same call (same pointers, sizes, mode and
// workspace) comes again, its launches are captured once into a HIP graph and
// replayed by one launch; the header reaches the host through page-locked
// memory.  Captured on the second sighting of a call, so one-off calls pay
// nothing; a small LRU bounds the cache.  Profiling, pair mode and forced
// device-wide calls run eagerly.
struct GraphKey {
  const float *ulo, *uhi, *slo, *shi;
  int64_t n, m;
  int d, mode;
  void *ws;
  size_t ws_bytes;
  int32_t *per_update;
  int axis;  // the swept-axis setting the launches were captured under
  bool same(const GraphKey &o) const {
    return ulo == o.ulo && uhi == o.uhi && slo == o.slo && shi == o.shi && n == o.n &&
           m == o.m && d == o.d && mode == o.mode && ws == o.ws && ws_bytes == o.ws_bytes &&
           per_update == o.per_update && axis == o.axis;
  }
};

struct CachedGraph {
  GraphKey key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  Header *hdr_host = nullptr;  // page-locked
  uint64_t used = 0;
  bool captured = false, failed = false;
};

constexpr size_t kGraphCache = 64;
std::mutex g_graph_mu;
std::vector<CachedGraph> g_graphs;
uint64_t g_graph_tick = 0;

void release(CachedGraph &e) {
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.graph) (void)hipGraphDestroy(e.graph);
  if (e.hdr_host) (void)hipHostFree(e.hdr_host);
  e.exec = nullptr;
  e.graph = nullptr;
  e.hdr_host = nullptr;
  e.captured = false;
}

// Captures the bucketed count / per-update launches of call c.
bool capture(CachedGraph &e, const Call &c) {
  if (hipHostMalloc(reinterpret_cast<void **>(&e.hdr_host), sizeof(Header), hipHostMallocDefault) !=
      hipSuccess)
    return false;
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return false;
  BucketArgs a{};
  a.d = c.d;
  a.ws = at<void>(c.ws, c.L.region);
  a.L = &c.L.B;
  a.hdr = c.hdr;
  a.zero = c.mode != DDM_COUNT && c.n > 0 ? c.cnt : nullptr;
  a.zero_count = (uint32_t)c.n;
  bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    bool enq = bucket_prepare(a, cs) == hipSuccess;
    enq = enq && bucket_sweep(a, c.mode == DDM_COUNT ? 0 : 1, c.cnt, nullptr, nullptr, nullptr,
                              nullptr, &c.hdr->total, cs) == hipSuccess;
    enq = enq && hipMemcpyAsync(e.hdr_host, c.hdr, sizeof(Header), hipMemcpyDeviceToHost, cs) ==
                     hipSuccess;
    hipGraph_t g = nullptr;
    ok = hipStreamEndCapture(cs, &g) == hipSuccess && enq;
    e.graph = g;
    ok = ok && hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0) == hipSuccess;
  }
  (void)hipStreamDestroy(cs);
  e.captured = ok;
  return ok;
}

// Replays a captured call: DDM_OK, DDM_E_INVAL, DDM_E_DEVICE or kFallback.
int replay(const CachedGraph &e, hipStream_t s, uint64_t *count_host) {
  DDM_HIP(hipGraphLaunch(e.exec, s));
  DDM_HIP(hipStreamSynchronize(s));
  Header h;
  memcpy(&h, e.hdr_host, sizeof(Header));  // written by the graph's copy, complete after the sync
  if (h.err) return DDM_E_INVAL;
  if (h.pad[0]) return h.pad[1] == kSplittable ? kSplit : kFallback;
  *count_host = h.total;
  return DDM_OK;
}

}  // namespace
}  // namespace ddm

using namespace ddm;

extern "C" size_t ddm_workspace_bytes(int64_t n, int64_t m, int d, int mode,
                                      int64_t pair_capacity) {
  int out;
  bool closed;
  if (!split_mode(mode, &out, &closed)) return 0;
  if (!sizes_ok(n, m, d, out) || pair_capacity < 0) return 0;
  return make_layout(n, m, d, out, pair_capacity).total;
}

extern "C" const char *ddm_strerror(int code) {
  switch (code) {
    case DDM_OK: return "success";
    case DDM_E_INVAL: return "invalid argument or input (NaN coordinate, lo > hi, bad size or pointer)";
    case DDM_E_CAPACITY: return "pair buffer too small (count_host holds the number of pairs)";
    case DDM_E_WORKSPACE: return "workspace smaller than ddm_workspace_bytes()";
    case DDM_E_DEVICE: return "HIP runtime error";
    case DDM_E_UNSUPPORTED: return "request outside the supported range";
    case DDM_E_SCRATCH:
      return "request needs more than the static scratch array of ddm_match_noalloc() holds";
    default: return "unknown error";
  }
}

extern "C" int ddm_set_path(int path) {
  if (path != DDM_PATH_AUTO && path != DDM_PATH_BUCKETED && path != DDM_PATH_GLOBAL)
    return DDM_E_INVAL;
  g_path_request.store(path, std::memory_order_relaxed);
  return DDM_OK;
}

extern "C" int ddm_last_path(void) { return t_last_path; }

extern "C" int ddm_set_sweep_axis(int axis) {
  if (axis < -1 || axis >= DDM_MAX_DIMS) return DDM_E_INVAL;
  set_sweep_axis(axis);
  return DDM_OK;
}

namespace {

// ddm_match and ddm_match_csr: the pair list goes to ``pairs``, or, with
// csr_off given, CSR rows to csr_off / csr_ids.
// ``cached``: repeated count / per-update calls may be captured into a graph
// (which allocates the graph and a page-locked header); false runs eagerly.
int match_entry(const float *upd_lo, const float *upd_hi, int64_t n, const float *sub_lo,
                const float *sub_hi, int64_t m, int d, int mode, void *workspace, size_t ws_bytes,
                void *stream, uint64_t *count_host, int32_t *per_update, int32_t *pairs,
                int64_t pair_capacity, int64_t *csr_off, int32_t *csr_ids, bool cached = true,
                bool record = true) {
  int last_path = 0;
  struct Record {  // reports the path on every return of a recorded call
    bool on;
    int &path;
    ~Record() {
      if (on) t_last_path = path;
    }
  } report{record, last_path};
  const int path_request = g_path_request.load(std::memory_order_relaxed);
  // host-side checks: nothing is launched when one fails
  const int mode_arg = mode;  // with the interval flag (the graph cache key)
  bool closed;
  if (!split_mode(mode_arg, &mode, &closed)) return DDM_E_INVAL;
  if (!sizes_ok(n, m, d, mode) || !count_host || pair_capacity < 0) return DDM_E_INVAL;
  if ((n > 0 && (!upd_lo || !upd_hi)) || (m > 0 && (!sub_lo || !sub_hi))) return DDM_E_INVAL;
  if (mode == DDM_PER_UPDATE && n > 0 && !per_update) return DDM_E_INVAL;
  if (mode == DDM_PAIRS && pair_capacity > 0 && !(csr_off ? csr_ids : pairs)) return DDM_E_INVAL;
  const bool graphable = cached && mode != DDM_PAIRS && n + m > 0 && !prof::enabled() &&
                         path_request != DDM_PATH_GLOBAL && workspace &&
                         !(reinterpret_cast<uintptr_t>(workspace) & 255);
  const GraphKey key{upd_lo, upd_hi, sub_lo, sub_hi, n, m, d, mode_arg, workspace, ws_bytes,
                     mode == DDM_COUNT ? nullptr : per_update, sweep_axis()};
  std::unique_lock<std::mutex> cache_lock(g_graph_mu, std::defer_lock);
  CachedGraph *entry = nullptr;
  bool global_only = false, replayed = false;
  if (graphable) {
    cache_lock.lock();
    for (CachedGraph &e : g_graphs)
      if (e.key.same(key)) entry = &e;
    if (entry && entry->captured) {
      entry->used = ++g_graph_tick;
      *count_host = 0;
      const int rc = replay(*entry, static_cast<hipStream_t>(stream), count_host);
      if (rc != kFallback && rc != kSplit) {
        last_path = rc == DDM_OK ? DDM_PATH_BUCKETED : 0;
        return rc;
      }
      entry = nullptr;
      // the replay made the first bucketed attempt: split its buckets below,
      // or go to the device-wide path
      replayed = rc == kSplit;
      global_only = !replayed;
      if (global_only && path_request == DDM_PATH_BUCKETED) return DDM_E_UNSUPPORTED;
    } else if (!entry) {  // first sighting: remember the call, run it eagerly
      if (g_graphs.size() >= kGraphCache) {
        size_t old = 0;
        for (size_t i = 1; i < g_graphs.size(); ++i)
          if (g_graphs[i].used < g_graphs[old].used) old = i;
        release(g_graphs[old]);
        g_graphs.erase(g_graphs.begin() + (std::ptrdiff_t)old);
      }
      g_graphs.push_back(CachedGraph{});
      g_graphs.back().key = key;
      g_graphs.back().used = ++g_graph_tick;
    } else if (entry->failed) {
      entry = nullptr;
    }
    // else: second sighting, captured below once the call is laid out
    if (!entry) cache_lock.unlock();  // an eager call needs no cache entry
  }
  Call c{};
  c.L = make_layout(n, m, d, mode, pair_capacity, upd_lo, upd_hi, sub_lo, sub_hi, closed);
  if (!workspace || ws_bytes < c.L.total) return DDM_E_WORKSPACE;
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return DDM_E_INVAL;
  *count_host = 0;
  c.ulo = upd_lo;
  c.uhi = upd_hi;
  c.slo = sub_lo;
  c.shi = sub_hi;
  c.n = n;
  c.m = m;
  c.d = d;
  c.mode = mode;
  c.closed = closed ? 1u : 0u;
  c.ws = workspace;
  c.s = static_cast<hipStream_t>(stream);
  c.count_host = count_host;
  c.per_update = per_update;
  c.pairs = pairs;
  c.cap = pair_capacity;
  c.hdr = at<Header>(workspace, c.L.hdr);
  c.cnt = mode == DDM_PAIRS ? (per_update ? per_update : at<int32_t>(workspace, c.L.cnt))
                            : per_update;
  c.csr_off = csr_off;
  c.csr_ids = csr_ids;
  last_path = 0;
  if (n + m == 0) {
    int rc = reset_outputs(c);
    if (rc == DDM_OK && hipStreamSynchronize(c.s) != hipSuccess) return DDM_E_DEVICE;
    if (rc == DDM_OK) rc = csr_zero(c);
    return rc;
  }
  if (path_request == DDM_PATH_BUCKETED && !c.L.bucket_ok) return DDM_E_UNSUPPORTED;
  int rc;
  if (entry && c.L.bucket_ok) {  // second sighting of a repeated call: capture and replay
    entry->used = ++g_graph_tick;
    if (capture(*entry, c)) {
      rc = replay(*entry, c.s, count_host);
      if (rc != kFallback && rc != kSplit) {
        if (rc == DDM_OK) last_path = DDM_PATH_BUCKETED;
        return rc;
      }
      if (rc == kSplit) {
        rc = run_bucketed(c, true);
        if (rc != kFallback) {
          if (rc == DDM_OK) last_path = DDM_PATH_BUCKETED;
          return rc;
        }
      }
      if (path_request == DDM_PATH_BUCKETED) return DDM_E_UNSUPPORTED;
      rc = run_global(c);
      if (rc == DDM_OK || rc == DDM_E_CAPACITY) last_path = DDM_PATH_GLOBAL;
      return rc;
    }
    release(*entry);
    entry->failed = true;  // run eagerly from now on
    (void)hipGetLastError();
  }
  if (path_request != DDM_PATH_GLOBAL && c.L.bucket_ok && !global_only) {
    rc = run_bucketed(c, replayed);
    if (rc != kFallback) {
      if (rc == DDM_OK || rc == DDM_E_CAPACITY) last_path = DDM_PATH_BUCKETED;
      return rc;
    }
    if (path_request == DDM_PATH_BUCKETED) return DDM_E_UNSUPPORTED;
  }
  rc = run_global(c);
  if (rc == DDM_OK || rc == DDM_E_CAPACITY) last_path = DDM_PATH_GLOBAL;
  return rc;
}

}  // namespace

namespace ddm {
int match_quiet(const float *upd_lo, const float *upd_hi, int64_t n, const float *sub_lo,
                const float *sub_hi, int64_t m, int d, int mode, void *workspace, size_t ws_bytes,
                void *stream, uint64_t *count_host, int32_t *per_update, int32_t *pairs,
                int64_t pair_capacity) {
  return match_entry(upd_lo, upd_hi, n, sub_lo, sub_hi, m, d, mode, workspace, ws_bytes, stream,
                     count_host, per_update, pairs, pair_capacity, nullptr, nullptr, true, false);
}
}  // namespace ddm

extern "C" int ddm_match(const float *upd_lo, const float *upd_hi, int64_t n, const float *sub_lo,
                         const float *sub_hi, int64_t m, int d, int mode, void *workspace,
                         size_t ws_bytes, void *stream, uint64_t *count_host, int32_t *per_update,
                         int32_t *pairs, int64_t pair_capacity) {
  return match_entry(upd_lo, upd_hi, n, sub_lo, sub_hi, m, d, mode, workspace, ws_bytes, stream,
                     count_host, per_update, pairs, pair_capacity, nullptr, nullptr);
}

extern "C" int ddm_match_csr(const float *upd_lo, const float *upd_hi, int64_t n,
                             const float *sub_lo, const float *sub_hi, int64_t m, int d, int flags,
                             void *workspace, size_t ws_bytes, void *stream, uint64_t *count_host,
                             int64_t *row_off, int32_t *sub_ids, int64_t capacity) {
  if ((flags & ~DDM_CLOSED) != 0 || !row_off) return DDM_E_INVAL;
  return match_entry(upd_lo, upd_hi, n, sub_lo, sub_hi, m, d, DDM_PAIRS | flags, workspace,
                     ws_bytes, stream, count_host, nullptr, nullptr, capacity, row_off, sub_ids);
}

// ------------------------------------------------- no-allocation variant
//
// ddm_match() with the workspace taken from a file-scope device array
// instead of the caller: for callers that cannot allocate device memory.
// The array's name is a host-side stand-in in host code; its device address
// is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that address is ever passed to kernels or copies.
namespace {

__device__ __align__(256) unsigned char scratch[DDM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

struct ScratchSlot {
  std::mutex mu;        // held for a whole call: calls on one device take turns
  void *ptr = nullptr;  // device address of this device's copy of `scratch`
};
ScratchSlot g_scratch[kMaxDevices];

}  // namespace

extern "C" int ddm_match_noalloc(const float *upd_lo, const float *upd_hi, int64_t n,
                                 const float *sub_lo, const float *sub_hi, int64_t m, int d,
                                 int mode, void *stream, uint64_t *count_host,
                                 int32_t *per_update, int32_t *pairs, int64_t pair_capacity) {
  // the size check needs no device: requests beyond the array are refused
  // before anything touches the GPU
  int out;
  bool closed;
  if (!split_mode(mode, &out, &closed)) return DDM_E_INVAL;
  if (!sizes_ok(n, m, d, out) || !count_host || pair_capacity < 0) return DDM_E_INVAL;
  if (make_layout(n, m, d, out, pair_capacity).total > DDM_NOALLOC_SCRATCH_BYTES)
    return DDM_E_SCRATCH;
  if (prof::enabled()) return DDM_E_UNSUPPORTED;  // the recorder creates events
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return DDM_E_DEVICE;
  if (dev < 0 || dev >= kMaxDevices) return DDM_E_UNSUPPORTED;
  ScratchSlot &slot = g_scratch[dev];
  std::lock_guard<std::mutex> hold(slot.mu);
  if (!slot.ptr) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DDM_E_DEVICE;
    slot.ptr = p;
  }
  const int rc = match_entry(upd_lo, upd_hi, n, sub_lo, sub_hi, m, d, mode, slot.ptr,
                             DDM_NOALLOC_SCRATCH_BYTES, stream, count_host, per_update, pairs,
                             pair_capacity, nullptr, nullptr, false);
  // every path has synchronised before it returns a result; an early error
  // may not have, and the next call must not overlap this one's kernels
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return DDM_E_DEVICE;
  return rc;
}

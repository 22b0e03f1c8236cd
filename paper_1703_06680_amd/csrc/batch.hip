// Batched matching and its captured-graph form (declared in include/ddm.h).
//
// A batch of B independent instances, stored back to back, runs through one
// launch sequence of the bucketed path: every kernel covers the blocks,
// buckets and pairs of all instances at once, so the per-launch cost is paid
// once per batch instead of once per instance.  The sequence needs no host
// round trip once the batch plan is on the device: outputs are cleared by
// fill kernels, the pair count is compared with the capacity on the device
// (the emitting sweep and the ordering sorts read the outcome from device
// memory), so the whole sequence can be recorded into a HIP graph and
// replayed by one launch.
//
// Pairs are produced as in a single call: per-update counts, an exclusive
// scan into per-update slots (the first pass of a two-pass compaction), an
// emitting sweep that writes each update's subscriptions into its row, and
// one wave per row that orders the row in LDS and writes it as
// instance-local (update, subscription) ids; each instance's first pair is
// the slot of its first update.  A row longer than the row sort holds sets
// a flag, and the batch is then finished instance by instance.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/ddm.h"
#include "internal.h"
#include "batch.h"
#include "bucket_path.h"
#include "common.h"
#include "match_global.h"
#include "primitives.h"
#include "profile.h"

namespace ddm {
namespace {

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <typename T>
T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

#define DDM_HIP(call)                              \
  do {                                             \
    if ((call) != hipSuccess) return DDM_E_DEVICE; \
  } while (0)

// ------------------------------------------------------------- kernels

// After the scan off[n_total] is the number of pairs K.  gate[0] = K if the
// pairs fit the capacity, else 0 (nothing is emitted); gate[1] = 1 if they do
// not fit; gate[2] = 0, set to 1 by the row sort if a row is longer than it
// holds.  pair_off[b] = off[first update row of instance b].
__global__ void bt_gate_kernel(const unsigned long long *__restrict__ off, uint32_t n_total,
                               uint64_t cap, const uint32_t *__restrict__ uoff, uint32_t B,
                               int64_t *__restrict__ pair_off, uint32_t *__restrict__ gate) {
  const unsigned long long K = off[n_total];
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b <= B; b += gridDim.x * blockDim.x)
    pair_off[b] = (int64_t)off[uoff[b]];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    gate[0] = K <= cap ? (uint32_t)K : 0u;
    gate[1] = K > cap ? 1u : 0u;
    gate[2] = 0u;
  }
}

// Instance of an update row: the last b < B with uoff[b] <= row (that
// instance is non-empty and holds the row).
__device__ __forceinline__ uint32_t instance_of_row(const uint32_t *__restrict__ uoff, uint32_t B,
                                                    uint32_t row) {
  uint32_t lo = 0, hi = B;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (uoff[mid] <= row)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Orders every row of the emitted pairs: row u (an update row of the
// concatenated arrays) holds the cnt[u] subscription rows it meets at
// in[off[u] ..), in the order the sweep found them.  One wave per row stages
// it in LDS as instance-local subscription ids and writes the pairs
// (instance-local update id, subscription id) in order at pairs[off[u] ..):
// up to 128 ids sorted across the wave in registers, longer rows by ranks
// (ids in a row are distinct).  A row longer than kRowMax is left and sets
// gate[2]; nothing runs if the pairs did not fit (gate[0] == 0).
constexpr int kBtRowThreads = 512;
constexpr int kBtRowWaves = kBtRowThreads / kWave;

__global__ __launch_bounds__(kBtRowThreads) void bt_row_sort_kernel(
    const unsigned long long *__restrict__ off, const int32_t *__restrict__ cnt,
    const uint32_t *__restrict__ in, uint32_t n, const uint32_t *__restrict__ uoff,
    const uint32_t *__restrict__ soff, uint32_t B, uint32_t *__restrict__ gate,
    int2 *__restrict__ pairs) {
  __shared__ __align__(16) uint32_t stage[kBtRowWaves][kRowMax];
  if (gate[0] == 0u) return;  // uniform: no pairs, or they did not fit
  const int w = threadIdx.x / kWave, lane = lane_id();
  uint32_t *row = stage[w];
  // each wave takes kGroups groups of 64 consecutive rows at a time (their
  // counts loaded together: most rows of a sparse output are empty), finds
  // with one ballot per group the rows with work and orders those one after
  // the other
  constexpr uint32_t kGroups = 4;
  const uint32_t step = gridDim.x * kBtRowWaves * kWave;
  for (uint32_t g0 = (blockIdx.x * kBtRowWaves + w) * kWave; g0 < n; g0 += kGroups * step) {
    uint32_t cg[kGroups];
#pragma unroll
    for (uint32_t k = 0; k < kGroups; ++k) {
      const uint32_t mine = g0 + k * step + (uint32_t)lane;
      cg[k] = mine < n ? (uint32_t)cnt[mine] : 0u;
    }
#pragma unroll
    for (uint32_t k = 0; k < kGroups; ++k) {
      const uint32_t u0 = g0 + k * step;
      const uint32_t c = cg[k];
      if (c > kRowMax) gate[2] = 1u;
      uint64_t todo = __ballot(c != 0u && c <= kRowMax);
      while (todo) {
        const uint32_t u = u0 + (uint32_t)(__ffsll((unsigned long long)todo) - 1);
        todo &= todo - 1;
        const uint32_t L = (uint32_t)cnt[u];
        const unsigned long long base = off[u];
        const uint32_t b = instance_of_row(uoff, B, u);
        const uint32_t ul = u - uoff[b], s0 = soff[b];
        const uint32_t L4 = (L + 3) & ~3u;  // padded with ids above every real one
        for (uint32_t i = lane; i < L4; i += kWave) row[i] = i < L ? in[base + i] - s0 : 0xFFFFFFFFu;
        __builtin_amdgcn_wave_barrier();
        if (L <= kWave)
          sort_row<1>(row, L, lane, ul, base, nullptr, pairs);
        else if (L <= 2 * kWave)
          sort_row<2>(row, L, lane, ul, base, nullptr, pairs);
        else
          for (uint32_t i0 = 0; i0 < L; i0 += 4 * kWave)
            rank_row<4>(row, L, L4, i0, lane, ul, base, nullptr, pairs);
        __builtin_amdgcn_wave_barrier();  // every lane done with the row before the next one
      }
    }
  }
}

unsigned grid_for(size_t count) {
  return (unsigned)std::max<size_t>(1, std::min<size_t>((count + 255) / 256, 2048));
}

// ------------------------------------------------------------- host side

BucketTuning to_tuning(const ddm_tuning *t) {
  BucketTuning b;
  if (t) {
    b.target = (uint32_t)t->target;
    b.sweep_threads = (uint32_t)t->sweep_threads;
    b.groups_per_thread = (uint32_t)t->groups_per_thread;
    b.max_blocks = (uint32_t)t->max_blocks;
  }
  return b;
}

bool tuning_valid(const ddm_tuning *t) {
  if (!t) return true;
  const bool big = t->sweep_threads == 1024;
  return t->target >= 64 && t->target <= (int32_t)((big ? kBigBucketCap : kBucketCap) * 3 / 4) &&
         (t->sweep_threads == 256 || t->sweep_threads == 512 || big) &&
         t->groups_per_thread >= 1 &&
         t->groups_per_thread <= 64 && t->max_blocks >= 1 && t->max_blocks <= 65536;
}

// The autotuner's candidates (the default is among them).
std::vector<BucketTuning> candidates() {
  std::vector<BucketTuning> out;
  for (uint32_t target : {768u, 1024u, 1536u})
    for (uint32_t threads : {256u, 512u})
      for (uint32_t gpt : {1u, 4u}) {
        BucketTuning t;
        t.target = target;
        t.sweep_threads = threads;
        t.groups_per_thread = gpt;
        out.push_back(t);
      }
  return out;
}

// The output mode of a mode argument (without the interval flag).
inline int out_mode(int mode) { return mode & ~DDM_CLOSED; }

bool mode_ok(int mode) {
  const int o = out_mode(mode);
  return o == DDM_COUNT || o == DDM_PER_UPDATE || o == DDM_PAIRS;
}

bool shape_ok(const int64_t *uoff, const int64_t *soff, int64_t B, int d, int mode,
              int64_t cap) {
  if (!uoff || !soff || B < 1 || B >= (int64_t(1) << 24)) return false;
  if (d < 1 || d > DDM_MAX_DIMS) return false;
  if (!mode_ok(mode)) return false;
  if (cap < 0 || cap >= (int64_t(1) << 31)) return false;
  if (uoff[0] != 0 || soff[0] != 0) return false;
  for (int64_t b = 0; b < B; ++b)
    if (uoff[b + 1] < uoff[b] || soff[b + 1] < soff[b]) return false;
  return uoff[B] + soff[B] < (int64_t(1) << 31);
}

BatchLayout batch_layout(const InstSpec *spec, int64_t B, int d, int mode, int64_t cap,
                         const BucketTuning &t) {
  mode = out_mode(mode);
  BatchLayout L{};
  size_t at_ = 0;
  auto take = [&](size_t bytes) {
    size_t o = at_;
    at_ += align256(bytes);
    return o;
  };
  size_t n_total = 0;
  for (int64_t b = 0; b < B; ++b) n_total += (size_t)spec[b].n;
  const size_t c = (size_t)cap;
  L.hdr = take(sizeof(Header));
  L.offs = take(2 * ((size_t)B + 1) * sizeof(uint32_t));
  L.gate = take(4 * sizeof(uint32_t));
  if (mode != DDM_COUNT) L.cnt = take(n_total * sizeof(int32_t));
  if (mode == DDM_PAIRS) {
    L.off = take((n_total + 1) * sizeof(unsigned long long));
    L.cur = take(n_total * sizeof(uint32_t));
    L.ps = take(c * sizeof(uint32_t));
    L.scan_tmp = take(scan_temp_bytes(n_total + 1));
  }
  L.region = at_;
  L.bk = bucket_layout(spec, B, d, t);
  L.total = L.region + align256(L.bk.bytes);
  return L;
}

// What the per-instance fallback needs: the largest single-call workspace.
size_t fallback_bytes(const InstSpec *spec, int64_t B, int d, int mode, int64_t cap) {
  size_t most = 0;
  for (int64_t b = 0; b < B; ++b)
    most = std::max(most, ddm_workspace_bytes(spec[b].n, spec[b].m, d, mode, cap));
  return most;
}

// Instances of a CSR batch (pointers into the shared arrays; null pointers
// when only the sizes matter).
std::vector<InstSpec> csr_specs(const float *ulo, const float *uhi, const int64_t *uoff,
                                const float *slo, const float *shi, const int64_t *soff,
                                int64_t B, int d) {
  std::vector<InstSpec> v((size_t)B);
  for (int64_t b = 0; b < B; ++b) {
    InstSpec &x = v[(size_t)b];
    x.n = uoff[b + 1] - uoff[b];
    x.m = soff[b + 1] - soff[b];
    x.ulo = ulo ? ulo + uoff[b] * d : nullptr;
    x.uhi = uhi ? uhi + uoff[b] * d : nullptr;
    x.slo = slo ? slo + soff[b] * d : nullptr;
    x.shi = shi ? shi + soff[b] * d : nullptr;
  }
  return v;
}

bool specs_ok(const InstSpec *spec, int64_t B, int d, int mode, int64_t cap) {
  if (!spec || B < 1 || B >= (int64_t(1) << 24)) return false;
  if (d < 1 || d > DDM_MAX_DIMS) return false;
  if (!mode_ok(mode)) return false;
  if (cap < 0 || cap >= (int64_t(1) << 31)) return false;
  int64_t N = 0;
  for (int64_t b = 0; b < B; ++b) {
    if (spec[b].n < 0 || spec[b].m < 0) return false;
    N += spec[b].n + spec[b].m;
    if (N >= (int64_t(1) << 31)) return false;
  }
  return true;
}

}  // namespace

// Validates a batch given as instances and fills c (no device work).
int make_batch(Batch &c, std::vector<InstSpec> spec, int d, int mode, void *ws, size_t ws_bytes,
               const ddm_tuning *tuning, uint64_t *counts, int32_t *per_update, int32_t *pairs,
               int64_t *pair_off, int64_t cap) {
  const int64_t B = (int64_t)spec.size();
  if (!specs_ok(spec.data(), B, d, mode, cap) || !tuning_valid(tuning)) return DDM_E_INVAL;
  const uint32_t closed = (mode & DDM_CLOSED) ? 1u : 0u;
  mode = out_mode(mode);
  int64_t n_total = 0;
  for (InstSpec &x : spec) {
    x.closed = closed;
    if ((x.n > 0 && (!x.ulo || !x.uhi)) || (x.m > 0 && (!x.slo || !x.shi))) return DDM_E_INVAL;
    n_total += x.n;
  }
  if (!counts) return DDM_E_INVAL;
  if (mode == DDM_PER_UPDATE && n_total > 0 && !per_update) return DDM_E_INVAL;
  if (mode == DDM_PAIRS && (!pair_off || (cap > 0 && !pairs))) return DDM_E_INVAL;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return ws ? DDM_E_INVAL : DDM_E_WORKSPACE;
  c.spec = std::move(spec);
  c.uoff.assign((size_t)B + 1, 0);
  c.soff.assign((size_t)B + 1, 0);
  for (int64_t b = 0; b < B; ++b) {
    c.uoff[(size_t)b + 1] = c.uoff[(size_t)b] + c.spec[(size_t)b].n;
    c.soff[(size_t)b + 1] = c.soff[(size_t)b] + c.spec[(size_t)b].m;
  }
  c.B = B;
  c.d = d;
  c.mode = mode;
  c.closed = closed;
  c.ws = ws;
  c.ws_bytes = ws_bytes;
  c.counts = counts;
  c.per_update = per_update;
  c.pairs = pairs;
  c.pair_off = pair_off;
  c.cap = cap;
  const BucketTuning t = to_tuning(tuning);
  c.bucketed = bucket_path_supported(d, c.spec.data(), B, t);
  if (c.bucketed) {
    c.L = batch_layout(c.spec.data(), B, d, mode, cap, t);
    if (ws_bytes < c.L.total) return DDM_E_WORKSPACE;
  }
  if (ws_bytes < fallback_bytes(c.spec.data(), B, d, c.match_mode(), cap)) return DDM_E_WORKSPACE;
  return DDM_OK;
}

int make_batch_csr(Batch &c, const float *ulo, const float *uhi, const int64_t *uoff,
                   const float *slo, const float *shi, const int64_t *soff, int64_t B, int d,
                   int mode, void *ws, size_t ws_bytes, const ddm_tuning *tuning, uint64_t *counts,
                   int32_t *per_update, int32_t *pairs, int64_t *pair_off, int64_t cap) {
  if (!shape_ok(uoff, soff, B, d, mode, cap)) return DDM_E_INVAL;
  return make_batch(c, csr_specs(ulo, uhi, uoff, slo, shi, soff, B, d), d, mode, ws, ws_bytes,
                    tuning, counts, per_update, pairs, pair_off, cap);
}

size_t workspace_for(const std::vector<InstSpec> &spec, int d, int mode, int64_t pair_capacity,
                          const ddm_tuning *tuning) {
  const int64_t B = (int64_t)spec.size();
  size_t most = fallback_bytes(spec.data(), B, d, mode, pair_capacity);
  std::vector<BucketTuning> ts;
  if (tuning) {
    ts.push_back(to_tuning(tuning));
  } else {
    ts = candidates();
    ts.push_back(BucketTuning{});
  }
  for (const BucketTuning &t : ts)
    if (bucket_path_supported(d, spec.data(), B, t))
      most = std::max(most, batch_layout(spec.data(), B, d, mode, pair_capacity, t).total);
  return std::max<size_t>(most, 256);
}

namespace {

BucketArgs bucket_args(const Batch &c) {
  BucketArgs a{};
  a.d = c.d;
  a.ws = at<void>(c.ws, c.L.region);
  a.L = &c.L.bk;
  a.hdr = at<Header>(c.ws, c.L.hdr);
  a.inst_total = reinterpret_cast<unsigned long long *>(c.counts);
  return a;
}

// Host-to-device copies of the 32-bit instance offsets and of the plan.
// With ``pinned`` (page-locked, batch_staging_bytes() bytes) the copies do
// not block the host; otherwise ``staging`` holds the offsets and must stay
// alive until the stream has passed the copies.
int upload(const Batch &c, hipStream_t s, std::vector<uint32_t> &staging, void *pinned) {
  const size_t words = 2 * ((size_t)c.B + 1);
  uint32_t *offs;
  if (pinned) {
    offs = static_cast<uint32_t *>(pinned);
  } else {
    staging.resize(words);
    offs = staging.data();
  }
  for (int64_t b = 0; b <= c.B; ++b) {
    offs[(size_t)b] = (uint32_t)c.uoff[(size_t)b];
    offs[(size_t)c.B + 1 + (size_t)b] = (uint32_t)c.soff[(size_t)b];
  }
  DDM_HIP(hipMemcpyAsync(at<void>(c.ws, c.L.offs), offs, words * sizeof(uint32_t),
                         hipMemcpyHostToDevice, s));
  void *plan_stage = pinned ? static_cast<char *>(pinned) + align256(words * sizeof(uint32_t))
                            : nullptr;
  DDM_HIP(bucket_upload_plan(bucket_args(c), s, plan_stage));
  return DDM_OK;
}

// Every launch of one batched call, device-driven (capturable).
int enqueue(const Batch &c, hipStream_t s) {
  const BatchLayout &L = c.L;
  const uint32_t n_total = (uint32_t)c.uoff[(size_t)c.B];
  Header *hdr = at<Header>(c.ws, L.hdr);
  const uint32_t *uoff = at<uint32_t>(c.ws, L.offs);
  const uint32_t *soff = uoff + c.B + 1;
  uint32_t *gate = at<uint32_t>(c.ws, L.gate);
  int32_t *cnt = c.mode == DDM_COUNT ? nullptr
                 : (c.per_update ? c.per_update : at<int32_t>(c.ws, L.cnt));
  const BucketArgs a = bucket_args(c);
  // the sampling pass clears the header and the per-instance counts, the
  // count pass the per-update counts
  BucketArgs prep = a;
  prep.zero = cnt;
  prep.zero_count = cnt ? n_total : 0u;
  DDM_HIP(bucket_prepare(prep, s));
  DDM_HIP(bucket_sweep(a, c.mode == DDM_COUNT ? 0 : 1, cnt, nullptr, nullptr, nullptr, nullptr,
                       &hdr->total, s, nullptr, c.mode == DDM_PAIRS));
  if (c.mode == DDM_PAIRS) {
    unsigned long long *off = at<unsigned long long>(c.ws, L.off);
    uint32_t *cur = at<uint32_t>(c.ws, L.cur);
    uint32_t *ps = at<uint32_t>(c.ws, L.ps);
    prof::mark(s, "batch.pairs.scan");
    DDM_HIP(exclusive_scan_widen(reinterpret_cast<const uint32_t *>(cnt), n_total, off,
                                 (size_t)n_total + 1, at<void>(c.ws, L.scan_tmp), s));
    bt_gate_kernel<<<grid_for((size_t)c.B + 1), 256, 0, s>>>(off, n_total, (uint64_t)c.cap, uoff,
                                                             (uint32_t)c.B, c.pair_off, gate);
    DDM_HIP(fill_u32(cur, 0u, n_total, s));
    BucketArgs emit = a;
    emit.inst_total = nullptr;  // the counting pass has set them
    // rows are implied by the offsets: the sweep writes subscription rows only
    DDM_HIP(bucket_sweep(emit, 2, nullptr, off, cur, nullptr, ps, &hdr->aux[0], s, gate));
    if (c.cap > 0 && n_total > 0) {
      prof::mark(s, "batch.pairs.order");
      const unsigned rgrid =
          (unsigned)std::max<size_t>(1, std::min<size_t>((n_total + kBtRowWaves * kWave - 1) /
                                                             (kBtRowWaves * kWave), 4096));
      bt_row_sort_kernel<<<rgrid, kBtRowThreads, 0, s>>>(off, cnt, ps, n_total, uoff, soff,
                                                         (uint32_t)c.B, gate,
                                                         reinterpret_cast<int2 *>(c.pairs));
    }
  }
  DDM_HIP(hipGetLastError());
  prof::end(s);
  return DDM_OK;
}

// Instance by instance through match_quiet() (any d; the path it picks falls
// back by itself), writing the batch outputs.
int run_each(const Batch &c, hipStream_t s, uint64_t *total_host) {
  const int64_t B = c.B;
  std::vector<uint64_t> counts((size_t)B, 0);
  std::vector<int64_t> poff((size_t)B + 1, 0);
  bool full = false;
  int64_t used = 0;
  uint64_t total = 0;
  for (int64_t b = 0; b < B; ++b) {
    const InstSpec &x = c.spec[(size_t)b];
    const int64_t u0 = c.uoff[(size_t)b], n = x.n, m = x.m;
    const int64_t room = full ? 0 : c.cap - used;
    uint64_t K = 0;
    const int rc = match_quiet(x.ulo, x.uhi, n, x.slo, x.shi, m, c.d, c.match_mode(), c.ws,
                             c.ws_bytes, s,
                             &K,
                             c.per_update && n > 0 ? c.per_update + u0 : nullptr,
                             c.mode == DDM_PAIRS && room > 0 ? c.pairs + 2 * used : nullptr,
                             room);
    if (rc == DDM_E_CAPACITY) {
      full = true;
    } else if (rc != DDM_OK) {
      return rc;
    }
    counts[(size_t)b] = K;
    total += K;
    poff[(size_t)b] = used;
    if (!full) used += (int64_t)K;
  }
  if (full) {  // offsets of every instance, as if the pairs had fit
    int64_t run = 0;
    for (int64_t b = 0; b < B; ++b) {
      poff[(size_t)b] = run;
      run += (int64_t)counts[(size_t)b];
    }
    used = run;
  }
  poff[(size_t)B] = used;
  DDM_HIP(hipMemcpyAsync(c.counts, counts.data(), counts.size() * sizeof(uint64_t),
                         hipMemcpyHostToDevice, s));
  if (c.mode == DDM_PAIRS)
    DDM_HIP(hipMemcpyAsync(c.pair_off, poff.data(), poff.size() * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
  DDM_HIP(hipStreamSynchronize(s));
  *total_host = total;
  return full ? DDM_E_CAPACITY : DDM_OK;
}

// Reads the outcome of an enqueued batch (stream synchronised first) and
// falls back to run_each() if a bucket overflowed.
int finish(const Batch &c, hipStream_t s, uint64_t *total_host, bool *fell_back) {
  Header h{};
  uint32_t gate[4] = {0, 0, 0, 0};
  DDM_HIP(hipMemcpyAsync(&h, at<Header>(c.ws, c.L.hdr), sizeof(Header), hipMemcpyDeviceToHost, s));
  DDM_HIP(hipMemcpyAsync(gate, at<uint32_t>(c.ws, c.L.gate), sizeof(gate), hipMemcpyDeviceToHost,
                         s));
  DDM_HIP(hipStreamSynchronize(s));
  prof::flush();
  if (h.err) return DDM_E_INVAL;
  // a bucket overflowed, or a row was longer than the row sort holds
  if (h.pad[0] || (c.mode == DDM_PAIRS && gate[0] != 0u && gate[2] != 0u)) {
    if (fell_back) *fell_back = true;
    return run_each(c, s, total_host);
  }
  *total_host = h.total;
  if (c.mode == DDM_PAIRS && gate[1]) return DDM_E_CAPACITY;
  return DDM_OK;
}

}  // namespace

size_t batch_staging_bytes(const Batch &c) {
  return align256(2 * ((size_t)c.B + 1) * sizeof(uint32_t)) + plan_bytes(c.L.bk);
}

int batch_begin(const Batch &c, hipStream_t s, void *pinned) {
  if (!c.bucketed) return DDM_E_UNSUPPORTED;
  std::vector<uint32_t> staging;
  int rc = upload(c, s, staging, pinned);
  if (rc != DDM_OK) return rc;
  rc = enqueue(c, s);
  if (rc == DDM_OK && !pinned && hipStreamSynchronize(s) != hipSuccess) rc = DDM_E_DEVICE;
  return rc;
}

int batch_finish(const Batch &c, hipStream_t s, uint64_t *total_host, bool *fell_back) {
  *total_host = 0;
  if (fell_back) *fell_back = !c.bucketed;
  if (!c.bucketed) return run_each(c, s, total_host);
  return finish(c, s, total_host, fell_back);
}

}  // namespace ddm

using namespace ddm;

struct ddm_batch_graph {
  Batch c;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" void ddm_default_tuning(ddm_tuning *out) {
  if (!out) return;
  const BucketTuning t;
  out->target = (int32_t)t.target;
  out->sweep_threads = (int32_t)t.sweep_threads;
  out->groups_per_thread = (int32_t)t.groups_per_thread;
  out->max_blocks = (int32_t)t.max_blocks;
}

extern "C" size_t ddm_batch_workspace_bytes(const int64_t *upd_off, const int64_t *sub_off,
                                            int64_t B, int d, int mode, int64_t pair_capacity,
                                            const ddm_tuning *tuning) {
  if (!shape_ok(upd_off, sub_off, B, d, mode, pair_capacity) || !tuning_valid(tuning)) return 0;
  const std::vector<InstSpec> spec =
      csr_specs(nullptr, nullptr, upd_off, nullptr, nullptr, sub_off, B, d);
  return workspace_for(spec, d, mode, pair_capacity, tuning);
}

extern "C" size_t ddm_multi_workspace_bytes(const ddm_instance *inst, int64_t B, int d, int mode,
                                            int64_t pair_capacity, const ddm_tuning *tuning) {
  if (!inst || B < 1 || !tuning_valid(tuning)) return 0;
  std::vector<InstSpec> spec((size_t)B);
  for (int64_t b = 0; b < B; ++b) spec[(size_t)b] = InstSpec{nullptr, nullptr, nullptr, nullptr,
                                                             inst[b].n, inst[b].m};
  if (!specs_ok(spec.data(), B, d, mode, pair_capacity)) return 0;
  return workspace_for(spec, d, mode, pair_capacity, tuning);
}


extern "C" int ddm_match_batched(const float *upd_lo, const float *upd_hi, const int64_t *upd_off,
                                 const float *sub_lo, const float *sub_hi, const int64_t *sub_off,
                                 int64_t B, int d, int mode, void *workspace, size_t ws_bytes,
                                 void *stream, const ddm_tuning *tuning, uint64_t *counts,
                                 uint64_t *total_host, int32_t *per_update, int32_t *pairs,
                                 int64_t *pair_off, int64_t pair_capacity) {
  if (!total_host) return DDM_E_INVAL;
  Batch c;
  int rc = make_batch_csr(c, upd_lo, upd_hi, upd_off, sub_lo, sub_hi, sub_off, B, d, mode,
                          workspace, ws_bytes, tuning, counts, per_update, pairs, pair_off,
                          pair_capacity);
  if (rc != DDM_OK) return rc;
  *total_host = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c.bucketed) {
    rc = batch_begin(c, s, nullptr);
    if (rc != DDM_OK) return rc;
  }
  return batch_finish(c, s, total_host);
}

extern "C" int ddm_match_multi(const ddm_instance *inst, int64_t B, int d, int mode,
                               void *workspace, size_t ws_bytes, void *stream,
                               const ddm_tuning *tuning, uint64_t *counts, uint64_t *total_host,
                               int32_t *per_update, int32_t *pairs, int64_t *pair_off,
                               int64_t pair_capacity) {
  if (!total_host || !inst || B < 1) return DDM_E_INVAL;
  std::vector<InstSpec> spec((size_t)B);
  for (int64_t b = 0; b < B; ++b)
    spec[(size_t)b] = InstSpec{inst[b].upd_lo, inst[b].upd_hi, inst[b].sub_lo, inst[b].sub_hi,
                               inst[b].n, inst[b].m};
  Batch c;
  int rc = make_batch(c, std::move(spec), d, mode, workspace, ws_bytes, tuning, counts,
                      per_update, pairs, pair_off, pair_capacity);
  if (rc != DDM_OK) return rc;
  *total_host = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c.bucketed) {
    rc = batch_begin(c, s, nullptr);
    if (rc != DDM_OK) return rc;
  }
  return batch_finish(c, s, total_host);
}

extern "C" int ddm_batch_graph_create(const float *upd_lo, const float *upd_hi,
                                      const int64_t *upd_off, const float *sub_lo,
                                      const float *sub_hi, const int64_t *sub_off, int64_t B,
                                      int d, int mode, void *workspace, size_t ws_bytes,
                                      const ddm_tuning *tuning, uint64_t *counts,
                                      int32_t *per_update, int32_t *pairs, int64_t *pair_off,
                                      int64_t pair_capacity, ddm_batch_graph **out) {
  if (!out) return DDM_E_INVAL;
  *out = nullptr;
  ddm_batch_graph *g = new (std::nothrow) ddm_batch_graph();
  if (!g) return DDM_E_DEVICE;
  int rc = make_batch_csr(g->c, upd_lo, upd_hi, upd_off, sub_lo, sub_hi, sub_off, B, d, mode,
                          workspace, ws_bytes, tuning, counts, per_update, pairs, pair_off,
                          pair_capacity);
  if (rc == DDM_OK && !g->c.bucketed) rc = DDM_E_UNSUPPORTED;
  if (rc != DDM_OK) {
    delete g;
    return rc;
  }
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    delete g;
    return DDM_E_DEVICE;
  }
  std::vector<uint32_t> staging;
  rc = upload(g->c, cs, staging, nullptr);
  if (rc == DDM_OK && hipStreamSynchronize(cs) != hipSuccess) rc = DDM_E_DEVICE;
  if (rc == DDM_OK) {
    const bool was = prof::swap_enabled(false);  // no event records inside the graph
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      rc = DDM_E_DEVICE;
    } else {
      rc = enqueue(g->c, cs);
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(cs, &graph);
      if (rc == DDM_OK && e != hipSuccess) rc = DDM_E_DEVICE;
      g->graph = graph;
      if (rc == DDM_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess)
        rc = DDM_E_DEVICE;
    }
    prof::swap_enabled(was);
  }
  (void)hipStreamDestroy(cs);
  if (rc != DDM_OK) {
    ddm_batch_graph_destroy(g);
    return rc;
  }
  *out = g;
  return DDM_OK;
}

extern "C" int ddm_batch_graph_launch(ddm_batch_graph *g, void *stream) {
  if (!g || !g->exec) return DDM_E_INVAL;
  if (hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)) != hipSuccess) return DDM_E_DEVICE;
  return DDM_OK;
}

extern "C" int ddm_batch_graph_result(ddm_batch_graph *g, void *stream, uint64_t *total_host) {
  if (!g || !g->exec || !total_host) return DDM_E_INVAL;
  *total_host = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  bool fell_back = false;
  const int rc = batch_finish(g->c, s, total_host, &fell_back);
  if (fell_back) {
    // the instance-by-instance fallback ran in the same workspace: put back
    // the batch plan and offsets that the captured launches read, so that the
    // next replay starts from them again
    std::vector<uint32_t> staging;
    const int up = upload(g->c, s, staging, nullptr);
    if (up != DDM_OK) return up;
    if (hipStreamSynchronize(s) != hipSuccess) return DDM_E_DEVICE;
  }
  return rc;
}

extern "C" int ddm_batch_graph_destroy(ddm_batch_graph *g) {
  if (!g) return DDM_OK;
  int rc = DDM_OK;
  if (g->exec && hipGraphExecDestroy(g->exec) != hipSuccess) rc = DDM_E_DEVICE;
  if (g->graph && hipGraphDestroy(g->graph) != hipSuccess) rc = DDM_E_DEVICE;
  delete g;
  return rc;
}

extern "C" int ddm_batch_autotune(const float *upd_lo, const float *upd_hi,
                                  const int64_t *upd_off, const float *sub_lo,
                                  const float *sub_hi, const int64_t *sub_off, int64_t B, int d,
                                  int mode, void *workspace, size_t ws_bytes, void *stream,
                                  uint64_t *counts, int32_t *per_update, int32_t *pairs,
                                  int64_t *pair_off, int64_t pair_capacity, ddm_tuning *best,
                                  double *best_ms) {
  if (!best) return DDM_E_INVAL;
  if (!shape_ok(upd_off, sub_off, B, d, mode, pair_capacity)) return DDM_E_INVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return DDM_E_DEVICE;
  std::vector<uint64_t> ref((size_t)B), got((size_t)B);
  bool have_ref = false, have_best = false;
  float best_t = 0.f;
  int rc = DDM_OK;
  for (const BucketTuning &t : candidates()) {
    ddm_tuning cand{(int32_t)t.target, (int32_t)t.sweep_threads, (int32_t)t.groups_per_thread,
                    (int32_t)t.max_blocks};
    ddm_batch_graph *g = nullptr;
    int r = ddm_batch_graph_create(upd_lo, upd_hi, upd_off, sub_lo, sub_hi, sub_off, B, d, mode,
                                   workspace, ws_bytes, &cand, counts, per_update, pairs, pair_off,
                                   pair_capacity, &g);
    if (r == DDM_E_UNSUPPORTED) continue;  // this shape does not fit the candidate
    if (r != DDM_OK) {
      rc = r;
      break;
    }
    uint64_t total = 0;
    float tmin = 0.f;
    for (int rep = 0; rep < 4 && r == DDM_OK; ++rep) {  // first replay warms up
      if (hipEventRecord(e0, s) != hipSuccess) r = DDM_E_DEVICE;
      if (r == DDM_OK) r = ddm_batch_graph_launch(g, stream);
      if (r == DDM_OK && hipEventRecord(e1, s) != hipSuccess) r = DDM_E_DEVICE;
      if (r == DDM_OK) r = ddm_batch_graph_result(g, stream, &total);
      float ms = 0.f;
      if (r == DDM_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) r = DDM_E_DEVICE;
      if (r == DDM_OK && rep > 0 && (rep == 1 || ms < tmin)) tmin = ms;
    }
    if (r == DDM_OK &&
        hipMemcpy(got.data(), counts, got.size() * sizeof(uint64_t), hipMemcpyDeviceToHost) !=
            hipSuccess)
      r = DDM_E_DEVICE;
    ddm_batch_graph_destroy(g);
    if (r == DDM_E_CAPACITY) r = DDM_OK;  // timing is still meaningful
    if (r != DDM_OK) {
      rc = r;
      break;
    }
    if (!have_ref) {
      ref = got;
      have_ref = true;
    } else if (ref != got) {  // every tuning must give the same result
      rc = DDM_E_DEVICE;
      break;
    }
    if (!have_best || tmin < best_t) {
      have_best = true;
      best_t = tmin;
      *best = cand;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != DDM_OK) return rc;
  if (!have_best) return DDM_E_UNSUPPORTED;
  if (best_ms) *best_ms = best_t;
  return DDM_OK;
}

// Serving runtime (declared in include/ddm.h).
//
// Simulations register their region state once; it stays in device memory
// and every request moves it one random-walk step and matches it.  Requests
// arrive open-loop (a driver thread releases each at its arrival time); the
// scheduler (the calling thread) admits them with continuous batching:
//   - whenever a slot (a stream with its own event, device counts and page-
//     locked staging) is free, it takes the pending requests in arrival
//     order, at most one per simulation and only for simulations with no
//     request in flight (so every simulation's steps stay in order), up to
//     max_batch of them;
//   - admission is bounded by the HBM budget: the group's workspace is carved
//     out of the caller's arena by a first-fit allocator, and the group is
//     cut from the back until it fits (if even its first request does not
//     fit, admission waits for a completion to free memory);
//   - the group is launched without blocking the host: each simulation's
//     step kernel, then one batched matching launch sequence over all of
//     them, then a copy of the per-request counts and an event;
//   - completed slots are found by polling their events; their memory is
//     returned to the arena and their simulations become free.
// Groups in different slots run on different streams and overlap on the
// device.  The plain policy is the per-request baseline: one request at a
// time in arrival order, each a step followed by match_quiet().  The incremental
// policy schedules like the batched one, but each simulation keeps a
// resident state (ddm_resident_*, carved from the front of the arena when it
// is registered) and a request is that state's step: no workspace is
// admitted per request.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/ddm.h"
#include "internal.h"
#include "batch.h"
#include "bucket_path.h"
#include "sim.h"

namespace ddm {
namespace {

using Clock = std::chrono::steady_clock;

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Sim {
  WalkArgs w;
  uint32_t steps = 0;  // steps enqueued so far
  bool busy = false;
  ddm_resident *res = nullptr;  // incremental policy: the resident state
};

// First-fit allocator of 256-byte aligned blocks over [0, size).
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = peak_ = 0;
  }
  bool take(size_t bytes, size_t *off) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t o = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[o + bytes] = rest;
      *off = o;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    bytes = align256(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0, peak_ = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  uint64_t *counts_dev = nullptr;   // [max_batch]
  uint64_t *counts_host = nullptr;  // page-locked [max_batch]
  void *staging = nullptr;          // page-locked plan staging
  size_t staging_bytes = 0;
  bool busy = false;
  Batch batch;
  std::vector<int64_t> reqs;
  size_t off = 0, bytes = 0;  // arena block
};

}  // namespace
}  // namespace ddm

using namespace ddm;

struct ddm_server {
  char *arena = nullptr;
  size_t arena_bytes = 0;
  int policy = DDM_SERVE_BATCHED;
  int max_batch = 1;
  int d = 0;
  size_t resident_top = 0;  // incremental policy: arena bytes held by resident states
  std::vector<Sim> sims;
  std::vector<Slot> slots;
  Arena alloc;
};

namespace {

void free_slot(Slot &s) {
  if (s.stream) (void)hipStreamDestroy(s.stream);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.counts_dev) (void)hipFree(s.counts_dev);
  if (s.counts_host) (void)hipHostFree(s.counts_host);
  if (s.staging) (void)hipHostFree(s.staging);
  s = Slot{};
}

std::vector<InstSpec> specs_of(const ddm_server &sv, const std::vector<int64_t> &reqs,
                               const int32_t *sim) {
  std::vector<InstSpec> out;
  out.reserve(reqs.size());
  for (int64_t r : reqs) {
    const WalkArgs &w = sv.sims[(size_t)sim[r]].w;
    out.push_back(InstSpec{w.upd_lo, w.upd_hi, w.sub_lo, w.sub_hi, w.n, w.m});
  }
  return out;
}

// Releases requests at their arrival times into the pending queue.
struct Driver {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<int64_t> pending;
  int64_t released = 0;
};

void drive(Driver *dv, const std::vector<int64_t> *order, const double *arrival,
           Clock::time_point t0) {
  for (int64_t i : *order) {
    const auto when = t0 + std::chrono::duration_cast<Clock::duration>(
                               std::chrono::duration<double>(arrival[i]));
    // sleep to shortly before, then spin: arrival times are kept to a few µs
    const auto early = when - std::chrono::microseconds(200);
    if (Clock::now() < early) std::this_thread::sleep_until(early);
    while (Clock::now() < when) std::this_thread::yield();
    {
      std::lock_guard<std::mutex> g(dv->mu);
      dv->pending.push_back(i);
      ++dv->released;
    }
    dv->cv.notify_one();
  }
}

double seconds_since(Clock::time_point t0, Clock::time_point t) {
  return std::chrono::duration<double>(t - t0).count();
}

}  // namespace

extern "C" int ddm_server_create(void *arena, size_t arena_bytes, int policy, int slots,
                                 int max_batch, ddm_server **out) {
  if (!out) return DDM_E_INVAL;
  *out = nullptr;
  if (!arena || (reinterpret_cast<uintptr_t>(arena) & 255) || arena_bytes < 256)
    return DDM_E_INVAL;
  if (policy != DDM_SERVE_BATCHED && policy != DDM_SERVE_PLAIN &&
      policy != DDM_SERVE_INCREMENTAL)
    return DDM_E_INVAL;
  if (slots < 1 || slots > 16 || max_batch < 1 || max_batch > 4096) return DDM_E_INVAL;
  ddm_server *sv = new (std::nothrow) ddm_server();
  if (!sv) return DDM_E_DEVICE;
  sv->arena = static_cast<char *>(arena);
  sv->arena_bytes = arena_bytes;
  sv->policy = policy;
  sv->max_batch = policy == DDM_SERVE_PLAIN ? 1 : max_batch;
  const int nslots = policy == DDM_SERVE_PLAIN ? 1 : slots;
  sv->slots.resize((size_t)nslots);
  bool ok = true;
  for (Slot &s : sv->slots) {
    s.staging_bytes = align256(2 * ((size_t)sv->max_batch + 1) * sizeof(uint32_t)) +
                      (size_t)sv->max_batch * sizeof(InstPlan);
    ok = ok && hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipMalloc(&s.counts_dev, (size_t)sv->max_batch * sizeof(uint64_t)) == hipSuccess;
    ok = ok && hipHostMalloc(&s.counts_host, (size_t)sv->max_batch * sizeof(uint64_t),
                             hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc(&s.staging, s.staging_bytes, hipHostMallocDefault) == hipSuccess;
    if (!ok) break;
  }
  if (!ok) {
    ddm_server_destroy(sv);
    return DDM_E_DEVICE;
  }
  *out = sv;
  return DDM_OK;
}

extern "C" int ddm_server_add_sim(ddm_server *sv, float *upd_lo, float *upd_hi, int64_t n,
                                  float *sub_lo, float *sub_hi, int64_t m, int d, float side,
                                  float sigma, uint64_t seed, int32_t *sim_id) {
  if (!sv || !sim_id || n < 0 || m < 0 || d < 1 || d > DDM_MAX_DIMS) return DDM_E_INVAL;
  if ((n > 0 && (!upd_lo || !upd_hi)) || (m > 0 && (!sub_lo || !sub_hi))) return DDM_E_INVAL;
  if ((n + m) * (int64_t)d >= (int64_t(1) << 32)) return DDM_E_INVAL;
  if (sv->d && d != sv->d) return DDM_E_INVAL;  // one batch holds one d
  if (sv->policy == DDM_SERVE_INCREMENTAL) {
    const size_t bytes = ddm_resident_bytes(n, m, d);
    if (bytes == 0) return DDM_E_INVAL;
    if (sv->resident_top + align256(bytes) > sv->arena_bytes) return DDM_E_WORKSPACE;
    Sim s;
    s.w = WalkArgs{upd_lo, upd_hi, n, sub_lo, sub_hi, m, d, side, sigma, seed, 0};
    const int e = ddm_resident_create(sv->arena + sv->resident_top, bytes, upd_lo, upd_hi, n,
                                      sub_lo, sub_hi, m, d, side, sigma, seed,
                                      sv->slots[0].stream, &s.res);
    if (e != DDM_OK) return e;
    sv->resident_top += align256(bytes);
    sv->d = d;
    sv->sims.push_back(s);
    *sim_id = (int32_t)sv->sims.size() - 1;
    return DDM_OK;
  }
  // the budget must hold any single request alone
  size_t need = ddm_workspace_bytes(n, m, d, DDM_COUNT, 0);
  if (sv->policy == DDM_SERVE_BATCHED) {
    const std::vector<InstSpec> one{InstSpec{upd_lo, upd_hi, sub_lo, sub_hi, n, m}};
    ddm_tuning t;
    ddm_default_tuning(&t);
    need = std::max(need, workspace_for(one, d, DDM_COUNT, 0, &t));
  }
  if (need == 0 || align256(need) > sv->arena_bytes) return DDM_E_WORKSPACE;
  sv->d = d;
  Sim s;
  s.w = WalkArgs{upd_lo, upd_hi, n, sub_lo, sub_hi, m, d, side, sigma, seed, 0};
  sv->sims.push_back(s);
  *sim_id = (int32_t)sv->sims.size() - 1;
  return DDM_OK;
}

extern "C" int ddm_server_run(ddm_server *sv, const int32_t *sim, const double *arrival_s,
                              int64_t count, uint64_t *counts, uint32_t *steps,
                              double *latency_s, ddm_serve_stats *stats) {
  if (!sv || count < 0 || (count > 0 && (!sim || !arrival_s || !counts || !steps || !latency_s)))
    return DDM_E_INVAL;
  for (int64_t i = 0; i < count; ++i)
    if (sim[i] < 0 || (size_t)sim[i] >= sv->sims.size() || !(arrival_s[i] >= 0.0))
      return DDM_E_INVAL;
  for (const Slot &s : sv->slots)
    if (s.busy) return DDM_E_INVAL;
  std::vector<int64_t> order((size_t)count);
  for (int64_t i = 0; i < count; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return arrival_s[a] < arrival_s[b]; });
  sv->alloc.reset(sv->arena_bytes);
  ddm_tuning tune;
  ddm_default_tuning(&tune);
  Driver dv;
  const Clock::time_point t0 = Clock::now() + std::chrono::milliseconds(2);
  std::thread driver(drive, &dv, &order, arrival_s, t0);

  int rc = DDM_OK;
  int64_t completed = 0, batches = 0, batched_requests = 0;
  auto fail = [&](int code) {
    if (rc == DDM_OK) rc = code;
  };

  if (sv->policy == DDM_SERVE_PLAIN) {
    Slot &s = sv->slots[0];
    while (completed < count) {
      int64_t r;
      {
        std::unique_lock<std::mutex> g(dv.mu);
        dv.cv.wait(g, [&] { return !dv.pending.empty(); });
        r = dv.pending.front();
        dv.pending.pop_front();
      }
      Sim &sm = sv->sims[(size_t)sim[r]];
      sm.w.step = ++sm.steps;
      steps[r] = sm.w.step;
      uint64_t K = 0;
      int e = launch_walk(sm.w, s.stream) == hipSuccess ? DDM_OK : DDM_E_DEVICE;
      if (e == DDM_OK)
        e = match_quiet(sm.w.upd_lo, sm.w.upd_hi, sm.w.n, sm.w.sub_lo, sm.w.sub_hi, sm.w.m, sm.w.d,
                      DDM_COUNT, sv->arena, sv->arena_bytes, s.stream, &K, nullptr, nullptr, 0);
      if (e != DDM_OK) fail(e);
      counts[r] = K;
      latency_s[r] = seconds_since(t0, Clock::now()) - arrival_s[r];
      ++completed;
      ++batches;
      ++batched_requests;
    }
  } else if (sv->policy == DDM_SERVE_INCREMENTAL) {
    while (completed < count) {
      bool progress = false;
      for (Slot &s : sv->slots) {
        if (!s.busy || hipEventQuery(s.done) != hipSuccess) continue;
        const double now = seconds_since(t0, Clock::now());
        for (int64_t r : s.reqs) {
          Sim &sm = sv->sims[(size_t)sim[r]];
          uint64_t K = 0;
          const int e = ddm_resident_finish(sm.res, &K);
          if (e != DDM_OK) fail(e);
          counts[r] = K;
          latency_s[r] = now - arrival_s[r];
          sm.busy = false;
        }
        completed += (int64_t)s.reqs.size();
        s.busy = false;
        s.reqs.clear();
        progress = true;
      }
      std::unique_lock<std::mutex> g(dv.mu);
      for (Slot &s : sv->slots) {
        if (s.busy || dv.pending.empty()) continue;
        std::vector<int64_t> group;
        for (size_t p = 0; p < dv.pending.size() && (int)group.size() < sv->max_batch;) {
          const int64_t r = dv.pending[p];
          Sim &sm = sv->sims[(size_t)sim[r]];
          if (sm.busy) {
            ++p;
            continue;
          }
          sm.busy = true;  // also keeps a second request of it out of this group
          group.push_back(r);
          dv.pending.erase(dv.pending.begin() + (std::ptrdiff_t)p);
        }
        if (group.empty()) break;
        s.reqs.clear();
        for (int64_t r : group) {
          Sim &sm = sv->sims[(size_t)sim[r]];
          sm.w.step = ++sm.steps;
          steps[r] = sm.w.step;
          const int e = ddm_resident_step(sm.res, sm.w.step, s.stream);
          if (e != DDM_OK) {
            fail(e);
            counts[r] = 0;
            latency_s[r] = seconds_since(t0, Clock::now()) - arrival_s[r];
            sm.busy = false;
            ++completed;
            continue;
          }
          s.reqs.push_back(r);
        }
        if (s.reqs.empty()) continue;
        if (hipEventRecord(s.done, s.stream) != hipSuccess) {
          fail(DDM_E_DEVICE);
          (void)hipStreamSynchronize(s.stream);
        }
        s.busy = true;
        ++batches;
        batched_requests += (int64_t)s.reqs.size();
        progress = true;
      }
      if (progress) continue;
      bool inflight = false;
      for (const Slot &s : sv->slots) inflight = inflight || s.busy;
      if (inflight) {
        g.unlock();
        std::this_thread::yield();
      } else if (completed < count) {
        const int64_t seen = dv.released;
        dv.cv.wait(g, [&] { return dv.released > seen || !dv.pending.empty(); });
      }
    }
  } else {
    while (completed < count) {
      bool progress = false;
      // completions
      for (Slot &s : sv->slots) {
        if (!s.busy || hipEventQuery(s.done) != hipSuccess) continue;
        uint64_t total = 0;
        bool fell_back = false;
        const int e = batch_finish(s.batch, s.stream, &total, &fell_back);
        if (e != DDM_OK) fail(e);
        if (fell_back) {
          // the counts were produced after the copy (per-instance fallback)
          if (hipMemcpy(s.counts_host, s.counts_dev, s.reqs.size() * sizeof(uint64_t),
                        hipMemcpyDeviceToHost) != hipSuccess)
            fail(DDM_E_DEVICE);
        }
        const double now = seconds_since(t0, Clock::now());
        for (size_t j = 0; j < s.reqs.size(); ++j) {
          const int64_t r = s.reqs[j];
          counts[r] = s.counts_host[j];
          latency_s[r] = now - arrival_s[r];
          sv->sims[(size_t)sim[r]].busy = false;
        }
        completed += (int64_t)s.reqs.size();
        sv->alloc.give(s.off, s.bytes);
        s.busy = false;
        s.reqs.clear();
        progress = true;
      }
      // admissions
      std::unique_lock<std::mutex> g(dv.mu);
      for (Slot &s : sv->slots) {
        if (s.busy || dv.pending.empty()) continue;
        std::vector<int64_t> group;
        std::vector<size_t> picked;  // positions in pending
        std::vector<int32_t> chosen;
        for (size_t p = 0; p < dv.pending.size() && (int)group.size() < sv->max_batch; ++p) {
          const int64_t r = dv.pending[p];
          const int32_t sm = sim[r];
          if (sv->sims[(size_t)sm].busy ||
              std::find(chosen.begin(), chosen.end(), sm) != chosen.end())
            continue;
          group.push_back(r);
          picked.push_back(p);
          chosen.push_back(sm);
        }
        if (group.empty()) break;
        size_t need = 0, off = 0;
        bool got = false;
        while (!group.empty()) {
          need = workspace_for(specs_of(*sv, group, sim), sv->d, DDM_COUNT, 0, &tune);
          if (sv->alloc.take(need, &off)) {
            got = true;
            break;
          }
          group.pop_back();
          picked.pop_back();
        }
        if (!got) break;  // wait for memory
        for (size_t k = picked.size(); k-- > 0;)
          dv.pending.erase(dv.pending.begin() + (std::ptrdiff_t)picked[k]);
        // launch: steps, then one batched match of the group
        s.reqs = group;
        s.off = off;
        s.bytes = need;
        for (int64_t r : group) {
          Sim &sm = sv->sims[(size_t)sim[r]];
          sm.busy = true;
          sm.w.step = ++sm.steps;
          steps[r] = sm.w.step;
          if (launch_walk(sm.w, s.stream) != hipSuccess) fail(DDM_E_DEVICE);
        }
        int e = make_batch(s.batch, specs_of(*sv, group, sim), sv->d, DDM_COUNT,
                           sv->arena + off, need, &tune, s.counts_dev, nullptr, nullptr, nullptr,
                           0);
        if (e == DDM_OK && s.batch.bucketed) {
          if (batch_staging_bytes(s.batch) > s.staging_bytes) e = DDM_E_INVAL;
          if (e == DDM_OK) e = batch_begin(s.batch, s.stream, s.staging);
          if (e == DDM_OK &&
              hipMemcpyAsync(s.counts_host, s.counts_dev, group.size() * sizeof(uint64_t),
                             hipMemcpyDeviceToHost, s.stream) != hipSuccess)
            e = DDM_E_DEVICE;
        }
        if (e == DDM_OK && hipEventRecord(s.done, s.stream) != hipSuccess) e = DDM_E_DEVICE;
        if (e != DDM_OK) {
          // nothing usable was enqueued for this group: finish it as failed
          fail(e);
          (void)hipStreamSynchronize(s.stream);
          const double now = seconds_since(t0, Clock::now());
          for (int64_t r : group) {
            counts[r] = 0;
            latency_s[r] = now - arrival_s[r];
            sv->sims[(size_t)sim[r]].busy = false;
          }
          completed += (int64_t)group.size();
          sv->alloc.give(off, need);
          s.reqs.clear();
          continue;
        }
        s.busy = true;
        ++batches;
        batched_requests += (int64_t)group.size();
        progress = true;
      }
      if (progress) continue;
      bool inflight = false;
      for (const Slot &s : sv->slots) inflight = inflight || s.busy;
      if (inflight) {
        g.unlock();
        std::this_thread::yield();
      } else if (completed < count) {
        const int64_t seen = dv.released;
        dv.cv.wait(g, [&] { return dv.released > seen || !dv.pending.empty(); });
      }
    }
  }
  driver.join();
  if (stats) {
    stats->wall_s = seconds_since(t0, Clock::now());
    stats->launches = batches;
    stats->mean_batch = batches ? (double)batched_requests / (double)batches : 0.0;
    stats->peak_arena_bytes = sv->policy == DDM_SERVE_INCREMENTAL ? (double)sv->resident_top
                                                                  : (double)sv->alloc.peak();
  }
  return rc;
}

extern "C" int ddm_server_export(ddm_server *sv, int32_t sim_id) {
  if (!sv || sim_id < 0 || (size_t)sim_id >= sv->sims.size()) return DDM_E_INVAL;
  for (const Slot &s : sv->slots)
    if (s.busy) return DDM_E_INVAL;
  const Sim &sm = sv->sims[(size_t)sim_id];
  if (!sm.res) return DDM_OK;
  return ddm_resident_export(sm.res, sm.w.upd_lo, sm.w.upd_hi, sm.w.sub_lo, sm.w.sub_hi,
                             sv->slots[0].stream);
}

extern "C" int ddm_server_destroy(ddm_server *sv) {
  if (!sv) return DDM_OK;
  for (Slot &s : sv->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
  }
  for (Sim &sm : sv->sims) {
    if (sm.res) (void)ddm_resident_destroy(sm.res);
    sm.res = nullptr;
  }
  for (Slot &s : sv->slots) {
    free_slot(s);
  }
  delete sv;
  return DDM_OK;
}

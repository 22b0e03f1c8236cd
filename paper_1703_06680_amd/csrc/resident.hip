// Resident simulations matched incrementally (declared in include/ddm.h):
// the dynamic matching problem of the paper's Sec. 6 (regions that move
// between requests).
//
// A simulation that issues one count request per time step moves its
// regions by a small random walk between requests (sigma = 0.1 side in the
// serving workload), so from one step to the next almost every region stays
// in the bucket of the bucketed path it was in: the bucket order, the part
// of Algorithm 5 that costs a sort, barely changes.  The resident state
// therefore keeps the regions themselves in bucket order, in fixed-capacity
// slabs (one per bucket, plus one for empty regions), and a step is
//   step    one workgroup per slab moves its regions in place (the motion of
//           ddm_sim_step, bit for bit), keeps those still in the slab's
//           bucket, compacted, with their sweep records and their
//           boundary-state copies (Algorithm 6's SubSet / UpdSet entries of
//           the later buckets their interval reaches), and lists the rest;
//   insert  every listed region joins the slab of its new bucket;
//   sweep   the bucket sweep of the bucketed path over the slabs.
// There is no sampling, counting, prefix sum or scattered store per region
// (the sort-like part of the matching call); the movers, a few per million
// regions per step, are the only scattered writes.
//
// Everything is exact: the bucket map stays the one chosen when the slabs
// were built, and any map gives the same pairs.  When a slab or the mover
// list fills up, or a bucket's boundary state does not fit, that step's
// state is written back in region order, counted by the full matching call
// (ddm_match), and the slabs are rebuilt from it; a simulation that needs
// this twice in a row, or whose regions do not fit the slabs at all, keeps
// its regions in region order and is matched by the full call, trying the
// slabs again every 64 steps (one repair in the first slab step sends it back).
#include <string.h>

#include <algorithm>
#include <new>

#include "../../include/ddm.h"
#include "internal.h"
#include "bucket_dev.h"
#include "bucket_path.h"
#include "philox.h"
#include "primitives.h"
#include "profile.h"
#include "sim.h"

namespace ddm {
namespace {

constexpr uint32_t kSlab = kBucketCap;  // region slots per bucket slab
constexpr uint32_t kBsSlab = 512;       // boundary-state records per bucket
constexpr int kStepThreads = 512;
constexpr int kStepItems = (int)kSlab / kStepThreads;
constexpr int kInsertThreads = 256;
constexpr int kRetrySteps = 64;  // full-match steps before the slabs are tried again

// Step flags (ResCounters::flags, one word per step parity).
constexpr uint32_t kResMoverFull = 1u;  // the mover list was full: a region stayed misplaced
constexpr uint32_t kResSlabFull = 2u;   // a mover found its new slab full
constexpr uint32_t kResBad = 4u;        // a moved coordinate is NaN

struct ResCounters {
  uint32_t flags[2];   // per step parity
  uint32_t movers[2];  // regions listed to change slab, per step parity
  uint32_t build_overflow;
  uint32_t pad[3];
};

// A region changing slab: its index, new slab and moved corners.
struct Mover {
  uint32_t id, dest;
  float lo[3], hi[3];
};

struct ResDev {
  uint32_t nb;     // buckets; slab nb holds the empty regions
  uint32_t nv;     // region slots over all slabs ((nb + 1) * kSlab)
  uint32_t n;      // updates (region indices below n)
  uint32_t mcap;   // mover list capacity per parity
  uint32_t *ids;   // [nv] region index of each slot
  float *lo, *hi;  // [nv][d]
  uint4 *rec;      // [nv] sweep records (slabs 0 .. nb-1)
  uint32_t *cnt;   // [nb + 1] filled slots per slab
  uint4 *bs_rec;   // [nb][kBsSlab]
  uint32_t *bs_cnt;  // [2][nb] boundary-state entries per bucket, per step parity
  Mover *movers;     // [2][mcap]
  ResCounters *ctr;
  Header *hdr;
  const BucketParams *P;
  float side, sigma;
  uint32_t k0, k1;
};

// The sweep record of a region at slot g: keys of the swept axis, the slot
// (offset by nv for a subscription: the sweep tells the kinds apart by it
// and reads the exact other-axis coordinates at that slot) and the
// quantised other axes.
template <int D>
__device__ __forceinline__ uint4 res_record(const Box<D> &b, uint32_t id, uint32_t g,
                                            const ResDev &a, const BucketParams &p) {
  return make_uint4(encode_coord(b.lo[0]), encode_coord(b.hi[0]), id < a.n ? g : a.nv + g,
                    qword_of<D>(b, p, 0u));
}

// Copies of the record into the boundary state of every later bucket the
// interval may still be active in (buckets past the first up to the bucket
// of its upper coordinate, as the bucketed path's count pass does).
template <int D>
__device__ __forceinline__ void res_boundary(const Box<D> &b, uint4 r, uint32_t first,
                                             const ResDev &a, const BucketParams &p,
                                             uint32_t par) {
  const uint32_t last = bucket_of(b.hi[0], p.vmin, p.scale, a.nb);
  for (uint32_t j = first + 1; j <= last; ++j) {
    const uint32_t k = atomicAdd(&a.bs_cnt[par * a.nb + j], 1u);
    if (k < kBsSlab) a.bs_rec[(size_t)j * kBsSlab + k] = r;
  }
}

template <int D>
__device__ __forceinline__ void res_store(const ResDev &a, size_t g, uint32_t id, const Box<D> &b) {
  a.ids[g] = id;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    a.lo[g * D + k] = b.lo[k];
    a.hi[g * D + k] = b.hi[k];
  }
}

// One workgroup per slab (blockIdx.x = nb: the empty regions).  move = 0
// recomputes the records and boundary state of the regions where they are.
template <int D>
__global__ __launch_bounds__(kStepThreads) void res_step_kernel(ResDev a, uint32_t step,
                                                                uint32_t move) {
  __shared__ uint32_t red[kStepThreads / kWave + 1];
  const uint32_t b = blockIdx.x;
  const uint32_t par = step & 1u;
  const int t = threadIdx.x;
  const BucketParams p = *a.P;
  if (t == 0) {
    if (b == 0) {
      // the other parity belongs to the previous step, finished and read
      a.hdr->total = 0ull;
      a.hdr->pad[0] = 0u;
      a.ctr->flags[par ^ 1u] = 0u;
      a.ctr->movers[par ^ 1u] = 0u;
    }
    if (b < a.nb) a.bs_cnt[(par ^ 1u) * a.nb + b] = 0u;
  }
  const uint32_t C = min(a.cnt[b], kSlab);
  uint32_t id[kStepItems];
  Box<D> bx[kStepItems];
  bool keep[kStepItems];
  uint32_t nkeep = 0, flags = 0;
#pragma unroll
  for (int i = 0; i < kStepItems; ++i) {
    const uint32_t s = (uint32_t)t + (uint32_t)i * kStepThreads;
    keep[i] = false;
    id[i] = 0;
    if (s >= C) continue;
    const size_t g = (size_t)b * kSlab + s;
    id[i] = a.ids[g];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      bx[i].lo[k] = a.lo[g * D + k];
      bx[i].hi[k] = move ? 0.f : a.hi[g * D + k];  // a move recomputes it
    }
    if (move) {
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const float z = irwin_hall12(id[i], (uint32_t)k, step, a.k0, a.k1);
        const float moved = __fadd_rn(bx[i].lo[k], __fmul_rn(a.sigma, z));
        bx[i].lo[k] = moved;
        bx[i].hi[k] = __fadd_rn(moved, a.side);
      }
    }
    bool empty;
    if (box_errors<D>(bx[i], empty, 0u)) flags |= kResBad;
    const uint32_t dest = empty ? a.nb : bucket_of(bx[i].lo[0], p.vmin, p.scale, a.nb);
    keep[i] = true;
    if (dest != b) {
      const uint32_t k = atomicAdd(&a.ctr->movers[par], 1u);
      if (k < a.mcap) {
        Mover mv;
        mv.id = id[i];
        mv.dest = dest;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          mv.lo[c] = c < D ? bx[i].lo[c % D] : 0.f;
          mv.hi[c] = c < D ? bx[i].hi[c % D] : 0.f;
        }
        a.movers[(size_t)par * a.mcap + k] = mv;
        keep[i] = false;
      } else {
        flags |= kResMoverFull;  // stays here, misplaced: the host rebuilds
      }
    }
    nkeep += keep[i] ? 1u : 0u;
  }
  if (flags) atomicOr(&a.ctr->flags[par], flags);
  // every slot of the slab is in registers before the scan's barriers, so
  // the compacted stores below overwrite nothing still to be read.  A slab
  // that lost no region keeps every region in its slot (its index need not
  // be written again); one that did is compacted.
  uint32_t total;
  uint32_t pos = block_exclusive_scan<uint32_t, kStepThreads>(nkeep, red, &total);
  const bool stay = total == C;
#pragma unroll
  for (int i = 0; i < kStepItems; ++i) {
    if (!keep[i]) continue;
    const size_t g =
        (size_t)b * kSlab + (stay ? (uint32_t)t + (uint32_t)i * kStepThreads : pos++);
    if (!stay) a.ids[g] = id[i];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      a.lo[g * D + k] = bx[i].lo[k];
      a.hi[g * D + k] = bx[i].hi[k];
    }
    if (b < a.nb) {
      const uint4 r = res_record<D>(bx[i], id[i], (uint32_t)g, a, p);
      a.rec[g] = r;
      res_boundary<D>(bx[i], r, b, a, p, par);
    }
  }
  if (t == 0) a.cnt[b] = total;
}

// Every listed region joins the slab of its new bucket.
template <int D>
__global__ __launch_bounds__(kInsertThreads) void res_insert_kernel(ResDev a, uint32_t step) {
  const uint32_t par = step & 1u;
  const BucketParams p = *a.P;
  const uint32_t count = min(a.ctr->movers[par], a.mcap);
  for (uint32_t i = blockIdx.x * kInsertThreads + threadIdx.x; i < count;
       i += gridDim.x * kInsertThreads) {
    const Mover mv = a.movers[(size_t)par * a.mcap + i];
    const uint32_t local = atomicAdd(&a.cnt[mv.dest], 1u);
    if (local >= kSlab) {
      atomicOr(&a.ctr->flags[par], kResSlabFull);  // it stays in the list only
      continue;
    }
    Box<D> bx;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      bx.lo[k] = mv.lo[k];
      bx.hi[k] = mv.hi[k];
    }
    const size_t g = (size_t)mv.dest * kSlab + local;
    res_store<D>(a, g, mv.id, bx);
    if (mv.dest < a.nb) {
      const uint4 r = res_record<D>(bx, mv.id, (uint32_t)g, a, p);
      a.rec[g] = r;
      res_boundary<D>(bx, r, mv.dest, a, p, par);
    }
  }
}

// Every region's corners into row arrays (region order): the filled slots of
// every slab, and the movers listed by the step of parity par (after a
// successful step they are in their slabs too, with the same values).
template <int D>
__global__ __launch_bounds__(256) void res_export_kernel(ResDev a, uint32_t par,
                                                         float *__restrict__ ulo,
                                                         float *__restrict__ uhi,
                                                         float *__restrict__ slo,
                                                         float *__restrict__ shi) {
  auto put = [&](uint32_t id, const float *l, const float *h) {
    const bool upd = id < a.n;
    float *L = upd ? ulo : slo;
    float *H = upd ? uhi : shi;
    const size_t row = upd ? id : id - a.n;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      L[row * D + k] = l[k];
      H[row * D + k] = h[k];
    }
  };
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < a.nv; x += stride) {
    const uint32_t b = x / kSlab, s = x - b * kSlab;
    if (s >= min(a.cnt[b], kSlab)) continue;
    put(a.ids[x], a.lo + (size_t)x * D, a.hi + (size_t)x * D);
  }
  const uint32_t count = min(a.ctr->movers[par], a.mcap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const Mover &mv = a.movers[(size_t)par * a.mcap + i];
    put(mv.id, mv.lo, mv.hi);
  }
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Device state, carved from the caller's buffer.
struct ResLayout {
  bool slabs = false;  // false: full-matching mode only (d > 3, no regions, or too large)
  uint32_t nb = 0, nv = 0, mcap = 0;
  size_t hdr = 0, ctr = 0, params = 0, cnt = 0, bs_cnt = 0, ids = 0, lo = 0, hi = 0, rec = 0,
         bs_rec = 0, movers = 0, home = 0, scratch = 0, scratch_bytes = 0, bytes = 0;
};

ResLayout res_layout(int64_t n, int64_t m, int d) {
  ResLayout R;
  const int64_t N = n + m;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t o = at;
    at += align256(bytes);
    return o;
  };
  R.hdr = take(sizeof(Header) + sizeof(ResCounters));
  R.ctr = R.hdr + sizeof(Header);
  R.params = take(sizeof(BucketParams));
  R.home = take(2 * (size_t)N * (size_t)d * sizeof(float));
  size_t build = 0;
  if (d <= 3 && N > 0 && bucket_path_supported(d, n, m)) {
    const BucketLayout L = bucket_layout(nullptr, nullptr, n, nullptr, nullptr, m, d);
    const uint64_t nv = (uint64_t)(L.nb + 1) * kSlab;
    if (2 * nv < (1ull << 32)) {
      R.slabs = true;
      R.nb = L.nb;
      R.nv = (uint32_t)nv;
      R.mcap = (uint32_t)(N / 32 + 1024);
      build = L.rec;  // the build uses the layout's buffers before the records
      R.cnt = take(((size_t)R.nb + 1) * sizeof(uint32_t));
      R.bs_cnt = take(2 * (size_t)R.nb * sizeof(uint32_t));
      R.ids = take(nv * sizeof(uint32_t));
      R.lo = take(nv * (size_t)d * sizeof(float));
      R.hi = take(nv * (size_t)d * sizeof(float));
      R.rec = take(nv * sizeof(uint4));
      R.bs_rec = take((size_t)R.nb * kBsSlab * sizeof(uint4));
      R.movers = take(2 * (size_t)R.mcap * sizeof(Mover));
    }
  }
  R.scratch_bytes = std::max(build, ddm_workspace_bytes(n, m, d, DDM_COUNT, 0));
  R.scratch = take(R.scratch_bytes);
  R.bytes = at;
  return R;
}

}  // namespace
}  // namespace ddm

using namespace ddm;

struct ddm_resident {
  char *state = nullptr;
  ResLayout R;
  int64_t n = 0, m = 0;
  int d = 0;
  float side = 0.f, sigma = 0.f;
  uint64_t seed = 0;
  bool full_mode = false;  // every step by launch_walk + ddm_match on the home rows
  int full_steps = 0;      // steps in full-match mode since it was entered or last retried
  bool pending = false;
  uint32_t step = 0;       // step of the pending (or last) request
  int consecutive_repairs = 0;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  char *host = nullptr;    // page-locked copy of Header + ResCounters
  ddm_resident_info info{};

  float *home(int which) const {  // 0 ulo, 1 uhi, 2 slo, 3 shi
    const size_t nu = (size_t)n * d, ns = (size_t)m * d;
    float *base = reinterpret_cast<float *>(state + R.home);
    const size_t off[4] = {0, nu, 2 * nu, 2 * nu + ns};
    return base + off[which];
  }
  ResDev dev() const {
    ResDev a{};
    a.nb = R.nb;
    a.nv = R.nv;
    a.n = (uint32_t)n;
    a.mcap = R.mcap;
    a.ids = reinterpret_cast<uint32_t *>(state + R.ids);
    a.lo = reinterpret_cast<float *>(state + R.lo);
    a.hi = reinterpret_cast<float *>(state + R.hi);
    a.rec = reinterpret_cast<uint4 *>(state + R.rec);
    a.cnt = reinterpret_cast<uint32_t *>(state + R.cnt);
    a.bs_rec = reinterpret_cast<uint4 *>(state + R.bs_rec);
    a.bs_cnt = reinterpret_cast<uint32_t *>(state + R.bs_cnt);
    a.movers = reinterpret_cast<Mover *>(state + R.movers);
    a.ctr = reinterpret_cast<ResCounters *>(state + R.ctr);
    a.hdr = reinterpret_cast<Header *>(state + R.hdr);
    a.P = reinterpret_cast<const BucketParams *>(state + R.params);
    a.side = side;
    a.sigma = sigma;
    a.k0 = (uint32_t)seed;
    a.k1 = (uint32_t)(seed >> 32);
    return a;
  }
};

namespace {

hipError_t launch_step(const ddm_resident &r, uint32_t step, uint32_t move, hipStream_t s) {
  const ResDev a = r.dev();
  // movers are a few per million regions: a small grid, striding over more
  const unsigned grid = std::max(1u, std::min(16u, (a.mcap + kInsertThreads - 1) / kInsertThreads));
  prof::mark(s, "resident.step");
  switch (r.d) {
    case 1:
      res_step_kernel<1><<<a.nb + 1, kStepThreads, 0, s>>>(a, step, move);
      res_insert_kernel<1><<<grid, kInsertThreads, 0, s>>>(a, step);
      break;
    case 2:
      res_step_kernel<2><<<a.nb + 1, kStepThreads, 0, s>>>(a, step, move);
      res_insert_kernel<2><<<grid, kInsertThreads, 0, s>>>(a, step);
      break;
    default:
      res_step_kernel<3><<<a.nb + 1, kStepThreads, 0, s>>>(a, step, move);
      res_insert_kernel<3><<<grid, kInsertThreads, 0, s>>>(a, step);
      break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  SlabSweep w{};
  w.rec = reinterpret_cast<const uint32_t *>(a.rec);
  w.bs_rec = reinterpret_cast<const uint32_t *>(a.bs_rec);
  w.cnt = a.cnt;
  w.bs_cnt = a.bs_cnt + (size_t)(step & 1u) * a.nb;
  w.cap = kSlab;
  w.bs_slab = kBsSlab;
  w.nb = a.nb;
  w.nv = a.nv;
  w.lo = a.lo;
  w.hi = a.hi;
  w.hdr = a.hdr;
  w.d = r.d;
  return bucket_sweep_slabs(w, s);
}

hipError_t launch_export(const ddm_resident &r, uint32_t par, float *ulo, float *uhi, float *slo,
                         float *shi, hipStream_t s) {
  const ResDev a = r.dev();
  const unsigned grid = std::max(1u, std::min(4096u, (a.nv + 255) / 256));
  switch (r.d) {
    case 1: res_export_kernel<1><<<grid, 256, 0, s>>>(a, par, ulo, uhi, slo, shi); break;
    case 2: res_export_kernel<2><<<grid, 256, 0, s>>>(a, par, ulo, uhi, slo, shi); break;
    default: res_export_kernel<3><<<grid, 256, 0, s>>>(a, par, ulo, uhi, slo, shi); break;
  }
  return hipGetLastError();
}

// Slabs from the home rows (region order).  Returns DDM_OK, DDM_E_INVAL for
// invalid rows, or 1 if the regions do not fit the slabs.
int build(ddm_resident &r, hipStream_t s) {
  const ResDev a = r.dev();
  const BucketLayout L =
      bucket_layout(r.home(0), r.home(1), r.n, r.home(2), r.home(3), r.m, r.d);
  BucketArgs ba{};
  ba.d = r.d;
  ba.ws = r.state + r.R.scratch;
  ba.L = &L;
  ba.hdr = a.hdr;
  SlabBuild sb{a.ids, a.lo, a.hi, a.cnt, kSlab, &a.ctr->build_overflow};
  bool ok = fill_u32(reinterpret_cast<uint32_t *>(a.ctr), 0u,
                     sizeof(ResCounters) / sizeof(uint32_t), s) == hipSuccess;
  ok = ok && fill_u32(a.bs_cnt, 0u, 2 * (size_t)a.nb, s) == hipSuccess;
  ok = ok && bucket_build_slabs(ba, sb, s) == hipSuccess;
  // the bucket map lives outside the scratch, which the full matching call reuses
  ok = ok && hipMemcpyAsync(const_cast<BucketParams *>(a.P), r.state + r.R.scratch + L.params,
                            sizeof(BucketParams), hipMemcpyDeviceToDevice, s) == hipSuccess;
  ok = ok && hipMemcpyAsync(r.host, a.hdr, sizeof(Header) + sizeof(ResCounters),
                            hipMemcpyDeviceToHost, s) == hipSuccess;
  ok = ok && hipStreamSynchronize(s) == hipSuccess;
  if (!ok) return DDM_E_DEVICE;
  const Header *h = reinterpret_cast<const Header *>(r.host);
  const ResCounters *c = reinterpret_cast<const ResCounters *>(r.host + sizeof(Header));
  if (h->err) return DDM_E_INVAL;
  return c->build_overflow ? 1 : DDM_OK;
}

// Count of the home rows by the full matching call.
int full_match(ddm_resident &r, hipStream_t s, uint64_t *count) {
  return match_quiet(r.home(0), r.home(1), r.n, r.home(2), r.home(3), r.m, r.d, DDM_COUNT,
                   r.state + r.R.scratch, r.R.scratch_bytes, s, count, nullptr, nullptr, 0);
}

}  // namespace

extern "C" size_t ddm_resident_bytes(int64_t n, int64_t m, int d) {
  if (n < 0 || m < 0 || d < 1 || d > DDM_MAX_DIMS || (n + m) * (int64_t)d >= (int64_t(1) << 31))
    return 0;
  const ResLayout R = res_layout(n, m, d);
  return R.scratch_bytes ? R.bytes : 0;
}

extern "C" int ddm_resident_create(void *state, size_t state_bytes, const float *upd_lo,
                                   const float *upd_hi, int64_t n, const float *sub_lo,
                                   const float *sub_hi, int64_t m, int d, float side, float sigma,
                                   uint64_t seed, void *stream, ddm_resident **out) {
  if (!out) return DDM_E_INVAL;
  *out = nullptr;
  const size_t need = ddm_resident_bytes(n, m, d);
  if (need == 0) return DDM_E_INVAL;
  if ((n > 0 && (!upd_lo || !upd_hi)) || (m > 0 && (!sub_lo || !sub_hi))) return DDM_E_INVAL;
  if (!(side >= 0.f && side <= 3.0e38f) || !(fabsf(sigma) <= 1.0e30f)) return DDM_E_INVAL;
  if (!state || (reinterpret_cast<uintptr_t>(state) & 255)) return DDM_E_INVAL;
  if (state_bytes < need) return DDM_E_WORKSPACE;
  ddm_resident *r = new (std::nothrow) ddm_resident();
  if (!r) return DDM_E_DEVICE;
  r->state = static_cast<char *>(state);
  r->R = res_layout(n, m, d);
  r->n = n;
  r->m = m;
  r->d = d;
  r->side = side;
  r->sigma = sigma;
  r->seed = seed;
  hipStream_t s = static_cast<hipStream_t>(stream);
  r->stream = s;
  bool ok = hipEventCreateWithFlags(&r->done, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void **>(&r->host), 256, hipHostMallocDefault) ==
                 hipSuccess;
  const size_t nu = (size_t)n * d * sizeof(float), ns = (size_t)m * d * sizeof(float);
  if (ok && nu) {
    ok = hipMemcpyAsync(r->home(0), upd_lo, nu, hipMemcpyDeviceToDevice, s) == hipSuccess &&
         hipMemcpyAsync(r->home(1), upd_hi, nu, hipMemcpyDeviceToDevice, s) == hipSuccess;
  }
  if (ok && ns) {
    ok = hipMemcpyAsync(r->home(2), sub_lo, ns, hipMemcpyDeviceToDevice, s) == hipSuccess &&
         hipMemcpyAsync(r->home(3), sub_hi, ns, hipMemcpyDeviceToDevice, s) == hipSuccess;
  }
  int rc = ok ? DDM_OK : DDM_E_DEVICE;
  if (rc == DDM_OK) {
    if (r->R.slabs) {
      const int b = build(*r, s);
      if (b == 1)
        r->full_mode = true;
      else
        rc = b;
    } else {
      // rows are validated by one full call (the state is matched that way)
      uint64_t k = 0;
      r->full_mode = true;
      rc = full_match(*r, s, &k);
    }
  }
  if (rc != DDM_OK) {
    ddm_resident_destroy(r);
    return rc;
  }
  r->info.buckets = r->full_mode ? 0 : (int32_t)r->R.nb;
  r->info.full_mode = r->full_mode ? 1 : 0;
  *out = r;
  return DDM_OK;
}

extern "C" int ddm_resident_step(ddm_resident *r, uint32_t step, void *stream) {
  if (!r || r->pending || step == 0) return DDM_E_INVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (r->full_mode) {
    WalkArgs w{r->home(0), r->home(1), r->n, r->home(2), r->home(3), r->m, r->d,
               r->side, r->sigma, r->seed, step};
    e = launch_walk(w, s);
  } else {
    e = launch_step(*r, step, 1u, s);
    prof::end(s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(r->host, r->state + r->R.hdr, sizeof(Header) + sizeof(ResCounters),
                         hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipEventRecord(r->done, s);
  if (e != hipSuccess) return DDM_E_DEVICE;
  r->stream = s;
  r->step = step;
  r->pending = true;
  return DDM_OK;
}

extern "C" int ddm_resident_finish(ddm_resident *r, uint64_t *count) {
  if (!r || !count || !r->pending) return DDM_E_INVAL;
  *count = 0;
  r->pending = false;
  if (hipEventSynchronize(r->done) != hipSuccess) return DDM_E_DEVICE;
  prof::flush();
  hipStream_t s = r->stream;
  ++r->info.steps;
  if (r->full_mode) {
    ++r->info.full_matches;
    const int rc = full_match(*r, s, count);
    if (rc != DDM_OK || !r->R.slabs || ++r->full_steps < kRetrySteps) return rc;
    // try the slabs again, from the home rows (the current state)
    r->full_steps = 0;
    ++r->info.rebuilds;
    const int b = build(*r, s);
    if (b == 1) return DDM_OK;
    if (b != DDM_OK) return b;
    r->full_mode = false;
    r->consecutive_repairs = 1;  // a repair in the next step returns to full-match mode
    r->info.full_mode = 0;
    r->info.buckets = (int32_t)r->R.nb;
    return DDM_OK;
  }
  const uint32_t par = r->step & 1u;
  const Header *h = reinterpret_cast<const Header *>(r->host);
  const ResCounters *c = reinterpret_cast<const ResCounters *>(r->host + sizeof(Header));
  const uint32_t flags = c->flags[par];
  const bool bs_full = h->pad[0] != 0;
  r->info.movers = c->movers[par];
  if (flags & kResBad) return DDM_E_INVAL;
  if (!flags && !bs_full) {
    r->consecutive_repairs = 0;
    *count = h->total;
    return DDM_OK;
  }
  // repair: every region back in region order, the count by the full call,
  // then new slabs (or none: full-matching mode from here on)
  if (launch_export(*r, par, r->home(0), r->home(1), r->home(2), r->home(3), s) != hipSuccess)
    return DDM_E_DEVICE;
  ++r->info.full_matches;
  const int rc = full_match(*r, s, count);
  if (rc != DDM_OK) return rc;
  if (bs_full || ++r->consecutive_repairs >= 2) {
    r->full_mode = true;
  } else {
    ++r->info.rebuilds;
    const int b = build(*r, s);
    if (b == 1)
      r->full_mode = true;
    else if (b != DDM_OK)
      return b;
  }
  if (r->full_mode) {
    r->full_steps = 0;
    r->info.full_mode = 1;
    r->info.buckets = 0;
  }
  return DDM_OK;
}

extern "C" int ddm_resident_export(ddm_resident *r, float *upd_lo, float *upd_hi, float *sub_lo,
                                   float *sub_hi, void *stream) {
  if (!r || r->pending) return DDM_E_INVAL;
  if ((r->n > 0 && (!upd_lo || !upd_hi)) || (r->m > 0 && (!sub_lo || !sub_hi)))
    return DDM_E_INVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (r->full_mode) {
    const size_t nu = (size_t)r->n * r->d * sizeof(float), ns = (size_t)r->m * r->d * sizeof(float);
    float *dst[4] = {upd_lo, upd_hi, sub_lo, sub_hi};
    for (int k = 0; k < 4 && e == hipSuccess; ++k) {
      const size_t bytes = k < 2 ? nu : ns;
      if (bytes) e = hipMemcpyAsync(dst[k], r->home(k), bytes, hipMemcpyDeviceToDevice, s);
    }
  } else {
    e = launch_export(*r, r->step & 1u, upd_lo, upd_hi, sub_lo, sub_hi, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? DDM_OK : DDM_E_DEVICE;
}

extern "C" int ddm_resident_get_info(const ddm_resident *r, ddm_resident_info *out) {
  if (!r || !out) return DDM_E_INVAL;
  *out = r->info;
  return DDM_OK;
}

extern "C" int ddm_resident_destroy(ddm_resident *r) {
  if (!r) return DDM_OK;
  if (r->pending && r->done) (void)hipEventSynchronize(r->done);
  if (r->done) (void)hipEventDestroy(r->done);
  if (r->host) (void)hipHostFree(r->host);
  delete r;
  return DDM_OK;
}

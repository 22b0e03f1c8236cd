// Bucketed sort-based matching (see bucket_path.h).
//
//   sample   min / max of the swept-axis lower coordinate over a pseudo-random
//            sample of regions;
//   plan     bucket(x) = clamp(floor((x - vmin) * scale), 0, nb - 1), a monotone
//            non-decreasing map, so every region of bucket b starts strictly
//            before every region of bucket b' > b;
//   count    validates every box, and per block of regions histograms the
//            buckets of the non-empty ones (block-major matrix); a region
//            whose upper coordinate maps to a later bucket than its lower one
//            may still be active in the buckets in between, so it is counted
//            into the boundary state of each of them (the sizes of Algorithm
//            6's SubSet[p] and UpdSet[p], taken at bucket boundaries);
//   scan     the matrix is transposed to bucket-major order and one
//            exclusive prefix sum over it, followed by the boundary-state
//            sizes, gives every block its output slot in every bucket, every
//            bucket's start and every boundary-state list's offset; the block
//            offsets are transposed back so that each block reads its own row;
//   scatter  writes one fixed-size record per non-empty region into its
//            bucket, and a copy into the boundary state of every later bucket
//            its interval may reach;
//   sweep    one workgroup per bucket: records to registers, then an LDS
//            counting sort of each kind into fine bins by a second monotone map
//            of the lower coordinate (order inside a bin is left arbitrary);
//            every region walks the other kind's entries in the bins from its
//            own lower to its own upper coordinate and keeps those whose lower
//            endpoint comes after its own and before its upper one (exact key
//            tests; at equal coordinates an update's lower endpoint precedes a
//            subscription's); boundary-state regions, whose lower endpoints
//            precede the whole bucket, walk from the first bin.  Each 1-D pair
//            is met exactly once, at the later of the two lower endpoints (the
//            pair Algorithm 4 reports at the earlier upper endpoint), and kept
//            if the boxes overlap on every other axis.
//
// A batch of instances runs through the same launches: each instance has its
// own bucket map, buckets, count matrix and blocks; blocks, buckets, sample
// blocks and transpose tiles are numbered over the whole batch and mapped
// back to their instance by small tables (a batch of one needs none).
#include "bucket_path.h"

#include <string.h>

#include <algorithm>
#include <atomic>

#include "bucket_dev.h"
#include "primitives.h"
#include "profile.h"

namespace ddm {

namespace {
std::atomic<int> g_sweep_axis{-1};
}  // namespace

void set_sweep_axis(int axis) { g_sweep_axis.store(axis, std::memory_order_relaxed); }
int sweep_axis() { return g_sweep_axis.load(std::memory_order_relaxed); }

namespace {

constexpr int kThreads = 1024;                 // count / scatter blocks
constexpr int kSampleThreads = 256;
constexpr uint32_t kSampleRows = 8192;         // rows per sample block (at most 256 blocks)
constexpr uint32_t kMaxSampleBlocks = 256;
// Floats per sample block partial: the number of valid boxes sampled, then
// for every axis k (input order) the least and greatest lower bound, the
// greatest upper bound and the sum of the extents hi - lo.
constexpr int kPartAxis = 4;
constexpr int kPart = 1 + kPartAxis * kBucketMaxDims;

// Combines partial b into a (slot 0 and the extents are sums, the others
// extremes).
__device__ __forceinline__ void part_merge(float (&a)[kPart], const float *b) {
  a[0] += b[0];
#pragma unroll
  for (int k = 0; k < kBucketMaxDims; ++k) {
    float *x = a + 1 + kPartAxis * k;
    const float *y = b + 1 + kPartAxis * k;
    x[0] = fminf(x[0], y[0]);
    x[1] = fmaxf(x[1], y[1]);
    x[2] = fmaxf(x[2], y[2]);
    x[3] += y[3];
  }
}

__device__ __forceinline__ void part_identity(float (&a)[kPart]) {
  const float inf = __int_as_float(0x7f800000);
  a[0] = 0.f;
#pragma unroll
  for (int k = 0; k < kBucketMaxDims; ++k) {
    a[1 + kPartAxis * k] = inf;
    a[2 + kPartAxis * k] = -inf;
    a[3 + kPartAxis * k] = -inf;
    a[4 + kPartAxis * k] = 0.f;
  }
}

// The partial reduced over a wave (result in every lane); axes from D on
// keep their identity values.
template <int D = kBucketMaxDims>
__device__ __forceinline__ void part_wave(float (&a)[kPart]) {
  a[0] = wave_sum(a[0]);
#pragma unroll
  for (int k = 0; k < (D < kBucketMaxDims ? D : kBucketMaxDims); ++k) {
    float *x = a + 1 + kPartAxis * k;
    x[0] = wave_min(x[0]);
    x[1] = wave_max(x[1]);
    x[2] = wave_max(x[2]);
    x[3] = wave_sum(x[3]);
  }
}

// Axis k of the sweep order (the swept axis first, the others after it in
// input order) as an input axis.
__device__ __forceinline__ uint32_t input_axis(uint32_t k, uint32_t axis) {
  return k == 0u ? axis : (k <= axis ? k - 1u : k);
}

// Puts input axis ``axis`` of a loaded box first and the others after it
// in their order, so that every kernel after the plan sweeps axis 0 of its
// boxes.
template <int D>
__device__ __forceinline__ void sweep_order(Box<D> &b, uint32_t axis) {
  if (D == 1 || axis == 0u) return;
  float l = b.lo[0], h = b.hi[0];
#pragma unroll
  for (int k = 1; k < D; ++k) {
    if ((uint32_t)k > axis) continue;
    const float tl = b.lo[k], th = b.hi[k];
    b.lo[k] = l;
    b.hi[k] = h;
    l = tl;
    h = th;
  }
  b.lo[0] = l;
  b.hi[0] = h;
}
// Sampled lower corners (swept axis, axis 1) the plan tries a grid on, the
// plan's workgroup size, and the mean slab walk (entries) from which rows
// are tried.
constexpr uint32_t kPlanPoints = 8192;
constexpr uint32_t kQLevelBits = 8;  // levels of the plan's quantisation measure
constexpr uint32_t kQLevels = 1u << kQLevelBits;
constexpr uint32_t kQPoints = 512;  // sampled corners it is taken on (one per plan thread)
constexpr int kPlanThreads = 512;
constexpr float kGridWalk = 2.0f;

// The sweep workgroup: at most kBucketCap records per bucket with 512 fine
// bins per kind (256 or 512 threads), or kBigBucketCap records with 1024
// bins per kind (1024 threads).
constexpr int kCap = (int)kBucketCap;
constexpr int kBigCap = (int)kBigBucketCap;

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Integer mixing function (xor-shift-multiply), used only to spread the
// sample positions.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

template <int D>
__device__ __forceinline__ Box<D> load_row(const float *__restrict__ lo,
                                           const float *__restrict__ hi, uint32_t row) {
  Box<D> b;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    b.lo[k] = global_ptr(lo)[(size_t)row * D + k];
    b.hi[k] = global_ptr(hi)[(size_t)row * D + k];
  }
  return b;
}

// The per-instance plan as the kernels see it: a device table for batches,
// the one plan by value otherwise, and the maps from global block, sample
// block, transpose tile and bucket numbers to instances.
struct View {
  const InstPlan *plan;  // null: a single instance, `one`
  InstPlan one;
  const uint32_t *blk_inst, *smp_inst, *bucket_inst;
  __device__ __forceinline__ InstPlan get(uint32_t i) const { return plan ? plan[i] : one; }
  __device__ __forceinline__ uint32_t of_blk(uint32_t x) const { return plan ? blk_inst[x] : 0u; }
  __device__ __forceinline__ uint32_t of_smp(uint32_t x) const { return plan ? smp_inst[x] : 0u; }
  __device__ __forceinline__ uint32_t of_bucket(uint32_t x) const {
    return plan ? bucket_inst[x] : 0u;
  }
};

// ---------------------------------------------------------------- sample

// Clears, before the count pass runs: the header, the boundary-state sizes
// and fill cursors (nb + 1 and nb words) and the per-instance totals.
struct Clear {
  Header *hdr;
  uint32_t *bs_size, *bs_cur;
  uint32_t *hits;  // per bucket: whether the counting sweep found pairs there
  uint32_t nb;
  unsigned long long *inst_total;
  uint32_t B;
  uint32_t *heavy;  // the heavy-bucket list's two counters
};

template <int D>
__global__ __launch_bounds__(kSampleThreads) void bk_sample_kernel(View V,
                                                                   float *__restrict__ part,
                                                                   float *__restrict__ pts,
                                                                   Clear clr) {
  {
    const uint32_t tid = blockIdx.x * kSampleThreads + threadIdx.x;
    const uint32_t stride = gridDim.x * kSampleThreads;
    if (tid < sizeof(Header) / sizeof(uint32_t)) reinterpret_cast<uint32_t *>(clr.hdr)[tid] = 0u;
    if (tid < 2 && clr.heavy) clr.heavy[tid] = 0u;
    for (uint32_t i = tid; i <= clr.nb; i += stride) {
      clr.bs_size[i] = 0u;
      if (i < clr.nb) {
        clr.bs_cur[i] = 0u;
        if (clr.hits) clr.hits[i] = 0u;
      }
    }
    if (clr.inst_total)
      for (uint32_t i = tid; i < clr.B; i += stride) clr.inst_total[i] = 0ull;
  }
  // per block, over the sampled valid non-empty boxes of the block's
  // instance, the partial described at kPart; the sampled lower corners of
  // every axis (input order) go to pts[i * D ..] for the plan and for
  // bucket splits
  constexpr int W = kSampleThreads / kWave;
  __shared__ float sred[W][kPart];
  const InstPlan I = V.get(V.of_smp(blockIdx.x));
  const uint32_t N = I.n + I.m;
  float v[kPart];
  part_identity(v);
  const uint32_t i = blockIdx.x * kSampleThreads + threadIdx.x;
  const uint32_t r =
      (uint32_t)(((unsigned long long)mix32(i * 0x9E3779B9u + 0x632BE5ABu) * N) >> 32);
  const bool upd = r < I.n;
  const Box<D> b = load_row<D>(upd ? I.ulo : I.slo, upd ? I.uhi : I.shi, upd ? r : r - I.n);
  bool empty;
  const uint32_t err = box_errors<D>(b, empty, I.closed);
  bool ok = !err && !empty;
#pragma unroll
  for (int k = 0; k < D; ++k) ok = ok && fabsf(b.lo[k]) <= 3.0e38f && fabsf(b.hi[k]) <= 3.0e38f;
  const float nan = __int_as_float(0x7fc00000);
  if (ok) {
    v[0] = 1.f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      v[1 + kPartAxis * k] = v[2 + kPartAxis * k] = b.lo[k];
      v[3 + kPartAxis * k] = b.hi[k];
      v[4 + kPartAxis * k] = b.hi[k] - b.lo[k];
    }
  }
#pragma unroll
  for (int k = 0; k < D; ++k) pts[(size_t)i * D + k] = ok ? b.lo[k] : nan;
  part_wave<D>(v);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0)
#pragma unroll
    for (int k = 0; k < kPart; ++k) sred[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 1; j < W; ++j) part_merge(v, sred[j]);
#pragma unroll
    for (int k = 0; k < kPart; ++k) part[blockIdx.x * kPart + k] = v[k];
  }
}

// The bucket map and quantisation parameters of instance I, reduced by the
// whole workgroup from the instance's sample partials: out[0] the slab map
// (nx = nb columns, one row), out[1] a grid of ny > 1 rows by axis 1 to try
// (out[1].ny = 1: none).  The grid's cells are about as long on axis 1 as
// on the swept axis, and its rows are at least eight mean axis-1 extents
// high, so that copies into later rows stay rare.
//
// The swept axis (axis < 0) is the input axis k with the fewest expected
// 1-D candidates, N^2 * (mean extent) / (range of lower bounds) for boxes
// spread over the range (Sec. 3: any axis gives the same pairs), unless that
// is not under half of axis 0's; axis >= 0 forces that axis (0 if it is not
// one of the instance's).  Axes 1, 2, ... of the plan are the other input
// axes in order.
template <int THREADS>
__device__ void block_plan(const float *__restrict__ part, const InstPlan &I, bool grid,
                           int force_axis, float (*sred)[kPart], BucketParams *out) {
  constexpr int W = THREADS / kWave;
  float v[kPart];
  part_identity(v);
  for (uint32_t i = threadIdx.x; i < I.nsmp; i += THREADS)
    part_merge(v, part + (size_t)(I.smp0 + i) * kPart);
  if (I.d <= 3)  // uniform: the other axes hold identity values
    part_wave<3>(v);
  else
    part_wave<kBucketMaxDims>(v);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0)
#pragma unroll
    for (int k = 0; k < kPart; ++k) sred[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll 1
    for (int j = 1; j < W; ++j) part_merge(v, sred[j]);
    const float c = v[0];
    const uint32_t d = I.d < (uint32_t)kBucketMaxDims ? I.d : (uint32_t)kBucketMaxDims;
    // the partial of input axis k, through LDS (the reduced partial is
    // indexed by axes chosen at run time)
#pragma unroll
    for (int k = 0; k < kPart; ++k) sred[0][k] = v[k];
    const float *st = sred[0];
    auto lo_min = [&](uint32_t k) { return st[1 + kPartAxis * k]; };
    auto lo_max = [&](uint32_t k) { return st[2 + kPartAxis * k]; };
    auto hi_max = [&](uint32_t k) { return st[3 + kPartAxis * k]; };
    auto ext_sum = [&](uint32_t k) { return st[4 + kPartAxis * k]; };
    uint32_t axis = force_axis >= 0 && (uint32_t)force_axis < d ? (uint32_t)force_axis : 0u;
    if (force_axis < 0 && c > 0.f) {
      auto cost = [&](uint32_t k) {
        const float range = lo_max(k) - lo_min(k);
        return range > 0.f ? ext_sum(k) / range : __int_as_float(0x7f800000);
      };
      float best = cost(0);
#pragma unroll 1
      for (uint32_t k = 1; k < d; ++k)
        if (cost(k) < 0.5f * best) {
          best = cost(k);
          axis = k;
        }
    }
    const uint32_t a0 = input_axis(0, axis), a1 = input_axis(1, axis), a2 = input_axis(2, axis);
    // in sweep order: swept axis lower-bound range and extent sum; axis 1's
    // range and extent sum; axes 1 and 2's ranges for the quantisation
    const float v0 = lo_min(a0), v1 = lo_max(a0), ext0 = ext_sum(a0);
    const float v4 = d >= 2 ? lo_min(a1) : 0.f, v5 = d >= 2 ? hi_max(a1) : 0.f;
    const float ext = d >= 2 ? ext_sum(a1) : 0.f;
    BucketParams q;
    q.split = nullptr;
    q.axis = axis;
    q.qenc = 0;
    q.qaxis = 1;
    q.nb = I.nb;
    q.vmin = 0.f;
    q.scale = 0.f;
    q.valid = 0;
    q.nx = I.nb;
    q.ny = 1;
    q.vmin1 = 0.f;
    q.scale1 = 0.f;
    for (uint32_t k = 0; k < 2; ++k) {
      q.qmin[k] = 0.f;
      q.qscale[k] = 0.f;  // every box quantises to 0: the pre-filter lets all pass
      if (k + 1 >= d) continue;
      const uint32_t ak = k == 0 ? a1 : a2;
      const float lo = lo_min(ak), hi = hi_max(ak);
      if (c > 0.f && hi > lo) {
        const float qs = 65535.0f / (hi - lo);
        if (qs > 0.f && qs <= 3.0e38f) {
          q.qmin[k] = lo;
          q.qscale[k] = qs;
        }
      }
    }
    BucketParams g = q;
    if (c > 0.f && v1 > v0 && I.nb > 0) {
      // the sample's extremes lie about (max - min) / c inside the true ones;
      // widening the map by two such gaps keeps the regions beyond them from
      // piling into the first and last bucket
      const float gap = 2.0f * (v1 - v0) / c;
      const float lo = v0 - gap, hi = v1 + gap;
      const float scale = (float)I.nb / (hi - lo);
      if (scale > 0.f && scale <= 3.0e38f && lo > -3.0e38f && hi < 3.0e38f) {
        q.vmin = lo;
        q.scale = scale;
        q.valid = 1;
      }
      // a walk in a slab meets about N * ext0 / (2 (hi - lo)) entries of the
      // other kind (ext0 the mean swept-axis extent); rows pay for their
      // extra plan, count and copy work only when that is a few
      const float walk = (float)(I.n + I.m) * (ext0 / c) / (2.0f * (hi - lo));
      if (q.valid && grid && I.d >= 2 && I.nb >= 4 && v5 > v4 && walk >= kGridWalk) {
        const float gap1 = 2.0f * (v5 - v4) / c;
        const float lo1 = v4 - gap1, hi1 = v5 + gap1;
        float t = sqrtf((float)I.nb * ((hi1 - lo1) / (hi - lo)));
        if (ext > 0.f) t = fminf(t, (hi1 - lo1) / (8.0f * (ext / c)));
        if (t >= 2.0f) {  // false for NaN
          const uint32_t ny = (uint32_t)fminf(t, (float)I.nb / 2.0f);
          const uint32_t nx = I.nb / ny;
          const float s0 = (float)nx / (hi - lo), s1 = (float)ny / (hi1 - lo1);
          if (ny >= 2 && s0 > 0.f && s0 <= 3.0e38f && s1 > 0.f && s1 <= 3.0e38f &&
              lo1 > -3.0e38f && hi1 < 3.0e38f) {
            g = q;
            g.scale = s0;
            g.nx = nx;
            g.ny = ny;
            g.vmin1 = lo1;
            g.scale1 = s1;
          }
        }
      }
    }
    out[0] = q;
    out[1] = g;
  }
  __syncthreads();
}


// One workgroup per instance: its bucket map and quantisation parameters,
// from block_plan and two measures on the sampled corners (below).  A grid
// (grid != 0, d >= 2) is kept if the corners' sum of squared cell counts,
// which grows as they crowd into fewer cells, is small enough: inputs whose
// axis-1 corners follow their swept-axis ones (which fill only a diagonal of
// the grid) keep the slabs.  LDS: 2 nb words with grid != 0.
// force_axis: the swept axis, or -1 to let the plan choose (block_plan).
__global__ __launch_bounds__(kPlanThreads) void bk_plan_kernel(const float *__restrict__ part,
                                                               const float *__restrict__ pts,
                                                               View V,
                                                               BucketParams *__restrict__ P,
                                                               uint32_t grid, int force_axis) {
  __shared__ float sred[kPlanThreads / kWave][kPart];
  __shared__ BucketParams shp[2];
  __shared__ unsigned long long ssq[3];
  __shared__ uint32_t qh[4][kQLevels];  // [2 axis + map][level]
  __shared__ uint32_t qsq[4];  // pairs of corners sharing a level, per map
  extern __shared__ uint32_t hist[];
  const InstPlan I = V.get(blockIdx.x);
  const uint32_t t = threadIdx.x;
  block_plan<kPlanThreads>(part, I, grid != 0u, force_axis, sred, shp);
  const BucketParams &q = shp[0], &g = shp[1];
  // the sampled lower corners on the swept axis and axis 1 (sweep order)
  constexpr int U = (int)(kPlanPoints / kPlanThreads);
  const uint32_t cnt = min(I.nsmp * (uint32_t)kSampleThreads, kPlanPoints);
  const uint32_t d = I.d;
  const float *pp = pts + (size_t)I.smp0 * kSampleThreads * d;
  // (and axis 2): all loads issued before any is used
  const uint32_t s0 = input_axis(0, q.axis), s1 = input_axis(d >= 2 ? 1 : 0, q.axis);
  const uint32_t s2 = input_axis(d >= 3 ? 2 : 0, q.axis);
  const float nan = __int_as_float(0x7fc00000);
  constexpr int UQ = (int)(kQPoints / kPlanThreads);
  float2 x[U];
  float z[UQ];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t i = (uint32_t)u * kPlanThreads + t;
    const bool in = d >= 2 && i < cnt;
    x[u] = in ? make_float2(pp[(size_t)i * d + s0], pp[(size_t)i * d + s1]) : make_float2(nan, nan);
    if (u < UQ) z[u] = in && d >= 3 ? pp[(size_t)i * d + s2] : nan;
  }
  // Two measures on the sampled corners, in one pass:
  // - the grid (g.ny > 1) is kept if its sum of squared cell counts is at
  //   most 5/4 of the slabs' and at most twice what S points spread evenly
  //   over nb cells give (S + S^2 / nb): a crowded grid would overflow cells,
  //   which cannot be split, where the slab buckets of a skewed input can;
  // - the other axes' quantisation is linear in the coordinate, unless the
  //   encoded form (about logarithmic) spreads the sampled lower bounds much
  //   better: the measure of a map is the number of pairs of kQPoints
  //   sampled corners that share one of its kQLevels levels, proportional to
  //   the chance that two boxes do, and the encoded map is taken where that
  //   is under half the linear one's.
  const bool try_grid = g.ny > 1;                    // uniform over the workgroup
  const bool qmeasure = d >= 2 && sred[0][0] > 0.f;  // uniform over the workgroup
  const uint32_t nb = I.nb;
  const uint32_t na = d >= 3 ? 2u : 1u;
  float e_min[2] = {0.f, 0.f}, e_scale[2] = {0.f, 0.f};
  if (qmeasure)
    for (uint32_t k = 0; k < 2; ++k) {
      const uint32_t ak = k == 0 ? s1 : s2;
      const uint32_t e0 = encode_coord(sred[0][1 + kPartAxis * ak]);
      const uint32_t e1 = encode_coord(sred[0][3 + kPartAxis * ak]);
      const float es = e1 > e0 ? 65535.0f / (float)(e1 - e0) : 0.f;
      e_min[k] = __uint_as_float(e0);
      e_scale[k] = es > 0.f && es <= 3.0e38f ? es : 0.f;
    }
  if (try_grid)
    for (uint32_t k = t; k < 2 * nb; k += kPlanThreads) hist[k] = 0u;
  if (qmeasure)
    for (uint32_t k = t; k < 4 * kQLevels; k += kPlanThreads) qh[k / kQLevels][k % kQLevels] = 0u;
  if (t < 3) ssq[t] = 0ull;
  if (t < 4) qsq[t] = 0u;
  __syncthreads();
  uint32_t points = 0;
  if (try_grid)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (x[u].x != x[u].x) continue;  // no valid box was sampled there
      ++points;
      atomicAdd(&hist[bucket_of(x[u].x, q.vmin, q.scale, nb)], 1u);
      const uint32_t a = bucket_of(x[u].x, g.vmin, g.scale, g.nx);
      const uint32_t c = bucket_of(x[u].y, g.vmin1, g.scale1, g.ny);
      atomicAdd(&hist[nb + a * g.ny + c], 1u);
    }
  constexpr uint32_t kShift = 16 - kQLevelBits;
  if (qmeasure)
#pragma unroll
    for (int u = 0; u < UQ; ++u)
#pragma unroll
      for (uint32_t k = 0; k < 2; ++k) {
        const float y = k == 0 ? x[u].y : z[u];
        if (k >= na || y != y) continue;  // no valid box was sampled there
        atomicAdd(&qh[2 * k][quant_lo(y, q.qmin[k], q.qscale[k], false) >> kShift], 1u);
        atomicAdd(&qh[2 * k + 1][quant_lo(y, e_min[k], e_scale[k], true) >> kShift], 1u);
      }
  __syncthreads();
  if (try_grid) {
    unsigned long long sq_slab = 0, sq_grid = 0;
    for (uint32_t k = t; k < nb; k += kPlanThreads) {
      sq_slab += (unsigned long long)hist[k] * hist[k];
      sq_grid += (unsigned long long)hist[nb + k] * hist[nb + k];
    }
    sq_slab = wave_sum(sq_slab);
    sq_grid = wave_sum(sq_grid);
    const unsigned long long pw = wave_sum((unsigned long long)points);
    if (lane_id() == 0) {
      atomicAdd(&ssq[0], sq_slab);
      atomicAdd(&ssq[1], sq_grid);
      atomicAdd(&ssq[2], pw);
    }
  }
  if (qmeasure) {  // wave w sums half of map w / 2 (maps beyond 2 na stay unused)
    static_assert(kPlanThreads / kWave == 8 && kQLevels % (2 * kWave) == 0, "map halves");
    const uint32_t m = (t / kWave) / 2u, k0 = (t / kWave) % 2u * (kQLevels / 2);
    uint32_t sq = 0;
    if (m < 2 * na)
      for (uint32_t k = k0 + (uint32_t)lane_id(); k < k0 + kQLevels / 2; k += kWave) {
        const uint32_t h = qh[m][k];
        sq += h * (h ? h - 1u : 0u);
      }
    sq = wave_sum(sq);
    if (lane_id() == 0 && m < 2 * na) atomicAdd(&qsq[m], sq);
  }
  __syncthreads();
  if (t == 0) {
    const unsigned long long S = ssq[2];
    const bool use_grid =
        try_grid && 4ull * ssq[1] <= 5ull * ssq[0] && ssq[1] <= 2ull * (S + S * S / nb);
    BucketParams out = shp[use_grid ? 1 : 0];
    uint32_t pairs_of[2] = {0u, 0u};  // the chosen map's measure per axis
    if (qmeasure)
      for (uint32_t k = 0; k < na; ++k) {
        pairs_of[k] = qsq[2 * k];
        if (e_scale[k] > 0.f && 2u * qsq[2 * k + 1] < qsq[2 * k]) {
          out.qenc |= 1u << k;
          out.qmin[k] = e_min[k];
          out.qscale[k] = e_scale[k];
          pairs_of[k] = qsq[2 * k + 1];
        }
      }
    // the pre-filter's axis (d >= 3): axis 2 on a grid, whose rows bound
    // axis 1 already; on slabs the axis whose levels fewer sampled pairs share
    out.qaxis = d >= 3 && (use_grid || pairs_of[1] < pairs_of[0]) ? 2u : 1u;
    P[blockIdx.x] = out;
  }
}

// ------------------------------------------------------ row groups

// Rows are read in groups of up to four consecutive rows of one kind of one
// instance, so that a full group of d-float rows is d 16-byte loads when the
// instance's arrays are 16-byte aligned.  An instance's groups 0 .. gu-1
// cover its updates, the rest its subscriptions.
struct Group {
  const float *lo, *hi;
  uint32_t row0, rows, r0;  // first row, rows in the group (<= 4), region index of row0
};

__device__ __forceinline__ Group group_of(uint32_t g, const InstPlan &I, uint32_t n_total) {
  Group q;
  const bool upd = g < I.gu;
  const uint32_t count = upd ? I.n : I.m;
  if (!upd) g -= I.gu;
  q.lo = upd ? I.ulo : I.slo;
  q.hi = upd ? I.uhi : I.shi;
  q.row0 = 4u * g;
  q.rows = min(4u, count - q.row0);
  q.r0 = upd ? I.u0 + q.row0 : n_total + I.s0 + q.row0;
  return q;
}

template <int D>
__device__ __forceinline__ void load_group(const Group &q, bool vec, Box<D> (&bx)[4]) {
  if (vec && q.rows == 4) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    const auto *l4 = global_ptr(reinterpret_cast<const v4f *>(q.lo + (size_t)q.row0 * D));
    const auto *h4 = global_ptr(reinterpret_cast<const v4f *>(q.hi + (size_t)q.row0 * D));
    float lf[4 * D], hf[4 * D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const v4f a = l4[i], b = h4[i];
      lf[4 * i] = a.x;
      lf[4 * i + 1] = a.y;
      lf[4 * i + 2] = a.z;
      lf[4 * i + 3] = a.w;
      hf[4 * i] = b.x;
      hf[4 * i + 1] = b.y;
      hf[4 * i + 2] = b.z;
      hf[4 * i + 3] = b.w;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int k = 0; k < D; ++k) {
        bx[r].lo[k] = lf[r * D + k];
        bx[r].hi[k] = hf[r * D + k];
      }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const bool ok = (uint32_t)r < q.rows;
        bx[r].lo[k] = ok ? global_ptr(q.lo)[(size_t)(q.row0 + r) * D + k] : 0.f;
        bx[r].hi[k] = ok ? global_ptr(q.hi)[(size_t)(q.row0 + r) * D + k] : 1.f;
      }
  }
}

// ------------------------------------------------------------ count pass

// Boundary-state copies are bounded before they are counted: a box that
// reaches one later cell counts its copy at once (at most one per box); a
// box that reaches more first claims them all on a 64-bit running total, and
// counts them only while that total stays within the buffer's capacity,
// otherwise it sets the fallback flag.  So a few boxes spanning the whole
// swept axis cannot cost one device atomic per cell, twice, before the
// sweep sees the overflow, and the 32-bit prefix sums over the sizes (at
// most n + m + the capacity) cannot wrap.  bs_size null (slab builds): no
// boundary state is counted.
template <int D>
__global__ __launch_bounds__(kThreads) void bk_count_kernel(
    uint32_t n_total, View V, const BucketParams *__restrict__ P, uint32_t *__restrict__ C,
    uint32_t *__restrict__ bs_size, uint32_t bs_cap, Header *__restrict__ hdr,
    int32_t *__restrict__ zero, uint32_t zero_count) {
  extern __shared__ uint32_t hist[];
  const uint32_t inst = V.of_blk(blockIdx.x);
  const InstPlan I = V.get(inst);
  const BucketParams p = P[inst];
  // the per-update output, cleared here for the sweep
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < zero_count; i += gridDim.x * kThreads)
    zero[i] = 0;
  const uint32_t nb = I.nb, lb = blockIdx.x - I.blk0;
  for (uint32_t b = threadIdx.x; b < nb; b += kThreads) hist[b] = 0;
  __syncthreads();
  const uint32_t g0 = lb * I.gpb, g1 = min(I.g, g0 + I.gpb);
  uint32_t err = 0;
  auto count = [&](auto tag) {
    constexpr bool GR = decltype(tag)::value;
    // the rows of a thread's next group are loaded before its current group
    // is counted, so that they are in flight meanwhile
    uint32_t g = g0 + threadIdx.x;
    Group qn = Group{};
    Box<D> bn[4];
    if (g < g1) {
      qn = group_of(g, I, n_total);
      load_group<D>(qn, I.vec != 0, bn);
    }
    for (; g < g1; g += kThreads) {
      const Group q = qn;
      Box<D> bx[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) bx[r] = bn[r];
      if (g + kThreads < g1) {
        qn = group_of(g + kThreads, I, n_total);
        load_group<D>(qn, I.vec != 0, bn);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if ((uint32_t)r >= q.rows) continue;
        sweep_order<D>(bx[r], p.axis);
        bool empty;
        err |= box_errors<D>(bx[r], empty, I.closed);
        if (empty) continue;
        const Cells<D> c = cells_of<D, GR>(bx[r], p);
        atomicAdd(&hist[cell_index<GR>(c.a0, c.c0, p)], 1u);
        for (uint32_t y = c.c0 + 1; y <= c.c1; ++y) atomicAdd(&hist[cell_index<GR>(c.a0, y, p)], 1u);
        if (!bs_size || c.a1 == c.a0) continue;
        const unsigned long long span = (unsigned long long)(c.a1 - c.a0) * (c.c1 - c.c0 + 1u);
        if (span > 1ull && atomicAdd(&hdr->bs_copies, span) + span > (unsigned long long)bs_cap) {
          atomicOr(&hdr->pad[0], 1u);
          atomicOr(&hdr->pad[1], kUnsplittable);
          continue;
        }
        for (uint32_t a = c.a0 + 1; a <= c.a1; ++a)
          for (uint32_t y = c.c0; y <= c.c1; ++y)
            atomicAdd(&bs_size[I.b0 + cell_index<GR>(a, y, p)], 1u);
      }
    }
  };
  if (D >= 2 && p.ny > 1)  // uniform
    count(GridTag<true>{});
  else
    count(GridTag<false>{});
  __syncthreads();
  uint32_t *row = C + I.cell0 + (size_t)lb * nb;
  for (uint32_t b = threadIdx.x; b < nb; b += kThreads) row[b] = hist[b];
  err = (__ballot(err & kErrNaN) ? kErrNaN : 0u) | (__ballot(err & kErrOrder) ? kErrOrder : 0u);
  if (err && lane_id() == 0) atomicOr(&hdr->err, err);
}

// Column prefix of every instance's block-major count matrix: for bucket j
// (local column lb) and block k, P[k][lb] = sum of C[k'][lb] over k' < k,
// written block-major like C, and the column total into tot[j].  One lane
// per bucket and block range: a workgroup takes kColBuckets consecutive
// buckets, and its kColRanges lane groups (two per wave) take consecutive
// ranges of blocks (consecutive lanes on consecutive columns, so every row
// access is coalesced) and combine their sums in LDS.
constexpr int kColWaves = 16;
constexpr int kColBuckets = kWave / 2;
constexpr int kColRanges = 2 * kColWaves;

// A bucket whose total exceeds ``cap`` records cannot be swept on chip: it
// sets the fallback flag, so that the scatter and the sweep stand down, and
// says whether splitting slab buckets could cure it (bp: the instances'
// bucket maps; a grid's cells are not split).
__global__ __launch_bounds__(kColWaves * kWave) void bk_colscan_kernel(
    const uint32_t *__restrict__ C, uint32_t *__restrict__ P, uint32_t *__restrict__ tot,
    View V, uint32_t nb_total, uint32_t cap, const BucketParams *__restrict__ bp,
    Header *__restrict__ hdr) {
  __shared__ uint32_t part[kColRanges][kColBuckets];
  const uint32_t col = threadIdx.x % kColBuckets, g = threadIdx.x / kColBuckets;  // g: range
  const uint32_t j = blockIdx.x * kColBuckets + col;
  uint32_t k0 = 0, k1 = 0, stride = 0, inst = 0;
  size_t base = 0;
  if (j < nb_total) {
    inst = V.of_bucket(j);
    const InstPlan I = V.get(inst);
    const uint32_t per = (I.nblk + kColRanges - 1) / kColRanges;
    k0 = min(I.nblk, g * per);
    k1 = min(I.nblk, k0 + per);
    stride = I.nb;
    base = I.cell0 + (size_t)(j - I.b0);
  }
  uint32_t sum = 0;
  for (uint32_t k = k0; k < k1; ++k) sum += C[base + (size_t)k * stride];
  part[g][col] = sum;
  __syncthreads();
  uint32_t run = 0;
  for (uint32_t v = 0; v < g; ++v) run += part[v][col];
  if (j < nb_total && g == kColRanges - 1) {
    tot[j] = run + sum;
    if (run + sum > cap) {
      atomicOr(&hdr->pad[0], 1u);
      atomicOr(&hdr->pad[1], bp[inst].ny <= 1u ? kSplittable : kUnsplittable);
    }
  }
  for (uint32_t k = k0; k < k1; ++k) {
    const size_t at = base + (size_t)k * stride;
    const uint32_t c = C[at];
    P[at] = run;
    run += c;
  }
}

// ---------------------------------------------------------- scatter pass

// Record (16 bytes): word 0 = encoded lower key (swept axis), 1 = encoded
// upper key, plus one for closed intervals (keys are integers, so x <= hi is
// x < enc(hi) + 1, and enc(+inf) + 1 does not wrap), 2 = region index
// (updates first), 3 = quantised bounds of the other axes (qword_of).
template <int D>
__device__ __forceinline__ void write_record(uint32_t *__restrict__ dst, const Box<D> &b,
                                             uint32_t r, const BucketParams &p, uint32_t closed,
                                             uint32_t row) {
  *reinterpret_cast<uint4 *>(dst) = make_uint4(encode_coord(b.lo[0]), encode_coord(b.hi[0]) + closed,
                                               r, qword_of<D>(b, p, row));
}

// Boundary-state copies of a box into the cells of the columns after its
// own that it overlaps, at positions handed out by the cells' cursors.
template <int D, bool GRID>
__device__ __forceinline__ void bs_copies(const Cells<D> &c, const Box<D> &b, uint32_t rid,
                                          const BucketParams &p, const InstPlan &I,
                                          const Offsets &O, uint32_t *__restrict__ bs_cur,
                                          uint32_t bs_cap, uint32_t *__restrict__ bs_rec) {
  for (uint32_t a = c.a0 + 1; a <= c.a1; ++a)
    for (uint32_t y = c.c0; y <= c.c1; ++y) {
      const uint32_t jg = I.b0 + cell_index<GRID>(a, y, p);
      const uint32_t pos = O.bs_begin(jg) + atomicAdd(&bs_cur[jg], 1u);
      if (pos < bs_cap) write_record<D>(bs_rec + (size_t)pos * 4, b, rid, p, I.closed, y);
    }
}

template <int D>
__global__ __launch_bounds__(kThreads) void bk_scatter_kernel(
    uint32_t n_total, View V, const BucketParams *__restrict__ P, Offsets O,
    const uint32_t *__restrict__ SB,
    uint32_t *__restrict__ bs_cur, uint32_t bs_cap, uint32_t *__restrict__ rec,
    uint32_t *__restrict__ bs_rec, const Header *__restrict__ hdr) {
  constexpr int RW = 4;
  extern __shared__ uint32_t cur[];
  if (hdr->pad[0]) return;  // uniform: the count pass gave up (boundary state)
  const uint32_t inst = V.of_blk(blockIdx.x);
  const InstPlan I = V.get(inst);
  const BucketParams p = P[inst];
  const uint32_t nb = I.nb, lb = blockIdx.x - I.blk0;
  const uint32_t *row = SB + I.cell0 + (size_t)lb * nb;
  for (uint32_t b = threadIdx.x; b < nb; b += kThreads) cur[b] = O.S[I.b0 + b] + row[b];
  __syncthreads();
  const uint32_t g0 = lb * I.gpb, g1 = min(I.g, g0 + I.gpb);
#pragma unroll 2
  for (uint32_t g = g0 + threadIdx.x; g < g1; g += kThreads) {
    const Group q = group_of(g, I, n_total);
    Box<D> bx[4];
    load_group<D>(q, I.vec != 0, bx);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if ((uint32_t)r >= q.rows) continue;
      sweep_order<D>(bx[r], p.axis);
      bool empty;
      (void)box_errors<D>(bx[r], empty, I.closed);
      if (empty) continue;
      const Cells<D> c = cells_of<D, true>(bx[r], p);
      for (uint32_t y = c.c0; y == c.c0 || y <= c.c1; ++y) {  // its own cell, then later rows
        const uint32_t slot = atomicAdd(&cur[c.a0 * p.ny + y], 1u);
        if (slot < O.rec_cap)
          write_record<D>(rec + (size_t)slot * RW, bx[r], q.r0 + r, p, I.closed, y);
      }
      bs_copies<D, true>(c, bx[r], q.r0 + r, p, I, O, bs_cur, bs_cap, bs_rec);
    }
  }
}

// Scatter with record pairs.  Random 16-byte stores are bound by their
// number, so two records of one bucket in the same aligned 32 bytes of the
// output are written together by one thread.  Records take their slots as
// in bk_scatter_kernel, one group per thread per round.  A record
// in an even slot s offers itself in its bucket's LDS mailbox (a tag, the
// pair index s / 2, claimed by compare-and-swap, and the record; a busy
// mailbox makes it a single store); after a barrier, the record in odd slot
// s + 1 takes the offer if the tag is its pair's and writes both (else it is
// written alone: its neighbour was another block's or wrote itself).  Offers
// left when the block ends (the last slot of its cell, even) are written
// alone.  Every record is written exactly once.  LDS: 24 bytes per bucket.
constexpr uint32_t kTagFree = 0xFFFFFFFFu;
constexpr uint32_t kPairScatterMaxBuckets = 6656;

template <int D>
__global__ __launch_bounds__(kThreads) void bk_scatter_pair_kernel(
    uint32_t n_total, View V, const BucketParams *__restrict__ P, Offsets O,
    const uint32_t *__restrict__ SB, uint32_t *__restrict__ bs_cur, uint32_t bs_cap,
    uint32_t *__restrict__ rec, uint32_t *__restrict__ bs_rec, const Header *__restrict__ hdr) {
  constexpr int RW = 4;
  extern __shared__ uint4 stash[];  // [max_nb] records, then tag[nb], cur[nb]
  if (hdr->pad[0]) return;  // uniform: the count pass gave up (boundary state)
  const uint32_t inst = V.of_blk(blockIdx.x);
  const InstPlan I = V.get(inst);
  const BucketParams p = P[inst];
  const uint32_t nb = I.nb, lb = blockIdx.x - I.blk0;
  uint32_t *tag = reinterpret_cast<uint32_t *>(stash + nb);
  uint32_t *cur = tag + nb;
  const uint32_t *row = SB + I.cell0 + (size_t)lb * nb;
  for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
    cur[b] = O.S[I.b0 + b] + row[b];
    tag[b] = kTagFree;
  }
  __syncthreads();
  const uint32_t g0 = lb * I.gpb, g1 = min(I.g, g0 + I.gpb);
  // One group per thread and round; the rows of the thread's group of the
  // next round are loaded at the start of this one, so that they are in
  // flight while this round's records take their slots.
  constexpr int G = 1;
  auto rounds = [&](auto mode) {
    constexpr bool GR = decltype(mode)::value;
    Group qn = Group{};  // rows == 0: no group
    Box<D> bn[4];
    if (g0 + threadIdx.x < g1) {
      qn = group_of(g0 + threadIdx.x, I, n_total);
      load_group<D>(qn, I.vec != 0, bn);
    }
    for (uint32_t base = g0; base < g1; base += G * kThreads) {  // uniform
      Group q[G];
      Box<D> bx[G][4];
      q[0] = qn;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        bx[0][r] = bn[r];
        sweep_order<D>(bx[0][r], p.axis);
      }
      qn = Group{};
      if (base + kThreads + threadIdx.x < g1) {
        qn = group_of(base + kThreads + threadIdx.x, I, n_total);
        load_group<D>(qn, I.vec != 0, bn);
      }
      uint32_t slot[G][4];  // odd slots still to collect, else ~0u
#pragma unroll
      for (int k = 0; k < G; ++k)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          slot[k][r] = ~0u;
          if ((uint32_t)r >= q[k].rows) continue;
          bool empty;
          (void)box_errors<D>(bx[k][r], empty, I.closed);
          if (empty) continue;
          const uint32_t rid = q[k].r0 + r;
          const Cells<D> c = cells_of<D, GR>(bx[k][r], p);
          const uint32_t b = cell_index<GR>(c.a0, c.c0, p);
          const uint32_t s = atomicAdd(&cur[b], 1u);
          bool alone = true;
          if ((s & 1u) == 0u) {
            if (atomicCAS(&tag[b], kTagFree, s >> 1) == kTagFree) {
              stash[b] = make_uint4(encode_coord(bx[k][r].lo[0]),
                                    encode_coord(bx[k][r].hi[0]) + I.closed, rid,
                                    qword_of<D>(bx[k][r], p, c.c0));
              alone = false;
            }
          } else {
            slot[k][r] = s;
            alone = false;
          }
          if (alone && s < O.rec_cap)
            write_record<D>(rec + (size_t)s * RW, bx[k][r], rid, p, I.closed, c.c0);
          for (uint32_t y = c.c0 + 1; y <= c.c1; ++y) {  // copies into later rows, alone
            const uint32_t sy = atomicAdd(&cur[cell_index<GR>(c.a0, y, p)], 1u);
            if (sy < O.rec_cap) write_record<D>(rec + (size_t)sy * RW, bx[k][r], rid, p, I.closed, y);
          }
          bs_copies<D, GR>(c, bx[k][r], rid, p, I, O, bs_cur, bs_cap, bs_rec);
        }
      __syncthreads();  // every offer of this round is in its mailbox
#pragma unroll
      for (int k = 0; k < G; ++k)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t s = slot[k][r];
          if (s == ~0u) continue;
          const uint32_t rid = q[k].r0 + r;
          const uint2 h = home_of<D, GR>(bx[k][r], p);
          const uint32_t b = h.x;
          const bool in = s < O.rec_cap;  // rec_cap is even: so is the pair's first slot
          if (tag[b] == (s >> 1)) {
            const uint4 even = stash[b];
            tag[b] = kTagFree;
            if (in) *reinterpret_cast<uint4 *>(rec + (size_t)(s - 1) * RW) = even;
          }
          if (in) write_record<D>(rec + (size_t)s * RW, bx[k][r], rid, p, I.closed, h.y);
        }
      __syncthreads();  // mailboxes are settled before the next round's offers
    }
  };
  if (D >= 2 && p.ny > 1)  // uniform
    rounds(GridTag<true>{});
  else
    rounds(GridTag<false>{});
  for (uint32_t b = threadIdx.x; b < nb; b += kThreads)  // offers without a partner here
    if (tag[b] != kTagFree && tag[b] < O.rec_cap / 2)
      *reinterpret_cast<uint4 *>(rec + (size_t)tag[b] * 2 * RW) = stash[b];
}

// Slab layout of a single instance (a resident simulation): every region
// goes, by its swept-axis lower coordinate, into its bucket's slab of cap
// slots, at the block's prefix within that bucket (from bk_colscan_kernel)
// plus an LDS cursor, as (region index, lower corner, upper corner); empty
// regions go to the extra slab nb.  Slots past cap are not written and set
// *overflow (the bucket's total is then above cap).
template <int D>
__global__ __launch_bounds__(kThreads) void bk_slab_scatter_kernel(
    View V, const BucketParams *__restrict__ P, const uint32_t *__restrict__ SB,
    const uint32_t *__restrict__ T, uint32_t *__restrict__ ids, float *__restrict__ lo,
    float *__restrict__ hi, uint32_t *__restrict__ cnt, uint32_t cap,
    uint32_t *__restrict__ overflow) {
  extern __shared__ uint32_t cur[];
  const InstPlan I = V.get(0);
  const BucketParams p = P[0];
  const uint32_t nb = I.nb, lb = blockIdx.x;
  const uint32_t *row = SB + (size_t)lb * nb;
  for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
    cur[b] = row[b];
    if (lb == 0) {
      cnt[b] = min(T[b], cap);
      if (T[b] > cap) atomicOr(overflow, 1u);
    }
  }
  __syncthreads();
  const uint32_t g0 = lb * I.gpb, g1 = min(I.g, g0 + I.gpb);
  for (uint32_t g = g0 + threadIdx.x; g < g1; g += kThreads) {
    const Group q = group_of(g, I, I.n);
    Box<D> bx[4];
    load_group<D>(q, I.vec != 0, bx);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if ((uint32_t)r >= q.rows) continue;
      bool empty;
      (void)box_errors<D>(bx[r], empty, 0u);
      uint32_t b, local;
      if (empty) {
        b = nb;
        local = atomicAdd(&cnt[nb], 1u);
      } else {
        b = bucket_of(bx[r].lo[0], p.vmin, p.scale, nb);
        local = atomicAdd(&cur[b], 1u);
      }
      if (local >= cap) {
        atomicOr(overflow, 1u);
        continue;
      }
      const size_t at = (size_t)b * cap + local;
      ids[at] = q.r0 + r;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        lo[at * D + k] = bx[r].lo[k];
        hi[at * D + k] = bx[r].hi[k];
      }
    }
  }
}

// Instance of every global block, sample block and bucket.
__device__ __forceinline__ uint32_t find_inst(const InstPlan *plan, uint32_t B, uint32_t x,
                                              int which) {
  // last instance whose first index (of the given kind) is <= x among those
  // that own at least one such index
  uint32_t lo = 0, hi = B;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    const InstPlan &I = plan[mid];
    const uint32_t first = which == 0 ? I.blk0 : which == 1 ? I.smp0 : I.b0;
    if (first <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__global__ void bk_expand_maps_kernel(const InstPlan *__restrict__ plan, uint32_t B,
                                      uint32_t *__restrict__ blk_inst, uint32_t nblk,
                                      uint32_t *__restrict__ smp_inst, uint32_t nsmp,
                                      uint32_t *__restrict__ bucket_inst, uint32_t nb) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < nblk; x += stride)
    blk_inst[x] = find_inst(plan, B, x, 0);
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < nsmp; x += stride)
    smp_inst[x] = find_inst(plan, B, x, 1);
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < nb; x += stride)
    bucket_inst[x] = find_inst(plan, B, x, 2);
}

// ------------------------------------------------------------ sweep pass

// Inverse of encode_coord (for non-NaN codes; -0 comes back as +0).
__device__ __forceinline__ float decode_coord(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// Whether intervals a = (al, ah) and b = (bl, bh), both non-empty, overlap:
// the larger lower bound below the smaller upper bound (at most it, for
// closed intervals).  For non-empty intervals this is the same as
// al < bh and bl < ah (<= for closed ones), with one comparison on the
// vector unit instead of four lane masks combined on the scalar unit.
__device__ __forceinline__ bool overlap(float al, float ah, float bl, float bh, uint32_t closed) {
  const float lo = fmaxf(al, bl), hi = fminf(ah, bh);
  return closed ? lo <= hi : lo < hi;
}

__device__ __forceinline__ uint32_t fine_of(float x, float vmin, float fscale, int fine) {
  float t = (x - vmin) * fscale;
  t = fminf(fmaxf(t, 0.0f), (float)(fine - 1));
  return (uint32_t)t;
}

// Two quantised intervals a = [alo, ahi] and b = [blo, bhi] pass the
// pre-filter iff alo <= bhi and blo <= ahi.  Stored one as an "entry" word
// alo | (65535 - ahi) << 16 and the other as a "walker" word
// bhi | (65535 - blo) << 16, both conditions are one saturating packed
// subtraction: entry -sat walker is zero in both halves exactly when
// alo - bhi <= 0 and blo - ahi <= 0.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t qdiff(uint32_t entry, uint32_t walker) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(
                                          __builtin_bit_cast(u16x2, entry),
                                          __builtin_bit_cast(u16x2, walker)));
}

// Pre-filter words (d >= 2): the 16-bit bounds of one other axis (the
// record word, qword_of) as above, the entry word lo | (65535 - hi) << 16
// and the walker word hi | (65535 - lo) << 16.
template <int DM1>
__device__ __forceinline__ uint32_t entry_word(uint32_t w) {
  return (w & 0xFFFFu) | ((65535u - (w >> 16)) << 16);
}

// The walker word of a region from its own entry word.
template <int DM1>
__device__ __forceinline__ uint32_t walker_from_entry(uint32_t e) {
  const uint32_t lq = e & 0xFFFFu, hq = 65535u - (e >> 16);
  return hq | ((65535u - lq) << 16);
}

template <int DM1>
__device__ __forceinline__ uint32_t walker_word(uint32_t w) {
  return walker_from_entry<DM1>(entry_word<DM1>(w));
}

// Padding of the per-bucket LDS arrays: the unrolled interior loop reads up
// to three entries past its range.
constexpr int kPad = 4;

// One walking region: keys, region index, pre-filter walker words.
template <int DM1>
struct Walker {
  uint32_t klo, khi, after_key, rid;
  uint32_t q;    // pre-filter walker word (d >= 2)
  uint32_t pos;  // LDS position of a bucket region, kNoPos for a boundary-state region
  bool upd;
  float c[4];    // heavy sweep: exact lower / upper bounds of axes 1 and 2
};
constexpr uint32_t kNoPos = 0xFFFFFFFFu;

// Pairs that pass the pre-filter wait in a small LDS queue for the exact
// test, which then runs for all of them at once after the walks, so that the
// latency of reading their coordinates overlaps; a full queue sends further
// pairs through the exact test at once.
constexpr int kQueue = 320;

// The sweep comes in three kinds.  kSlabSweep: slabs of a resident
// simulation; a pair beyond the queue's capacity gets its exact test at
// once, on coordinates read from the rows.  kLightSweep: packed buckets; a
// bucket whose pre-filter passes more pairs than the queue holds is not
// counted, but listed as heavy.  kHeavySweep: the listed buckets again, with
// the exact coordinates of their regions' axes 1 and 2 staged in LDS (one
// row read per region instead of two per pair) and, for per-update counts,
// the bucket's updates counted in LDS and flushed once each.
constexpr int kSlabSweep = 0;
constexpr int kLightSweep = 1;
constexpr int kHeavySweep = 2;

struct SweepCtx {
  InstPlan I;  // the bucket's instance: rows of its regions
  uint32_t n;  // updates over the batch (region indices below are updates)
  int32_t *per_update;
  const unsigned long long *pair_off;
  uint32_t *cursor;
  uint32_t *out_u, *out_s;
  uint2 *queue;     // LDS: (walker region, entry region) pairs awaiting the exact test
  uint32_t *queued; // LDS: number of pairs offered to the queue
  // d = 1 only (else unused): per LDS position of the bucket's updates, a
  // difference array of their pairs found in this bucket (count pass) or
  // their emission cursors (emitting pass); and, per update, the number of
  // its pairs found in its own bucket (written by the count pass, read by
  // the emitting pass), or null
  uint32_t *dl;
  uint32_t *own;
  // a grid cell (ny > 1): its row, and the row map of axis 1's lower bounds;
  // a pair counts here only if the larger of its two axis-1 lower bounds
  // falls in this row (both regions are also present in the cells of later
  // rows they both reach)
  uint32_t ny = 1, row = 0;
  float vmin1 = 0.f, scale1 = 0.f;
  // light sweep: set (LDS) once the bucket is found heavy; heavy sweep:
  // exact bounds (lo1, hi1, lo2, hi2) and per-update counts by LDS position
  uint32_t *heavy = nullptr;
  const float4 *xc = nullptr;
  uint32_t *cntl = nullptr;
  // the input axis swept, and where axes 1 and 2 of the sweep order sit in
  // an input row
  uint32_t axis = 0, k1 = 1, k2 = 2;
};

// The row test of a pair whose axis-1 lower bounds are ly and lx; the sweep
// takes its walks in a slab form (GRID = false, no test) and a grid form.
template <bool GRID>
__device__ __forceinline__ bool in_row(const SweepCtx &o, float ly, float lx) {
  return !GRID || bucket_of(fmaxf(ly, lx), o.vmin1, o.scale1, o.ny) == o.row;
}

// DM1 is d - 1 for d <= 3; DM1 = 3 stands for every d >= 4, whose records
// and pre-filter are those of d = 3 (axes 1 and 2) and whose exact test also
// reads axes 3 .. d-1 (extra_axes).  Axes held in the walkers' caches:
template <int DM1>
constexpr int kNearAxes = DM1 < 2 ? DM1 : 2;

// Exact coordinates of axes 1 and 2 (at most, in sweep order) of region
// rid, from its row.  PERM = false: the swept axis is input axis 0, so the
// offsets are known at compile time (the only form on the hot paths of the
// usual inputs); PERM = true reads them from the context.
template <int DM1, bool PERM = false>
__device__ __forceinline__ void other_axes(const SweepCtx &o, uint32_t rid, float (&lo)[2],
                                           float (&hi)[2]) {
  const bool upd = rid < o.n;
  const size_t row = upd ? rid - o.I.u0 : rid - o.n - o.I.s0;
  const size_t D = DM1 == 3 ? (size_t)o.I.d : (size_t)(DM1 + 1);  // floats per row
  const auto *L = global_ptr(upd ? o.I.ulo : o.I.slo) + row * D;
  const auto *H = global_ptr(upd ? o.I.uhi : o.I.shi) + row * D;
#pragma unroll
  for (int c = 0; c < kNearAxes<DM1>; ++c) {
    const uint32_t k = !PERM ? 1u + (uint32_t)c : (c == 0 ? o.k1 : o.k2);
    lo[c] = L[k];
    hi[c] = H[k];
  }
}

// Axes 3 .. d-1 of regions ry and rx (d >= 4; the pre-filter and the
// cached test cover axes 1 and 2): whether they overlap on all of them.
__device__ __forceinline__ bool extra_axes(const SweepCtx &o, uint32_t ry, uint32_t rx) {
  const uint32_t d = o.I.d;
  const bool uy = ry < o.n, ux = rx < o.n;
  const size_t y = uy ? ry - o.I.u0 : ry - o.n - o.I.s0;
  const size_t x = ux ? rx - o.I.u0 : rx - o.n - o.I.s0;
  const auto *yl = global_ptr(uy ? o.I.ulo : o.I.slo) + y * d;
  const auto *yh = global_ptr(uy ? o.I.uhi : o.I.shi) + y * d;
  const auto *xl = global_ptr(ux ? o.I.ulo : o.I.slo) + x * d;
  const auto *xh = global_ptr(ux ? o.I.uhi : o.I.shi) + x * d;
  bool hit = true;
  for (uint32_t j = 3; j < d; ++j) {
    const uint32_t k = input_axis(j, o.axis);
    hit = hit && overlap(yl[k], yh[k], xl[k], xh[k], o.I.closed);
  }
  return hit;
}

// A pair of walker y and entry j that passed the key and pre-filter tests:
// exact test on the other axes (d >= 2), then count or emit.
template <int DM1, int MODE, bool GR, int KIND>
__device__ __forceinline__ void visit(const Walker<DM1> &y, bool &have_y, float (&ylo)[2],
                                      float (&yhi)[2], uint32_t j,
                                      const uint32_t *__restrict__ RID, unsigned long long &hits,
                                      uint32_t &own, const SweepCtx &o) {
  if (KIND == kHeavySweep && DM1 > 0) {  // the exact test on staged coordinates
    const float4 x = o.xc[j];
    bool hit = overlap(y.c[0], y.c[1], x.x, x.y, o.I.closed);
    if (DM1 >= 2) hit = hit & overlap(y.c[2], y.c[3], x.z, x.w, o.I.closed);
    if (DM1 == 3 && hit) hit = extra_axes(o, y.rid, RID[j]);
    if (!hit || !in_row<GR>(o, y.c[0], x.x)) return;
    ++hits;
    if (MODE == 1) {
      if (y.upd)
        ++own;
      else
        atomicAdd(&o.cntl[j], 1u);
    } else if (MODE == 2) {
      const uint32_t rx = RID[j];
      const uint32_t uu = y.upd ? y.rid : rx;
      const unsigned long long slot = o.pair_off[uu] + atomicAdd(&o.cursor[uu], 1u);
      if (o.out_u) o.out_u[slot] = uu;  // null: rows are implied by the offsets
      o.out_s[slot] = (y.upd ? rx : y.rid) - o.n;
    }
    return;
  }
  const uint32_t rx = RID[j];
  if (DM1 > 0) {
    if (KIND == kLightSweep && *o.heavy) return;  // the heavy sweep counts this bucket
    const uint32_t at = atomicAdd(o.queued, 1u);
    if (at < (uint32_t)kQueue) {
      o.queue[at] = make_uint2(y.rid, rx);
      return;
    }
    if (KIND == kLightSweep) {
      *o.heavy = 1u;
      return;
    }
    if (!have_y) {
      have_y = true;
      other_axes<DM1>(o, y.rid, ylo, yhi);
    }
    float xlo[2], xhi[2];
    other_axes<DM1>(o, rx, xlo, xhi);
    bool hit = true;
#pragma unroll
    for (int c = 0; c < kNearAxes<DM1>; ++c)
      hit = hit & overlap(ylo[c], yhi[c], xlo[c], xhi[c], o.I.closed);
    if (DM1 == 3 && hit) hit = extra_axes(o, y.rid, rx);
    if (!hit || !in_row<GR>(o, ylo[0], xlo[0])) return;
  }
  ++hits;
  if (MODE == 1) {
    if (y.upd) {
      ++own;
    } else if (DM1 == 0) {  // +1 on update entry j, in LDS
      atomicAdd(&o.dl[j], 1u);
      atomicAdd(&o.dl[j + 1], 0xFFFFFFFFu);
    } else {
      atomicAdd(&o.per_update[rx], 1);
    }
  } else if (MODE == 2) {
    const uint32_t uu = y.upd ? y.rid : rx;
    const uint32_t sid = (y.upd ? rx : y.rid) - o.n;
    unsigned long long slot;
    if (DM1 == 0 && o.own) {
      // an update's row: first its pairs found in its own bucket (LDS
      // cursor of its entry), then those its boundary-state copies find
      if (!y.upd)
        slot = o.pair_off[uu] + atomicAdd(&o.dl[j], 1u);
      else if (y.pos != kNoPos)
        slot = o.pair_off[uu] + atomicAdd(&o.dl[y.pos], 1u);
      else
        slot = o.pair_off[uu] + o.own[uu] + atomicAdd(&o.cursor[uu], 1u);
    } else {
      slot = o.pair_off[uu] + atomicAdd(&o.cursor[uu], 1u);
    }
    if (o.out_u) o.out_u[slot] = uu;  // null: rows are implied by the offsets
    o.out_s[slot] = sid;
  }
}

// The exact test of a queued pair (ry walked, rx was met), then count or
// emit as visit() does.
template <int DM1, int MODE, bool GR, bool PERM>
__device__ __forceinline__ void resolve(uint32_t ry, uint32_t rx, unsigned long long &hits,
                                        const SweepCtx &o) {
  float ylo[2], yhi[2], xlo[2], xhi[2];
  other_axes<DM1, PERM>(o, ry, ylo, yhi);
  other_axes<DM1, PERM>(o, rx, xlo, xhi);
  bool hit = true;
#pragma unroll
  for (int c = 0; c < kNearAxes<DM1>; ++c)
    hit = hit & overlap(ylo[c], yhi[c], xlo[c], xhi[c], o.I.closed);
  if (DM1 == 3 && hit) hit = extra_axes(o, ry, rx);
  if (!hit || !in_row<GR>(o, ylo[0], xlo[0])) return;
  ++hits;
  const uint32_t uu = ry < o.n ? ry : rx, ss = ry < o.n ? rx : ry;
  if (MODE == 1) {
    atomicAdd(&o.per_update[uu], 1);
  } else if (MODE == 2) {
    const unsigned long long slot = o.pair_off[uu] + atomicAdd(&o.cursor[uu], 1u);
    if (o.out_u) o.out_u[slot] = uu;  // null: rows are implied by the offsets
    o.out_s[slot] = ss - o.n;
  }
}

// Zero iff entry word e passes the walker's pre-filter (d >= 2).
template <int DM1>
__device__ __forceinline__ uint32_t qfail(uint32_t e, uint32_t wq) {
  return DM1 > 0 ? qdiff(e, wq) : 0u;
}

__device__ __forceinline__ uint32_t min4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  return min(min(a, b), min(c, d));
}

// Walk of y over the other kind's entries [jA, jD) of the bucket.  Entries in
// [jA, jB) (the first fine bin) must come after y's lower endpoint
// (KLO >= after_key), entries in [jC, jD) (the last fine bin) must start
// before its upper endpoint (KLO < khi); entries of the bins in between
// satisfy both by the monotonicity of the fine-bin map.  The edge loop tests
// keys on the first and last bin; the interior loop reads four aligned entry
// words at a time, masks the ones outside the interior and runs only the
// pre-filter (skipping a chunk with one compare when none of the four
// passes).
template <int DM1, int MODE, bool GR, int KIND>
__device__ __forceinline__ void walk(const uint32_t *__restrict__ KLO,
                                     const uint32_t *__restrict__ RID,
                                     const uint32_t *__restrict__ Q, const Walker<DM1> &y,
                                     uint32_t jA, uint32_t jB, uint32_t jC, uint32_t jD,
                                     unsigned long long &hits, const SweepCtx &o) {
  uint32_t own = 0;
  bool have_y = false;
  float ylo[2] = {0.f, 0.f}, yhi[2] = {0.f, 0.f};
  // the first bin [jA, jB) and, if it is another one, the last bin
  // [jC, jD) are the edge entries, with key tests; the bins between,
  // [jB, jC), need the pre-filter alone and are read in aligned chunks of
  // four whose entries outside the range are masked off
  const bool split = jC > jB;
  const uint32_t e1 = (split ? jB : jD) - jA;
  const uint32_t e = e1 + (split ? jD - jC : 0u);
  for (uint32_t t = 0; t < e; ++t) {
    const uint32_t j = t < e1 ? jA + t : jC + (t - e1);
    // both LDS reads issued before either is needed
    const uint32_t k = KLO[j];
    const uint32_t fail = DM1 > 0 ? qfail<DM1>(Q[j], y.q) : 0u;
    if ((k >= y.after_key) & (k < y.khi) & (fail == 0u))
      visit<DM1, MODE, GR, KIND>(y, have_y, ylo, yhi, j, RID, hits, own, o);
  }
  if (!split) {
    // first and last bin coincide: the edge loop has seen every entry
  } else if (KIND == kHeavySweep && DM1 > 0 && DM1 <= 2 && MODE != 2) {
    // heavy bucket: the quantised pre-filter passes most entries, so every
    // interior entry gets the exact test on its staged bounds, four at a
    // time without branches; counts go to the walker (an update) or to the
    // entries' LDS counters (a subscription walking updates).
    // Both regions are non-empty on axes 1 and 2 (lower < upper, or <= for
    // closed boxes), so each axis' two tests are one: the larger lower
    // bound below the smaller upper bound.  In a grid cell that larger
    // axis-1 lower bound also decides the row the pair counts in.
    auto interior = [&](auto cl) {
      constexpr bool CL = decltype(cl)::value;
      auto exact = [&](uint32_t j) {
        const float4 x = o.xc[j];
        const float a0 = fmaxf(y.c[0], x.x), b0 = fminf(y.c[1], x.y);
        bool h = CL ? a0 <= b0 : a0 < b0;
        if (DM1 >= 2) {
          const float a1 = fmaxf(y.c[2], x.z), b1 = fminf(y.c[3], x.w);
          h = h & (CL ? a1 <= b1 : a1 < b1);
        }
        if (GR) h = h & (bucket_of(a0, o.vmin1, o.scale1, o.ny) == o.row);
        return h;
      };
      uint32_t j = jB;
      for (; j + 4 <= jC; j += 4) {
        const bool h0 = exact(j), h1 = exact(j + 1), h2 = exact(j + 2), h3 = exact(j + 3);
        const uint32_t c = (uint32_t)h0 + (uint32_t)h1 + (uint32_t)h2 + (uint32_t)h3;
        hits += c;
        if (MODE == 1) {
          if (y.upd) {
            own += c;
          } else if (c) {
            if (h0) atomicAdd(&o.cntl[j], 1u);
            if (h1) atomicAdd(&o.cntl[j + 1], 1u);
            if (h2) atomicAdd(&o.cntl[j + 2], 1u);
            if (h3) atomicAdd(&o.cntl[j + 3], 1u);
          }
        }
      }
      for (; j < jC; ++j) {
        if (!exact(j)) continue;
        ++hits;
        if (MODE == 1) {
          if (y.upd)
            ++own;
          else
            atomicAdd(&o.cntl[j], 1u);
        }
      }
    };
    if (o.I.closed)  // uniform
      interior(GridTag<true>{});
    else
      interior(GridTag<false>{});
  } else if (DM1 == 0) {
    if (MODE == 0) {
      hits += jC - jB;
    } else if (MODE == 1) {  // every interior entry matches: the range at once
      hits += jC - jB;
      if (y.upd) {
        own += jC - jB;
      } else {
        atomicAdd(&o.dl[jB], 1u);
        atomicAdd(&o.dl[jC], 0xFFFFFFFFu);
      }
    } else {
      for (uint32_t j = jB; j < jC; ++j) visit<DM1, MODE, GR, KIND>(y, have_y, ylo, yhi, j, RID, hits, own, o);
    }
  } else {
    // one aligned chunk of four: entries outside [jB, jC) get a non-zero
    // fail value when ``masked``
    auto chunk = [&](uint32_t j, bool masked) {
      const uint4 q4 = reinterpret_cast<const uint4 *>(Q)[j >> 2];
      uint32_t f0 = qfail<DM1>(q4.x, y.q), f1 = qfail<DM1>(q4.y, y.q);
      uint32_t f2 = qfail<DM1>(q4.z, y.q), f3 = qfail<DM1>(q4.w, y.q);
      if (masked) {
        f0 |= (j < jB || j >= jC) ? 1u : 0u;
        f1 |= (j + 1 < jB || j + 1 >= jC) ? 1u : 0u;
        f2 |= (j + 2 < jB || j + 2 >= jC) ? 1u : 0u;
        f3 |= (j + 3 < jB || j + 3 >= jC) ? 1u : 0u;
      }
      if (min4(f0, f1, f2, f3) == 0u) {
        if (f0 == 0u) visit<DM1, MODE, GR, KIND>(y, have_y, ylo, yhi, j, RID, hits, own, o);
        if (f1 == 0u) visit<DM1, MODE, GR, KIND>(y, have_y, ylo, yhi, j + 1, RID, hits, own, o);
        if (f2 == 0u) visit<DM1, MODE, GR, KIND>(y, have_y, ylo, yhi, j + 2, RID, hits, own, o);
        if (f3 == 0u) visit<DM1, MODE, GR, KIND>(y, have_y, ylo, yhi, j + 3, RID, hits, own, o);
      }
    };
    uint32_t j = jB & ~3u;
    if (j != jB || j + 4 > jC) {  // head chunk (partial)
      chunk(j, true);
      j += 4;
    }
    for (; j + 8 <= jC; j += 8) {  // two chunks per step: both reads in flight
      // a bucket found heavy is swept again by the heavy sweep: stop walking
      if (KIND == kLightSweep && *(volatile const uint32_t *)o.heavy) {
        j = jC;
        break;
      }
      const uint4 qa = reinterpret_cast<const uint4 *>(Q)[j >> 2];
      const uint4 qb = reinterpret_cast<const uint4 *>(Q)[(j >> 2) + 1];
      const uint32_t f0 = qfail<DM1>(qa.x, y.q), f1 = qfail<DM1>(qa.y, y.q);
      const uint32_t f2 = qfail<DM1>(qa.z, y.q), f3 = qfail<DM1>(qa.w, y.q);
      const uint32_t f4 = qfail<DM1>(qb.x, y.q), f5 = qfail<DM1>(qb.y, y.q);
      const uint32_t f6 = qfail<DM1>(qb.z, y.q), f7 = qfail<DM1>(qb.w, y.q);
      if (min(min4(f0, f1, f2, f3), min4(f4, f5, f6, f7)) == 0u) {
        chunk(j, false);
        chunk(j + 4, false);
      }
    }
    for (; j + 4 <= jC; j += 4) chunk(j, false);
    if (j < jC) chunk(j, true);  // tail chunk (partial)
  }
  if (MODE == 1 && own) {
    if (DM1 == 0 && y.pos != kNoPos) {  // a bucket update: into its LDS entry
      atomicAdd(&o.dl[y.pos], own);
      atomicAdd(&o.dl[y.pos + 1], 0u - own);
    } else if (KIND == kHeavySweep && y.pos != kNoPos) {
      atomicAdd(&o.cntl[y.pos], own);
    } else {
      atomicAdd(&o.per_update[y.rid], (int)own);
    }
  }
}

// d = 1 emission by rows.  One wave per update of the bucket collects, with
// ballots, the subscriptions it meets here: those of the bucket starting in
// [its lower key, its upper key) (the forward walk), those of the bucket
// starting before it and still active at its lower key (at most ``span``
// fine bins back), and the boundary-state subscriptions still active there
// (staged in LDS first).  These are the update's pairs found in its own
// bucket, in any order; ranked in LDS (ids in a row are distinct), they are
// written as the finished row when the update has no other pairs, otherwise
// at the start of its row in the staging array (the pairs its
// boundary-state copies find in later buckets follow them; a final row sort
// orders the whole row).  Then the boundary-state updates walk as usual and
// emit through device-wide cursors; subscriptions emit nothing.  If the
// bucket's boundary state holds more than kBsSubCap subscriptions, or a row
// more than kRowStage pairs, R.flag is set and the caller emits pair by pair
// instead.
template <int THREADS, int FINE>
__device__ __forceinline__ void emit_rows(
    const uint32_t *KLO, const uint32_t *KHI, const uint32_t *RID, const uint32_t *BIN,
    uint32_t *stage, uint32_t *BSH, uint32_t *BSR, uint32_t *nbsub, uint32_t *maxbsh,
    uint32_t span,
    float vmn, float fscale, uint32_t Cu, uint32_t nbs, const uint32_t *__restrict__ bsr,
    const RowEmit &R, unsigned long long &hits, const SweepCtx &o) {
  constexpr int W = THREADS / kWave;
  const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
  const uint32_t n = o.n;
  auto bin_begin = [&](uint32_t k) { return k ? BIN[k - 1] : 0u; };
  // (a) the boundary-state subscriptions, into LDS
  for (uint32_t i = (uint32_t)t; i < nbs; i += THREADS) {
    const uint4 r = reinterpret_cast<const uint4 *>(bsr)[i];
    if (r.z >= n) {
      const uint32_t at = atomicAdd(nbsub, 1u);
      if (at < kBsSubCap) {
        BSH[at] = r.y;
        BSR[at] = r.z;
      }
      atomicMax(maxbsh, r.y);
    }
  }
  __syncthreads();
  const uint32_t nsb = *nbsub, reach = *maxbsh;
  if (nsb > kBsSubCap) {  // uniform over the workgroup
    if (t == 0) atomicOr(R.flag, 1u);
    return;
  }
  // (b) one wave per bucket update.  The update's pair count and row offset
  // are read one row ahead, so that their latency overlaps the walk of the
  // row before.
  int cnt_next = 0;
  unsigned long long base_next = 0;
  if ((uint32_t)w < Cu) {
    const uint32_t r0 = RID[w];
    cnt_next = R.cnt[r0];
    base_next = o.pair_off[r0];
  }
  for (uint32_t up = (uint32_t)w; up < Cu; up += W) {
    const uint32_t ku = KLO[up], hu = KHI[up], ru = RID[up];
    const int cnt_u = cnt_next;
    const unsigned long long base = base_next;
    if (up + W < Cu) {
      const uint32_t rn = RID[up + W];
      cnt_next = R.cnt[rn];
      base_next = o.pair_off[rn];
    }
    const uint32_t fl = fine_of(decode_coord(ku), vmn, fscale, FINE);
    const uint32_t fh = fine_of(decode_coord(hu - o.I.closed), vmn, fscale, FINE);
    const uint32_t j0 = bin_begin(FINE + (fl > span ? fl - span : 0u));
    const uint32_t j1 = BIN[FINE + fh];
    uint32_t L = 0;
    auto append = [&](bool hit, uint32_t sid) {
      const uint64_t m = __ballot(hit);
      const uint32_t at = L + (uint32_t)__popcll(m & lanemask_lt());
      if (hit && at < kRowStage) stage[at] = sid;
      L += (uint32_t)__popcll(m);
    };
    // every lane reads (lanes past the end read the last entry and are
    // masked off), so that the reads of a chunk go out together and nothing
    // branches
    for (uint32_t j = j0; j < j1; j += kWave) {
      const uint32_t jj = min(j + (uint32_t)lane, j1 - 1u);
      const uint32_t k = KLO[jj], kh = KHI[jj], r = RID[jj];
      append(j + (uint32_t)lane < j1 && k < hu && (k >= ku || kh > ku), r - n);
    }
    // boundary-state subscriptions reach only the start of the bucket (they
    // start in an earlier one)
    for (uint32_t i = 0; ku < reach && i < nsb; i += kWave) {
      const uint32_t ii = min(i + (uint32_t)lane, nsb - 1u);
      const uint32_t bh = BSH[ii], br = BSR[ii];
      append(i + (uint32_t)lane < nsb && bh > ku, br - n);
    }
    if (L == 0) continue;
    if (L > kRowStage || L > (uint32_t)cnt_u) {  // uniform over the wave; never expected
      if (lane == 0) atomicOr(R.flag, 1u);
      continue;
    }
    if (lane == 0) hits += L;
    const uint32_t L4 = (L + 3) & ~3u;
    if ((uint32_t)lane < L4 - L) stage[L + lane] = 0xFFFFFFFFu;
    __builtin_amdgcn_wave_barrier();
    const bool full = (uint32_t)cnt_u == L;  // no pairs in later buckets
    uint32_t *ids = full ? R.ids : o.out_s;
    int2 *pairs = full ? reinterpret_cast<int2 *>(R.pairs) : nullptr;
    if (L <= kWave)
      sort_row<1>(stage, L, lane, ru, base, ids, pairs);
    else if (L <= 2 * kWave)
      sort_row<2>(stage, L, lane, ru, base, ids, pairs);
    else
      for (uint32_t i0 = 0; i0 < L; i0 += 4 * kWave)
        rank_row<4>(stage, L, L4, i0, lane, ru, base, ids, pairs);
    __builtin_amdgcn_wave_barrier();  // the row is read before the next one is staged
  }
  // (c) the boundary-state updates: the rest of their rows
  for (uint32_t i = (uint32_t)t; i < nbs; i += THREADS) {
    const uint4 yr = reinterpret_cast<const uint4 *>(bsr)[i];
    if (yr.z >= n) continue;
    Walker<0> y;
    y.klo = yr.x;
    y.khi = yr.y;
    y.rid = yr.z;
    y.pos = kNoPos;
    y.upd = true;
    y.after_key = 0u;
    y.q = 0u;
    const uint32_t jA = bin_begin(FINE);
    const uint32_t fh = fine_of(decode_coord(y.khi - o.I.closed), vmn, fscale, FINE);
    walk<0, 2, false, kLightSweep>(KLO, RID, nullptr, y, jA, jA, bin_begin(FINE + fh),
                                   BIN[FINE + fh], hits, o);
  }
}

// The sweep of bucket b (every kind; see SweepCtx).  heavy: the heavy-bucket
// list ([0] buckets listed by the count sweeps, [1] by the emitting ones,
// then the list), filled by the light sweep.
template <int DM1, int MODE, int CAP, int THREADS, int FINE, int KIND, bool MARK = false>
__device__ __forceinline__ void sweep_bucket(
    uint32_t b, const uint32_t *__restrict__ rec, const Offsets &O, const View &V,
    const uint32_t *__restrict__ bs_rec, uint32_t bs_cap, uint32_t n, Header *__restrict__ hdr,
    int32_t *__restrict__ per_update, const unsigned long long *__restrict__ pair_off,
    uint32_t *__restrict__ cursor, uint32_t *__restrict__ out_u, uint32_t *__restrict__ out_s,
    unsigned long long *__restrict__ total, unsigned long long *__restrict__ inst_total,
    const uint32_t *__restrict__ gate, uint32_t *__restrict__ own_cnt, const RowEmit &R,
    uint32_t *__restrict__ heavy, uint32_t *__restrict__ bucket_hits) {
  constexpr bool SLAB = KIND == kSlabSweep;
  constexpr bool HV = KIND == kHeavySweep && DM1 > 0;
  constexpr int ITEMS = CAP / THREADS;
  constexpr int W = THREADS / kWave;
  constexpr int NBINS = 2 * FINE;
  constexpr int BPT = NBINS / THREADS;  // bins per thread in the scan
  static_assert(NBINS % THREADS == 0, "bins must split evenly over the threads");
  // the bucket in LDS, in fine-bin order (updates first): lower and upper
  // key, region index and the pre-filter entry words of the other axes
  __shared__ uint32_t KLO[CAP + kPad];
  __shared__ uint32_t KHI[CAP + kPad];
  __shared__ uint32_t RID[CAP + kPad];
  __shared__ __align__(16) uint32_t Q[DM1 > 0 ? CAP + kPad : 4];
  __shared__ uint32_t BIN[NBINS];
  __shared__ float redf[2 * W + 2];
  __shared__ uint32_t red[W + 2];
  __shared__ unsigned long long red64[W];
  __shared__ uint2 queue[DM1 > 0 && !HV ? kQueue : 1];
  __shared__ uint32_t queued, heavy_flag;
  __shared__ float4 XC[HV ? CAP + kPad : 1];
  __shared__ uint32_t CNTL[HV && MODE == 1 ? CAP + kPad : 1];
  // d = 1: the per-position array DL of the count pass and of the
  // pair-by-pair emission, or, for the emission by rows, one row stage per
  // wave and the bucket's boundary-state subscriptions (upper key, region);
  // the two uses share the space
  constexpr bool kDL = DM1 == 0 && MODE != 0;
  constexpr bool kRows = DM1 == 0 && MODE == 2;
  constexpr uint32_t kStageWords = W * (kRowStage + kPad);
  constexpr uint32_t kRowsWords = kStageWords + 2 * kBsSubCap;
  constexpr uint32_t kDLWords = CAP + kPad;
  __shared__ __align__(16) uint32_t SCR[kRows ? (kRowsWords > kDLWords ? kRowsWords : kDLWords)
                                              : (kDL ? kDLWords : 1)];
  uint32_t *DL = SCR;
  __shared__ uint32_t nbsub, maxspan, maxbsh;
  // the swept input axis, read once at the start (a read of the instance's
  // parameters near the end, where it is first needed, would stall every
  // workgroup on its way out)
  __shared__ uint32_t swept;
  const bool rows = kRows && R.cnt != nullptr && own_cnt != nullptr;

  if (MODE == 2 && gate && *gate == 0u) return;  // uniform over the grid
  // the counting sweep found no pair here: the emitting one has nothing to do
  if (MODE == 2 && bucket_hits && bucket_hits[b] == 0u) return;  // uniform
  // the count pass gave up, or another bucket did not fit: the records may
  // be incomplete and the host falls back (uniform over the workgroup)
  if (!SLAB && hdr->pad[0]) return;
  const uint32_t inst = V.of_bucket(b);
  const InstPlan I = V.get(inst);
  uint32_t start, C, bs_begin, nbs;
  bool fits;
  if (SLAB) {
    start = b * O.cap;
    C = O.cnt[b];
    bs_begin = b * O.bs_slab;
    nbs = O.bs_cnt[b];
    fits = C <= (uint32_t)CAP && nbs <= O.bs_slab;
  } else {
    start = O.S[b];
    C = O.S[b + 1] - start;
    bs_begin = O.bs_begin(b);
    nbs = O.bs_begin(b + 1) - bs_begin;
    fits = O.bs_begin(O.nb) <= bs_cap && C <= (uint32_t)CAP && start + C <= O.rec_cap;
  }
  if (!fits) {  // uniform: the host falls back
    if (threadIdx.x == 0) {
      atomicOr(&hdr->pad[0], 1u);
      atomicOr(&hdr->pad[1], kUnsplittable);
    }
    return;
  }
  const int t = threadIdx.x;
  SweepCtx o{I, n, per_update, pair_off, cursor, out_u, out_s, queue, &queued, DL, own_cnt};
  o.heavy = &heavy_flag;
  o.xc = XC;
  o.cntl = CNTL;
  if (DM1 > 0 && !SLAB && O.P) {
    const BucketParams &bp = O.P[inst];
    if (bp.ny > 1) {
      o.ny = bp.ny;
      o.row = (b - I.b0) % bp.ny;
      o.vmin1 = bp.vmin1;
      o.scale1 = bp.scale1;
    }
  }

  // 1. records into registers (slot s = t + i * THREADS); value range
  uint4 rk[ITEMS];
  float vmn = __int_as_float(0x7f800000), vmx = -__int_as_float(0x7f800000);
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t s = t + i * THREADS;
    rk[i] = make_uint4(0u, 0u, 0u, 0u);
    if (s < C) {
      rk[i] = reinterpret_cast<const uint4 *>(rec)[start + s];
      const float x = decode_coord(rk[i].x);
      vmn = fminf(vmn, x);
      vmx = fmaxf(vmx, x);
    }
  }
  vmn = wave_min(vmn);
  vmx = wave_max(vmx);
  if (lane_id() == 0) {
    redf[2 * (t / kWave)] = vmn;
    redf[2 * (t / kWave) + 1] = vmx;
  }
  for (int k = t; k < NBINS; k += THREADS) BIN[k] = 0;
  if (kDL && !rows)
    for (int k = t; k < CAP + kPad; k += THREADS) DL[k] = 0;
  if (t == 0) {
    queued = 0;
    heavy_flag = 0;
    nbsub = 0;
    maxspan = 0;
    maxbsh = 0;
    swept = DM1 > 0 && !SLAB && O.P ? O.P[inst].axis : 0u;
  }
  if (HV && MODE == 1)
    for (int k = t; k < CAP + kPad; k += THREADS) CNTL[k] = 0;
  if (t < kPad) {  // defined values in the padding (never counted)
    KLO[CAP + t] = 0;
    if (DM1 > 0) Q[CAP + t] = 0;
  }
  __syncthreads();
  vmn = redf[0];
  vmx = redf[1];
#pragma unroll
  for (int w = 1; w < W; ++w) {
    vmn = fminf(vmn, redf[2 * w]);
    vmx = fmaxf(vmx, redf[2 * w + 1]);
  }
  float fscale = 0.f;
  if (vmx > vmn) {
    fscale = (float)FINE / (vmx - vmn);
    if (!(fscale <= 3.0e38f)) fscale = 0.f;
  }

  // 2. counting sort into fine bins, updates first: bin = kind * FINE + fine(lo)
  uint32_t key[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t s = t + i * THREADS;
    if (s < C) {
      const uint32_t f = fine_of(decode_coord(rk[i].x), vmn, fscale, FINE);
      key[i] = (rk[i].z >= n ? (uint32_t)FINE : 0u) + f;
      atomicAdd(&BIN[key[i]], 1u);
      if (rows && rk[i].z >= n)  // fine bins a subscription spans past its own
        atomicMax(&maxspan, fine_of(decode_coord(rk[i].y - I.closed), vmn, fscale, FINE) - f);
    }
  }
  __syncthreads();
  {
    uint32_t v[BPT], sum = 0;
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
      v[k] = BIN[t * BPT + k];
      sum += v[k];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan<uint32_t, THREADS>(sum, red, &tot);
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
      BIN[t * BPT + k] = run;
      run += v[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t s = t + i * THREADS;
    if (s < C) {
      const uint32_t qpos = atomicAdd(&BIN[key[i]], 1u);
      KLO[qpos] = rk[i].x;
      KHI[qpos] = rk[i].y;
      RID[qpos] = rk[i].z;
      if (DM1 > 0) Q[qpos] = entry_word<DM1>(rk[i].w);
      key[i] = qpos;
    }
  }
  if (HV) {  // the exact bounds of axes 1 and 2 of every region, one row read each
    o.axis = swept;
    o.k1 = input_axis(1, o.axis);
    o.k2 = input_axis(2, o.axis);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t s = t + i * THREADS;
      if (s < C) {
        float lo[2] = {0.f, 0.f}, hi[2] = {0.f, 0.f};
        if (o.axis == 0u)
          other_axes<DM1, false>(o, rk[i].z, lo, hi);
        else
          other_axes<DM1, true>(o, rk[i].z, lo, hi);
        XC[key[i]] = make_float4(lo[0], hi[0], lo[1], hi[1]);
      }
    }
  }
  __syncthreads();
  // BIN[k] is now the end of fine bin k; bin k starts at BIN[k - 1] (0 for k = 0)
  auto bin_begin = [&](uint32_t k) { return k ? BIN[k - 1] : 0u; };
  const uint32_t Cu = BIN[FINE - 1];  // updates occupy [0, Cu)

  // 3. the walks.  Walkers are the bucket's regions in bin order followed by
  //    its boundary-state regions; each wave takes chunks of 64 consecutive
  //    walkers in turn, so the lanes of a wave walk neighbouring, overlapping
  //    ranges and the boundary-state walkers are spread over all waves.
  unsigned long long hits = 0;
  const int lane = lane_id(), w = t / kWave;
  const uint32_t walkers = rows ? 0u : C + nbs;
  if (kRows && rows)
    emit_rows<THREADS, FINE>(KLO, KHI, RID, BIN, SCR + (size_t)w * (kRowStage + kPad),
                             SCR + kStageWords, SCR + kStageWords + kBsSubCap, &nbsub, &maxbsh,
                             maxspan, vmn, fscale, Cu, nbs, bs_rec + (size_t)bs_begin * 4, R,
                             hits, o);
  auto walks = [&](auto tag) {
    constexpr bool GR = decltype(tag)::value;
    for (uint32_t base = (uint32_t)w * kWave; base < walkers; base += (uint32_t)THREADS) {
      const uint32_t q = base + (uint32_t)lane;
      if (q >= walkers) continue;
      if (KIND == kLightSweep && DM1 > 0 && *(volatile const uint32_t *)&heavy_flag) break;
      Walker<DM1> y;
      uint32_t jA, jB;
      if (q < C) {  // a region of the bucket, from its own bin
        y.klo = KLO[q];
        y.khi = KHI[q];
        y.rid = RID[q];
        y.pos = q;
        y.upd = q < Cu;
        y.after_key = y.upd ? y.klo : y.klo + 1u;
        y.q = DM1 > 0 ? walker_from_entry<DM1>(Q[q]) : 0u;
        if (HV) {
          const float4 x = XC[q];
          y.c[0] = x.x;
          y.c[1] = x.y;
          y.c[2] = x.z;
          y.c[3] = x.w;
        }
        const uint32_t fl = fine_of(decode_coord(y.klo), vmn, fscale, FINE);
        const uint32_t other = y.upd ? (uint32_t)FINE : 0u;
        jA = bin_begin(other + fl);
        jB = BIN[other + fl];
      } else {  // a boundary-state region: every lower endpoint of the bucket comes after it
        const uint4 yr = reinterpret_cast<const uint4 *>(bs_rec)[bs_begin + (q - C)];
        y.klo = yr.x;
        y.khi = yr.y;
        y.rid = yr.z;
        y.pos = kNoPos;
        y.upd = yr.z < n;
        y.after_key = 0u;
        y.q = DM1 > 0 ? walker_word<DM1>(yr.w) : 0u;
        if (HV) {
          float lo[2] = {0.f, 0.f}, hi[2] = {0.f, 0.f};
          if (o.axis == 0u)
            other_axes<DM1, false>(o, y.rid, lo, hi);
          else
            other_axes<DM1, true>(o, y.rid, lo, hi);
          y.c[0] = lo[0];
          y.c[1] = hi[0];
          y.c[2] = lo[1];
          y.c[3] = hi[1];
        }
        jA = jB = bin_begin(y.upd ? (uint32_t)FINE : 0u);
      }
      const uint32_t fh = fine_of(decode_coord(y.khi - I.closed), vmn, fscale, FINE);
      const uint32_t last = (y.upd ? (uint32_t)FINE : 0u) + fh;
      walk<DM1, MODE, GR, KIND>(KLO, RID, Q, y, jA, jB, bin_begin(last), BIN[last], hits, o);
    }
    if (DM1 == 0 && MODE == 1) {
      // 4. d = 1: the pairs of each bucket update found here, by a prefix sum
      //    of the difference array, into the per-update counts
      __syncthreads();
      constexpr int PER = CAP / THREADS;
      const uint32_t j0 = (uint32_t)t * PER;
      uint32_t v[PER], sum = 0;
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        v[k] = DL[j0 + k];
        sum += v[k];
      }
      uint32_t tot;
      uint32_t run = block_exclusive_scan<uint32_t, THREADS>(sum, red, &tot);
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        run += v[k];
        const uint32_t j = j0 + k;
        if (j < Cu) {
          if (run) atomicAdd(&per_update[RID[j]], (int)run);
          if (own_cnt) own_cnt[RID[j]] = run;
        }
      }
    }
    if (HV && MODE == 1) {  // 4. the bucket's updates: their counts, once each
      __syncthreads();
      for (uint32_t j = t; j < Cu; j += THREADS)
        if (CNTL[j]) atomicAdd(&per_update[RID[j]], (int)CNTL[j]);
    } else if (DM1 > 0 && !HV) {  // 4. the exact test of the queued pairs, all at once
      __syncthreads();
      if (KIND == kLightSweep && heavy_flag) {  // uniform: listed, counted by the heavy sweep
        if (t == 0) {
          heavy[2 + atomicAdd(&heavy[MODE == 2 ? 1 : 0], 1u)] = b;
          if (MARK) bucket_hits[b] = 1u;  // it has pairs to emit
        }
      } else {
        const uint32_t nq = min(queued, (uint32_t)kQueue);
        // the swept axis is fetched here, not held through the walks
        o.axis = swept;
        o.k1 = input_axis(1, o.axis);
        o.k2 = input_axis(2, o.axis);
        if (o.axis == 0u) {  // uniform
          for (uint32_t k = t; k < nq; k += THREADS) {
            const uint2 pr = queue[k];
            resolve<DM1, MODE, GR, false>(pr.x, pr.y, hits, o);
          }
        } else {
          for (uint32_t k = t; k < nq; k += THREADS) {
            const uint2 pr = queue[k];
            resolve<DM1, MODE, GR, true>(pr.x, pr.y, hits, o);
          }
        }
      }
    }
  };
  if (DM1 > 0 && o.ny > 1)  // uniform
    walks(GridTag<true>{});
  else
    walks(GridTag<false>{});
  hits = wave_sum(hits);
  if (lane_id() == 0) red64[t / kWave] = hits;
  __syncthreads();
  if (t == 0) {
    unsigned long long tot = 0;
    for (int i = 0; i < W; ++i) tot += red64[i];
    if (tot) {
      atomicAdd(total, tot);
      if (inst_total) atomicAdd(&inst_total[inst], tot);
      // the emitting sweep visits only the buckets marked here (the marks
      // start cleared).  Only the counting sweeps of pair-mode calls mark
      // (MARK): the store's mere presence in the kernel made the sweeps of
      // the other calls a sixth slower.
      if (MARK) bucket_hits[b] = 1u;
    }
  }
}

// ------------------------------------------------------ split buckets

// Mean records per bucket of a split column, and the split plan's workgroup.
constexpr uint32_t kSplitTarget = 1024;
constexpr int kSplitThreads = 1024;

// After an attempt that failed only because slab buckets held more records
// than a sweep workgroup can (one instance; its map, the totals of its
// buckets and the input's validation are in the workspace): column a with
// more than cap records becomes ceil(T[a] / kSplitTarget) consecutive
// buckets, by a map linear in the encoded coordinate (see split_of), every
// other column one bucket.  The encoded range a split column is cut over is
// its nominal range under the map, narrowed to the sampled lower corners
// that fell in it (widened by 1/64 of their spread), so that a column whose
// boxes fill only part of it (the first one, stretched below the least
// coordinate, above all) is still cut where its boxes are; corners beyond
// the range land in its first or last bucket.  Writes the table and the new
// bucket map, the new bucket count into hdr->split_nb (0 if the failure was
// of another kind or more than max_nb buckets would be needed) and clears
// the header and what the next count pass accumulates.  LDS: 2 nb words.
__global__ __launch_bounds__(kSplitThreads) void bk_split_kernel(
    uint32_t *__restrict__ T, uint32_t nb, uint32_t cap, uint32_t max_nb,
    BucketParams *__restrict__ P, uint4 *__restrict__ split, Header *__restrict__ hdr,
    uint32_t *__restrict__ bs_cur, uint32_t *__restrict__ hits, uint32_t *__restrict__ heavy,
    const float *__restrict__ pts, uint32_t sampled, uint32_t d) {
  constexpr int PER = (int)(kMaxBuckets / kSplitThreads);
  __shared__ uint32_t red[kSplitThreads / kWave + 2];
  extern __shared__ uint32_t kext[];  // least and greatest sampled key per column
  const uint32_t t = threadIdx.x;
  const BucketParams p = P[0];
  const uint32_t why = hdr->pad[1];
  const bool splittable = (why & kSplittable) && !(why & kUnsplittable) && p.ny <= 1u && !p.split;
  uint32_t *kmin = kext, *kmax = kext + nb;
  for (uint32_t b = t; b < nb; b += kSplitThreads) {
    kmin[b] = 0xFFFFFFFFu;
    kmax[b] = 0u;
  }
  uint32_t k[PER], sum = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const uint32_t b = t * (uint32_t)PER + (uint32_t)i;
    k[i] = 0u;
    if (b < nb) {
      const uint32_t tb = T[b];
      k[i] = tb > cap ? (tb + kSplitTarget - 1u) / kSplitTarget : 1u;
    }
    sum += k[i];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan<uint32_t, kSplitThreads>(sum, red, &total);
  const bool ok = splittable && total <= max_nb;  // uniform
  if (ok) {
    // eight sampled corners per thread in flight at a time
    constexpr uint32_t kLoads = 8;
    for (uint32_t i0 = t; i0 < sampled; i0 += kLoads * kSplitThreads) {
      float xs[kLoads];
#pragma unroll
      for (uint32_t u = 0; u < kLoads; ++u) {
        const uint32_t i = i0 + u * kSplitThreads;
        xs[u] = i < sampled ? pts[(size_t)i * d + p.axis] : __int_as_float(0x7fc00000);
      }
      // a run of corners in one column (most of them, where the corners
      // crowd into a few columns) is folded in registers before its two
      // LDS atomics
      uint32_t col = 0xFFFFFFFFu, lo = 0xFFFFFFFFu, hi = 0u;
#pragma unroll
      for (uint32_t u = 0; u < kLoads; ++u) {
        const float x = xs[u];
        if (x != x) continue;  // no valid box was sampled there (or past the end)
        const uint32_t a = bucket_of(x, p.vmin, p.scale, p.nx), e = encode_coord(x);
        if (a != col) {
          if (col != 0xFFFFFFFFu) {
            atomicMin(&kmin[col], lo);
            atomicMax(&kmax[col], hi);
          }
          col = a;
          lo = e;
          hi = e;
        } else {
          lo = min(lo, e);
          hi = max(hi, e);
        }
      }
      if (col != 0xFFFFFFFFu) {
        atomicMin(&kmin[col], lo);
        atomicMax(&kmax[col], hi);
      }
    }
  }
  __syncthreads();  // every total of the failed attempt has been read
  if (ok) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const uint32_t b = t * (uint32_t)PER + (uint32_t)i;
      if (b >= nb) continue;
      const float x0 = p.vmin + (float)b / p.scale, x1 = p.vmin + (float)(b + 1u) / p.scale;
      uint32_t z = encode_coord(x0), z1 = encode_coord(x1);
      if (k[i] > 1u && kmax[b] >= kmin[b]) {
        const uint32_t w = (kmax[b] - kmin[b]) / 64u + 1u;
        const uint32_t lo = kmin[b] > w ? kmin[b] - w : 0u;
        const uint32_t hi = kmax[b] < 0xFFFFFFFFu - w ? kmax[b] + w : 0xFFFFFFFFu;
        if (lo > z && lo < z1) z = lo;
        if (hi < z1 && hi > z) z1 = hi;
      }
      const float sc = z1 > z ? (float)k[i] / (float)(z1 - z) : 0.f;
      split[b] = make_uint4(run, k[i], z, __float_as_uint(sc));
      run += k[i];
    }
    // the boundary-state sizes, the zero after them, the cursors and the
    // pair marks of the split layout (its bucket totals come from the next
    // column scan)
    for (uint32_t j = t; j <= total; j += kSplitThreads) {
      T[total + j] = 0u;
      if (j < total) {
        bs_cur[j] = 0u;
        hits[j] = 0u;
      }
    }
    if (t < 2) heavy[t] = 0u;
  }
  if (t == 0) {
    hdr->split_nb = ok ? total : 0u;
    if (ok) {
      hdr->pad[0] = 0u;
      hdr->pad[1] = 0u;
      hdr->bs_copies = 0ull;
      hdr->total = 0ull;
      BucketParams q = p;
      q.split = split;
      q.nb = total;
      P[0] = q;
    }
  }
}

template <int DM1, int MODE, int CAP, int THREADS, int FINE, bool SLAB = false, bool MARK = false>
__global__ __launch_bounds__(THREADS) void bk_sweep_kernel(
    const uint32_t *__restrict__ rec, Offsets O, View V, const uint32_t *__restrict__ bs_rec,
    uint32_t bs_cap, uint32_t n, Header *__restrict__ hdr, int32_t *__restrict__ per_update,
    const unsigned long long *__restrict__ pair_off, uint32_t *__restrict__ cursor,
    uint32_t *__restrict__ out_u, uint32_t *__restrict__ out_s,
    unsigned long long *__restrict__ total, unsigned long long *__restrict__ inst_total,
    const uint32_t *__restrict__ gate, uint32_t *__restrict__ own_cnt, RowEmit R,
    uint32_t *__restrict__ heavy, uint32_t *__restrict__ bucket_hits) {
  sweep_bucket<DM1, MODE, CAP, THREADS, FINE, SLAB ? kSlabSweep : kLightSweep, MARK>(
      blockIdx.x, rec, O, V, bs_rec, bs_cap, n, hdr, per_update, pair_off, cursor, out_u, out_s,
      total, inst_total, gate, own_cnt, R, heavy, bucket_hits);
}

// The heavy buckets the light sweep listed, a workgroup at a time.
template <int DM1, int MODE, int CAP, int THREADS, int FINE, bool MARK = false>
__global__ __launch_bounds__(THREADS) void bk_heavy_sweep_kernel(
    const uint32_t *__restrict__ rec, Offsets O, View V, const uint32_t *__restrict__ bs_rec,
    uint32_t bs_cap, uint32_t n, Header *__restrict__ hdr, int32_t *__restrict__ per_update,
    const unsigned long long *__restrict__ pair_off, uint32_t *__restrict__ cursor,
    uint32_t *__restrict__ out_u, uint32_t *__restrict__ out_s,
    unsigned long long *__restrict__ total, unsigned long long *__restrict__ inst_total,
    const uint32_t *__restrict__ gate, uint32_t *__restrict__ heavy,
    uint32_t *__restrict__ bucket_hits) {
  const uint32_t listed = heavy[MODE == 2 ? 1 : 0];
  for (uint32_t i = blockIdx.x; i < listed; i += gridDim.x) {  // uniform
    sweep_bucket<DM1, MODE, CAP, THREADS, FINE, kHeavySweep, MARK>(
        heavy[2 + i], rec, O, V, bs_rec, bs_cap, n, hdr, per_update, pair_off, cursor, out_u,
        out_s, total, inst_total, gate, nullptr, RowEmit{}, heavy, bucket_hits);
    __syncthreads();  // LDS is reused by the next bucket
  }
}

struct Ptrs {
  BucketParams *P;
  float *part;
  float *pts;
  uint32_t *C, *T, *S, *SB, *bs_cur, *rec, *bs_rec, *heavy, *hits;
  uint4 *split;
  void *scan_tmp;
  Offsets O;
  View V;
};

Ptrs pointers(const BucketArgs &a) {
  const BucketLayout &L = *a.L;
  char *ws = static_cast<char *>(a.ws);
  Ptrs p;
  p.P = reinterpret_cast<BucketParams *>(ws + L.params);
  p.part = reinterpret_cast<float *>(ws + L.sample_part);
  p.pts = reinterpret_cast<float *>(ws + L.sample_pts);
  p.C = reinterpret_cast<uint32_t *>(ws + L.counts);
  p.T = reinterpret_cast<uint32_t *>(ws + L.totals);
  p.S = reinterpret_cast<uint32_t *>(ws + L.offsets);
  p.SB = reinterpret_cast<uint32_t *>(ws + L.block_offsets);
  p.bs_cur = reinterpret_cast<uint32_t *>(ws + L.bs_cur);
  p.rec = reinterpret_cast<uint32_t *>(ws + L.rec);
  p.bs_rec = reinterpret_cast<uint32_t *>(ws + L.bs_rec);
  p.heavy = reinterpret_cast<uint32_t *>(ws + L.heavy);
  p.hits = reinterpret_cast<uint32_t *>(ws + L.hits);
  p.split = reinterpret_cast<uint4 *>(ws + L.split);
  p.scan_tmp = ws + L.scan_tmp;
  p.O.S = p.S;
  p.O.nb = L.nb;
  p.O.P = p.P;
  p.O.rec_cap = L.rec_cap;
  p.V = View{};
  if (L.B == 1) {
    p.V.plan = nullptr;
    p.V.one = L.inst[0];
  } else {
    p.V.plan = reinterpret_cast<const InstPlan *>(ws + L.plan);
    uint32_t *maps = reinterpret_cast<uint32_t *>(ws + L.maps);
    p.V.blk_inst = maps;
    p.V.smp_inst = maps + L.nblk;
    p.V.bucket_inst = maps + L.nblk + L.nsmp;
  }
  return p;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <int D>
void count_scatter_impl(const BucketArgs &a, hipStream_t s, int32_t *zero, uint32_t zero_count) {
  const BucketLayout &L = *a.L;
  Ptrs p = pointers(a);
  const size_t lds = (size_t)L.max_nb * sizeof(uint32_t);
  prof::mark(s, "bucket.count");
  bk_count_kernel<D><<<L.nblk, kThreads, lds, s>>>(L.n_total, p.V, p.P, p.C, p.T + L.nb, L.bs_cap,
                                                   a.hdr, zero, zero ? zero_count : 0u);
  prof::mark(s, "bucket.offsets");
  bk_colscan_kernel<<<(L.nb + kColBuckets - 1) / kColBuckets, kColWaves * kWave, 0, s>>>(
      p.C, p.SB, p.T, p.V, L.nb, bucket_cap(L.tune), p.P, a.hdr);
  (void)exclusive_scan_u32(p.T, p.S, 2 * (size_t)L.nb + 1, p.scan_tmp, s);
  prof::mark(s, "bucket.scatter");
  if (L.max_nb <= kPairScatterMaxBuckets)
    bk_scatter_pair_kernel<D><<<L.nblk, kThreads, (size_t)L.max_nb * 24, s>>>(
        L.n_total, p.V, p.P, p.O, p.SB, p.bs_cur, L.bs_cap, p.rec, p.bs_rec, a.hdr);
  else
    bk_scatter_kernel<D><<<L.nblk, kThreads, lds, s>>>(L.n_total, p.V, p.P, p.O, p.SB, p.bs_cur,
                                                       L.bs_cap, p.rec, p.bs_rec, a.hdr);
}

template <int D>
void prepare_impl(const BucketArgs &a, hipStream_t s) {
  const BucketLayout &L = *a.L;
  Ptrs p = pointers(a);
  const size_t lds = (size_t)L.max_nb * sizeof(uint32_t);
  prof::mark(s, "bucket.sample");
  const Clear clr{a.hdr, p.T + L.nb, p.bs_cur, p.hits, L.nb, a.inst_total, L.B, p.heavy};
  bk_sample_kernel<D><<<L.nsmp, kSampleThreads, 0, s>>>(p.V, p.part, p.pts, clr);
  const uint32_t grid = D >= 2 ? 1u : 0u;
  bk_plan_kernel<<<L.B, kPlanThreads, grid ? 2 * lds : 0, s>>>(p.part, p.pts, p.V, p.P, grid,
                                                               sweep_axis());
  count_scatter_impl<D>(a, s, a.zero, a.zero_count);
}

template <int DM1, int MODE, bool MARK = false>
void sweep_impl(const BucketArgs &a, int32_t *per_update, const unsigned long long *pair_off,
                uint32_t *cursor, uint32_t *out_u, uint32_t *out_s, unsigned long long *total,
                hipStream_t s, const uint32_t *gate) {
  const BucketLayout &L = *a.L;
  Ptrs p = pointers(a);
  // the light sweep of every bucket, then (d >= 2) the heavy sweep of those
  // it listed: two workgroups per CU (one with 1024 threads), looping
  const uint32_t hgrid = std::max<uint32_t>(1, std::min<uint32_t>(L.nb, 512));
  if (L.tune.sweep_threads == 1024) {
    bk_sweep_kernel<DM1, MODE, kBigCap, 1024, 1024, false, MARK><<<L.nb, 1024, 0, s>>>(
        p.rec, p.O, p.V, p.bs_rec, L.bs_cap, L.n_total, a.hdr, per_update, pair_off, cursor,
        out_u, out_s, total, a.inst_total, gate, a.own, a.rows, p.heavy, p.hits);
    if (DM1 > 0) prof::mark(s, MODE == 2 ? "bucket.sweep.emit.heavy" : "bucket.sweep.heavy");
    if (DM1 > 0)
      bk_heavy_sweep_kernel<DM1, MODE, kBigCap, 1024, 1024, MARK><<<(hgrid + 1) / 2, 1024, 0, s>>>(
          p.rec, p.O, p.V, p.bs_rec, L.bs_cap, L.n_total, a.hdr, per_update, pair_off, cursor,
          out_u, out_s, total, a.inst_total, gate, p.heavy, p.hits);
  } else if (L.tune.sweep_threads == 256) {
    bk_sweep_kernel<DM1, MODE, kCap, 256, 512, false, MARK><<<L.nb, 256, 0, s>>>(
        p.rec, p.O, p.V, p.bs_rec, L.bs_cap, L.n_total, a.hdr, per_update, pair_off, cursor,
        out_u, out_s, total, a.inst_total, gate, a.own, a.rows, p.heavy, p.hits);
    if (DM1 > 0) prof::mark(s, MODE == 2 ? "bucket.sweep.emit.heavy" : "bucket.sweep.heavy");
    if (DM1 > 0)
      bk_heavy_sweep_kernel<DM1, MODE, kCap, 256, 512, MARK><<<hgrid, 256, 0, s>>>(
          p.rec, p.O, p.V, p.bs_rec, L.bs_cap, L.n_total, a.hdr, per_update, pair_off, cursor,
          out_u, out_s, total, a.inst_total, gate, p.heavy, p.hits);
  } else {
    bk_sweep_kernel<DM1, MODE, kCap, 512, 512, false, MARK><<<L.nb, 512, 0, s>>>(
        p.rec, p.O, p.V, p.bs_rec, L.bs_cap, L.n_total, a.hdr, per_update, pair_off, cursor,
        out_u, out_s, total, a.inst_total, gate, a.own, a.rows, p.heavy, p.hits);
    if (DM1 > 0) prof::mark(s, MODE == 2 ? "bucket.sweep.emit.heavy" : "bucket.sweep.heavy");
    if (DM1 > 0)
      bk_heavy_sweep_kernel<DM1, MODE, kCap, 512, 512, MARK><<<hgrid, 512, 0, s>>>(
          p.rec, p.O, p.V, p.bs_rec, L.bs_cap, L.n_total, a.hdr, per_update, pair_off, cursor,
          out_u, out_s, total, a.inst_total, gate, p.heavy, p.hits);
  }
}

template <int D>
void build_slabs_impl(const BucketArgs &a, const SlabBuild &sb, hipStream_t s) {
  const BucketLayout &L = *a.L;
  Ptrs p = pointers(a);
  const size_t lds = (size_t)L.max_nb * sizeof(uint32_t);
  const Clear clr{a.hdr, p.T + L.nb, p.bs_cur, nullptr, L.nb, nullptr, L.B, nullptr};
  bk_sample_kernel<D><<<L.nsmp, kSampleThreads, 0, s>>>(p.V, p.part, p.pts, clr);
  // slabs of the swept axis 0 only: resident simulations move regions by it
  bk_plan_kernel<<<L.B, kPlanThreads, 0, s>>>(p.part, p.pts, p.V, p.P, 0u, 0);
  bk_count_kernel<D><<<L.nblk, kThreads, lds, s>>>(L.n_total, p.V, p.P, p.C, nullptr, 0u, a.hdr,
                                                   nullptr, 0u);
  bk_colscan_kernel<<<(L.nb + kColBuckets - 1) / kColBuckets, kColWaves * kWave, 0, s>>>(
      p.C, p.SB, p.T, p.V, L.nb, 0xFFFFFFFFu, p.P, a.hdr);  // the slabs report their own overflow
  (void)fill_u32(sb.cnt + L.nb, 0u, 1, s);
  bk_slab_scatter_kernel<D><<<L.nblk, kThreads, lds, s>>>(p.V, p.P, p.SB, p.T, sb.ids, sb.lo,
                                                          sb.hi, sb.cnt, sb.cap, sb.overflow);
}

template <int DM1>
void sweep_slabs_impl(const SlabSweep &w, hipStream_t s) {
  View V{};
  V.plan = nullptr;
  V.one = InstPlan{};
  V.one.ulo = V.one.slo = w.lo;
  V.one.uhi = V.one.shi = w.hi;
  V.one.nb = w.nb;
  V.one.d = (uint32_t)w.d;
  Offsets O{};
  O.S = nullptr;
  O.nb = w.nb;
  O.cnt = w.cnt;
  O.bs_cnt = w.bs_cnt;
  O.cap = w.cap;
  O.bs_slab = w.bs_slab;
  bk_sweep_kernel<DM1, 0, kCap, 512, 512, true><<<w.nb, 512, 0, s>>>(
      w.rec, O, V, w.bs_rec, 0u, w.nv, w.hdr, nullptr, nullptr, nullptr, nullptr, nullptr,
      &w.hdr->total, nullptr, nullptr, nullptr, RowEmit{}, nullptr, nullptr);
}

// Host-side plan of one instance; returns false if it does not fit.
bool plan_instance(const InstSpec &sp, int64_t u0, int64_t s0, const BucketTuning &t,
                   InstPlan &I) {
  const int64_t n = sp.n, m = sp.m;
  I = InstPlan{};
  I.ulo = sp.ulo;
  I.uhi = sp.uhi;
  I.slo = sp.slo;
  I.shi = sp.shi;
  I.vec = aligned16(sp.ulo) && aligned16(sp.uhi) && aligned16(sp.slo) && aligned16(sp.shi);
  I.closed = sp.closed ? 1u : 0u;
  I.u0 = (uint32_t)u0;
  I.n = (uint32_t)n;
  I.s0 = (uint32_t)s0;
  I.m = (uint32_t)m;
  const uint64_t gu = (uint64_t)(n + 3) / 4;
  const uint64_t gs = (uint64_t)(m + 3) / 4;
  I.gu = (uint32_t)gu;
  I.g = (uint32_t)(gu + gs);
  const uint64_t N = (uint64_t)(n + m);
  if (N == 0) return true;  // no blocks, buckets or samples
  const uint64_t nb = (N + t.target - 1) / t.target;
  if (nb > kMaxBuckets) return false;
  I.nb = (uint32_t)nb;
  const uint64_t per_blk = (uint64_t)kThreads * t.groups_per_thread;
  uint64_t nblk = (I.g + per_blk - 1) / per_blk;
  nblk = std::max<uint64_t>(1, std::min<uint64_t>(nblk, t.max_blocks));
  I.nblk = (uint32_t)nblk;
  I.gpb = (uint32_t)((I.g + nblk - 1) / nblk);
  const uint64_t nsmp = std::min<uint64_t>(kMaxSampleBlocks, (N + kSampleRows - 1) / kSampleRows);
  I.nsmp = (uint32_t)std::max<uint64_t>(1, nsmp);
  return true;
}

}  // namespace

bool bucket_path_supported(int d, const InstSpec *inst, int64_t B, const BucketTuning &t) {
  if (d < 1 || d > kBucketMaxDims || B < 1) return false;
  if (t.target < 64 || t.target > bucket_cap(t) * 3 / 4) return false;
  if (t.sweep_threads != 256 && t.sweep_threads != 512 && t.sweep_threads != 1024) return false;
  if (t.groups_per_thread < 1 || t.max_blocks < 1) return false;
  uint64_t cells = 0, nb = 0, N = 0;
  for (int64_t i = 0; i < B; ++i) {
    InstPlan I;
    if (!plan_instance(inst[i], 0, 0, t, I)) return false;
    cells += (uint64_t)I.nb * I.nblk;
    nb += I.nb;
    N += (uint64_t)(inst[i].n + inst[i].m);
  }
  return cells + nb + 1 < (1ull << 31) && N > 0 && N < (1ull << 31);
}

bool bucket_path_supported(int d, int64_t n, int64_t m) {
  const InstSpec sp{nullptr, nullptr, nullptr, nullptr, n, m};
  return bucket_path_supported(d, &sp, 1, BucketTuning{});
}

BucketLayout bucket_layout(const InstSpec *inst, int64_t B, int d, const BucketTuning &t) {
  BucketLayout L{};
  L.B = (uint32_t)B;
  L.tune = t;
  L.inst.resize((size_t)B);
  uint32_t blk = 0, smp = 0, bkt = 0;
  size_t cell = 0;
  int64_t u0 = 0, s0 = 0;
  for (int64_t i = 0; i < B; ++i) {
    InstPlan &I = L.inst[(size_t)i];
    plan_instance(inst[i], u0, s0, t, I);
    I.d = (uint32_t)d;
    u0 += inst[i].n;
    s0 += inst[i].m;
    I.blk0 = blk;
    I.smp0 = smp;
    I.b0 = bkt;
    I.cell0 = (uint32_t)cell;
    blk += I.nblk;
    smp += I.nsmp;
    bkt += I.nb;
    cell += (size_t)I.nb * I.nblk;
    L.max_nb = std::max(L.max_nb, I.nb);
  }
  L.nb = bkt;
  L.nblk = blk;
  L.nsmp = smp;
  L.cells = cell;
  L.n_total = (uint32_t)u0;
  L.m_total = (uint32_t)s0;
  const uint64_t N = (uint64_t)L.n_total + L.m_total;
  L.bs_cap = (uint32_t)(N / 2 + 4096);
  // d >= 2: room for copies into later grid rows (the plan keeps them to
  // about an eighth of the regions); the sweep sends the call back if they
  // are more
  L.rec_cap = (uint32_t)(d >= 2 ? (N + N / 4 + 4096) & ~(uint64_t)1 : (N + 1) & ~(uint64_t)1);
  L.rec_words = 4;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t o = at;
    at += align256(bytes);
    return o;
  };
  // a single instance keeps room for its overfull buckets to be split: at
  // most one more bucket per kSplitTarget records (bucket_split)
  L.nb_split = L.nb;
  if (B == 1 && L.nb > 0)
    L.nb_split = (uint32_t)std::min<uint64_t>(kMaxBuckets, L.nb + (N + kSplitTarget - 1) / kSplitTarget);
  const size_t cell_room = (size_t)L.nblk * L.nb_split;
  const size_t scanned = 2 * (size_t)L.nb_split + 1;  // bucket sizes + boundary-state sizes + 0
  L.params = take((size_t)B * sizeof(BucketParams));
  L.sample_part = take((size_t)std::max<uint32_t>(L.nsmp, 1) * kPart * sizeof(float));
  L.sample_pts = take((size_t)std::max<uint32_t>(L.nsmp, 1) * kSampleThreads * (size_t)d *
                      sizeof(float));
  L.counts = take(std::max(cell, cell_room) * sizeof(uint32_t));
  L.totals = take(scanned * sizeof(uint32_t));
  L.offsets = take(scanned * sizeof(uint32_t));
  L.block_offsets = take(std::max(cell, cell_room) * sizeof(uint32_t));
  L.scan_tmp = take(scan_temp_bytes(scanned));
  L.bs_cur = take((size_t)std::max<uint32_t>(L.nb_split, 1) * sizeof(uint32_t));
  L.rec = take((size_t)L.rec_cap * L.rec_words * sizeof(uint32_t));
  L.bs_rec = take((size_t)L.bs_cap * L.rec_words * sizeof(uint32_t));
  L.heavy = take(((size_t)L.nb_split + 2) * sizeof(uint32_t));
  L.hits = take((size_t)std::max<uint32_t>(L.nb_split, 1) * sizeof(uint32_t));
  L.split = take((size_t)std::max<uint32_t>(L.nb, 1) * sizeof(uint4));
  L.plan = take(B > 1 ? (size_t)B * sizeof(InstPlan) : 0);
  L.maps = take(B > 1 ? ((size_t)L.nblk + L.nsmp + L.nb) * sizeof(uint32_t) : 0);
  L.bytes = at;
  return L;
}

BucketLayout bucket_layout(const float *ulo, const float *uhi, int64_t n, const float *slo,
                           const float *shi, int64_t m, int d, bool closed) {
  const InstSpec sp{ulo, uhi, slo, shi, n, m, closed ? 1u : 0u};
  return bucket_layout(&sp, 1, d, BucketTuning{});
}

size_t plan_bytes(const BucketLayout &L) { return L.inst.size() * sizeof(InstPlan); }

hipError_t bucket_upload_plan(const BucketArgs &a, hipStream_t s, void *pinned) {
  const BucketLayout &L = *a.L;
  if (L.B <= 1) return hipSuccess;
  Ptrs p = pointers(a);
  InstPlan *plan = reinterpret_cast<InstPlan *>(static_cast<char *>(a.ws) + L.plan);
  const void *src = L.inst.data();
  if (pinned) {
    memcpy(pinned, L.inst.data(), plan_bytes(L));
    src = pinned;
  }
  hipError_t e = hipMemcpyAsync(plan, src, plan_bytes(L), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  const uint32_t most = std::max(std::max(L.nblk, L.nsmp), L.nb);
  const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((most + 255) / 256, 1024));
  bk_expand_maps_kernel<<<grid, 256, 0, s>>>(plan, L.B, const_cast<uint32_t *>(p.V.blk_inst),
                                             L.nblk, const_cast<uint32_t *>(p.V.smp_inst), L.nsmp,
                                             const_cast<uint32_t *>(p.V.bucket_inst), L.nb);
  return hipGetLastError();
}

hipError_t bucket_prepare(const BucketArgs &a, hipStream_t s) {
  switch (a.d) {
    case 1: prepare_impl<1>(a, s); break;
    case 2: prepare_impl<2>(a, s); break;
    case 3: prepare_impl<3>(a, s); break;
    case 4: prepare_impl<4>(a, s); break;
    case 5: prepare_impl<5>(a, s); break;
    case 6: prepare_impl<6>(a, s); break;
    case 7: prepare_impl<7>(a, s); break;
    default: prepare_impl<8>(a, s); break;
  }
  return hipGetLastError();
}

hipError_t bucket_split(const BucketArgs &a, hipStream_t s) {
  const BucketLayout &L = *a.L;
  if (L.B != 1 || L.nb == 0 || L.nb_split <= L.nb) return hipErrorInvalidValue;
  Ptrs p = pointers(a);
  prof::mark(s, "bucket.split");
  bk_split_kernel<<<1, kSplitThreads, 2 * (size_t)L.nb * sizeof(uint32_t), s>>>(
      p.T, L.nb, bucket_cap(L.tune), L.nb_split, p.P, p.split, a.hdr, p.bs_cur, p.hits, p.heavy,
      p.pts,
      L.inst[0].nsmp * (uint32_t)kSampleThreads, (uint32_t)a.d);
  return hipGetLastError();
}

BucketLayout split_layout(const BucketLayout &L, uint32_t nb) {
  BucketLayout R = L;
  R.nb = nb;
  R.max_nb = nb;
  R.inst[0].nb = nb;
  R.cells = (size_t)R.inst[0].nblk * nb;
  return R;
}

hipError_t bucket_prepare_split(const BucketArgs &a, hipStream_t s) {
  switch (a.d) {  // the output was cleared by the first attempt's count pass
    case 1: count_scatter_impl<1>(a, s, nullptr, 0u); break;
    case 2: count_scatter_impl<2>(a, s, nullptr, 0u); break;
    case 3: count_scatter_impl<3>(a, s, nullptr, 0u); break;
    case 4: count_scatter_impl<4>(a, s, nullptr, 0u); break;
    case 5: count_scatter_impl<5>(a, s, nullptr, 0u); break;
    case 6: count_scatter_impl<6>(a, s, nullptr, 0u); break;
    case 7: count_scatter_impl<7>(a, s, nullptr, 0u); break;
    default: count_scatter_impl<8>(a, s, nullptr, 0u); break;
  }
  return hipGetLastError();
}

hipError_t bucket_build_slabs(const BucketArgs &a, const SlabBuild &sb, hipStream_t s) {
  if (a.L->B != 1 || a.L->nb == 0 || sb.cap != kBucketCap) return hipErrorInvalidValue;
  switch (a.d) {
    case 1: build_slabs_impl<1>(a, sb, s); break;
    case 2: build_slabs_impl<2>(a, sb, s); break;
    case 3: build_slabs_impl<3>(a, sb, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t bucket_sweep_slabs(const SlabSweep &w, hipStream_t s) {
  if (w.nb == 0) return hipSuccess;
  if (w.cap != kBucketCap) return hipErrorInvalidValue;
  prof::mark(s, "resident.sweep");
  switch (w.d) {
    case 1: sweep_slabs_impl<0>(w, s); break;
    case 2: sweep_slabs_impl<1>(w, s); break;
    case 3: sweep_slabs_impl<2>(w, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t bucket_sweep(const BucketArgs &a, int mode, int32_t *per_update,
                        const unsigned long long *pair_off, uint32_t *cursor, uint32_t *out_u,
                        uint32_t *out_s, unsigned long long *total, hipStream_t s,
                        const uint32_t *gate, bool mark) {
  prof::mark(s, mode == 2 ? "bucket.sweep.emit" : "bucket.sweep");
#define DDM_SWEEP(DM1)                                                                     \
  if (mode == 0)                                                                           \
    sweep_impl<DM1, 0>(a, per_update, pair_off, cursor, out_u, out_s, total, s, gate);    \
  else if (mode == 1 && mark)                                                              \
    sweep_impl<DM1, 1, true>(a, per_update, pair_off, cursor, out_u, out_s, total, s, gate); \
  else if (mode == 1)                                                                      \
    sweep_impl<DM1, 1>(a, per_update, pair_off, cursor, out_u, out_s, total, s, gate);    \
  else                                                                                     \
    sweep_impl<DM1, 2>(a, per_update, pair_off, cursor, out_u, out_s, total, s, gate);
  switch (a.d) {
    case 1: DDM_SWEEP(0) break;
    case 2: DDM_SWEEP(1) break;
    case 3: DDM_SWEEP(2) break;
    default: DDM_SWEEP(3) break;
  }
#undef DDM_SWEEP
  return hipGetLastError();
}

}  // namespace ddm

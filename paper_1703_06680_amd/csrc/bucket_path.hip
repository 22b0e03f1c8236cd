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
#include "bucket_path.h"
#include "primitives.h"
#include "profile.h"

namespace ddm {
namespace {

constexpr int kThreads = 1024;                 // count / scatter blocks
constexpr uint32_t kMaxBlocks = 512;           // one resident round on 256 CUs
constexpr int kSampleBlocks = 256;
constexpr int kSampleThreads = 256;
constexpr uint32_t kTargetBucket = 1536;       // mean records per bucket

// The sweep workgroup: kCap records at most per bucket, kFine fine bins per
// kind.
constexpr int kSweepThreads = 512;
constexpr int kCap = 2048;
constexpr int kFine = 512;

struct BucketParams {
  float vmin;
  float scale;
  uint32_t nb;
  uint32_t valid;
};

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

__device__ __forceinline__ uint32_t bucket_of(float x, float vmin, float scale, uint32_t nb) {
  float t = (x - vmin) * scale;
  t = fminf(fmaxf(t, 0.0f), (float)(nb - 1));
  return (uint32_t)t;
}

template <int D>
struct Box {
  float lo[D];
  float hi[D];
};

template <int D>
__device__ __forceinline__ Box<D> load_box(const float *__restrict__ ulo,
                                           const float *__restrict__ uhi,
                                           const float *__restrict__ slo,
                                           const float *__restrict__ shi, uint32_t n, uint32_t r) {
  Box<D> b;
  const bool upd = r < n;
  const size_t row = (size_t)(upd ? r : r - n) * D;
  const float *lo = (upd ? ulo : slo) + row;
  const float *hi = (upd ? uhi : shi) + row;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    b.lo[k] = lo[k];
    b.hi[k] = hi[k];
  }
  return b;
}

// Error bits and emptiness of one box.
template <int D>
__device__ __forceinline__ uint32_t box_errors(const Box<D> &b, bool &empty) {
  uint32_t err = 0;
  empty = false;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float l = b.lo[k], h = b.hi[k];
    if (l != l || h != h) err |= kErrNaN;
    if (l > h) err |= kErrOrder;
    if (l == h) empty = true;
  }
  return err;
}

// Offsets produced by the one prefix sum: S[b * nblk + k] is block k's first
// slot in bucket b, S[cells] the number of records, S[cells + j] - S[cells]
// the first boundary-state entry of bucket j (j <= nb).
struct Offsets {
  const uint32_t *S;
  size_t cells;
  uint32_t nblk, nb;
  __device__ uint32_t records() const { return S[cells]; }
  __device__ uint32_t bucket_begin(uint32_t b) const { return S[(size_t)b * nblk]; }
  __device__ uint32_t bucket_end(uint32_t b) const {
    return b + 1 < nb ? S[(size_t)(b + 1) * nblk] : S[cells];
  }
  __device__ uint32_t bs_begin(uint32_t j) const { return S[cells + j] - S[cells]; }
};

// ---------------------------------------------------------------- sample

template <int D>
__global__ __launch_bounds__(kSampleThreads) void bk_sample_kernel(
    const float *__restrict__ ulo, const float *__restrict__ uhi, const float *__restrict__ slo,
    const float *__restrict__ shi, uint32_t n, uint32_t m, float4 *__restrict__ part) {
  __shared__ float smin[kSampleThreads / kWave], smax[kSampleThreads / kWave];
  __shared__ uint32_t scnt[kSampleThreads / kWave];
  const uint32_t N = n + m;
  float mn = __int_as_float(0x7f800000), mx = -__int_as_float(0x7f800000);
  uint32_t c = 0;
  const uint32_t i = blockIdx.x * kSampleThreads + threadIdx.x;
  const uint32_t r =
      (uint32_t)(((unsigned long long)mix32(i * 0x9E3779B9u + 0x632BE5ABu) * N) >> 32);
  const Box<D> b = load_box<D>(ulo, uhi, slo, shi, n, r);
  bool empty;
  const uint32_t err = box_errors<D>(b, empty);
  const float x = b.lo[0];
  if (!err && !empty && fabsf(x) <= 3.0e38f) {
    mn = x;
    mx = x;
    c = 1;
  }
  mn = wave_min(mn);
  mx = wave_max(mx);
  c = wave_sum(c);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    smin[w] = mn;
    smax[w] = mx;
    scnt[w] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kSampleThreads / kWave; ++k) {
      mn = fminf(mn, smin[k]);
      mx = fmaxf(mx, smax[k]);
      c += scnt[k];
    }
    part[blockIdx.x] = make_float4(mn, mx, __uint_as_float(c), 0.f);
  }
}

__global__ __launch_bounds__(kSampleThreads) void bk_plan_kernel(const float4 *__restrict__ part,
                                                                 uint32_t nb,
                                                                 BucketParams *__restrict__ P) {
  __shared__ float smin[kSampleThreads / kWave], smax[kSampleThreads / kWave];
  __shared__ uint32_t scnt[kSampleThreads / kWave];
  float mn = __int_as_float(0x7f800000), mx = -__int_as_float(0x7f800000);
  uint32_t c = 0;
  for (int i = threadIdx.x; i < kSampleBlocks; i += kSampleThreads) {
    const float4 p = part[i];
    const uint32_t pc = __float_as_uint(p.z);
    if (pc) {
      mn = fminf(mn, p.x);
      mx = fmaxf(mx, p.y);
      c += pc;
    }
  }
  mn = wave_min(mn);
  mx = wave_max(mx);
  c = wave_sum(c);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    smin[w] = mn;
    smax[w] = mx;
    scnt[w] = c;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 1; k < kSampleThreads / kWave; ++k) {
    mn = fminf(mn, smin[k]);
    mx = fmaxf(mx, smax[k]);
    c += scnt[k];
  }
  BucketParams q;
  q.nb = nb;
  q.vmin = 0.f;
  q.scale = 0.f;
  q.valid = 0;
  if (c && mx > mn) {
    const float scale = (float)nb / (mx - mn);
    if (scale > 0.f && scale <= 3.0e38f) {
      q.vmin = mn;
      q.scale = scale;
      q.valid = 1;
    }
  }
  *P = q;
}

// ------------------------------------------------------ row groups

// Rows are read in groups of four consecutive rows of one kind, so that a
// group of d-float rows is d aligned 16-byte loads.  Groups 0 .. Gu-1 cover the
// updates, the rest the subscriptions.
struct Group {
  const float *lo, *hi;
  uint32_t row0, rows, r0;  // first row, rows in the group (<= 4), region index of row0
};

__device__ __forceinline__ Group group_of(uint32_t g, uint32_t Gu, const float *ulo,
                                          const float *uhi, const float *slo, const float *shi,
                                          uint32_t n, uint32_t m) {
  Group q;
  if (g < Gu) {
    q.lo = ulo;
    q.hi = uhi;
    q.row0 = 4 * g;
    q.rows = min(4u, n - q.row0);
    q.r0 = q.row0;
  } else {
    q.lo = slo;
    q.hi = shi;
    q.row0 = 4 * (g - Gu);
    q.rows = min(4u, m - q.row0);
    q.r0 = n + q.row0;
  }
  return q;
}

template <int D>
__device__ __forceinline__ void load_group(const Group &q, bool vec, Box<D> (&bx)[4]) {
  if (vec && q.rows == 4) {
    const float4 *l4 = reinterpret_cast<const float4 *>(q.lo + (size_t)q.row0 * D);
    const float4 *h4 = reinterpret_cast<const float4 *>(q.hi + (size_t)q.row0 * D);
    float lf[4 * D], hf[4 * D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const float4 a = l4[i], b = h4[i];
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
        bx[r].lo[k] = ok ? q.lo[(size_t)(q.row0 + r) * D + k] : 0.f;
        bx[r].hi[k] = ok ? q.hi[(size_t)(q.row0 + r) * D + k] : 1.f;
      }
  }
}

// ------------------------------------------------------------ count pass

template <int D>
__global__ __launch_bounds__(kThreads) void bk_count_kernel(
    const float *__restrict__ ulo, const float *__restrict__ uhi, const float *__restrict__ slo,
    const float *__restrict__ shi, uint32_t n, uint32_t m, int vec,
    const BucketParams *__restrict__ P, uint32_t nb, uint32_t gpb, uint32_t *__restrict__ C,
    uint32_t *__restrict__ bs_size, Header *__restrict__ hdr) {
  extern __shared__ uint32_t hist[];
  const BucketParams p = *P;
  for (uint32_t b = threadIdx.x; b < nb; b += kThreads) hist[b] = 0;
  __syncthreads();
  const uint32_t Gu = (n + 3) / 4, G = Gu + (m + 3) / 4;
  const uint32_t g0 = blockIdx.x * gpb, g1 = min(G, g0 + gpb);
  uint32_t err = 0;
#pragma unroll 2
  for (uint32_t g = g0 + threadIdx.x; g < g1; g += kThreads) {
    const Group q = group_of(g, Gu, ulo, uhi, slo, shi, n, m);
    Box<D> bx[4];
    load_group<D>(q, vec != 0, bx);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if ((uint32_t)r >= q.rows) continue;
      bool empty;
      err |= box_errors<D>(bx[r], empty);
      if (empty) continue;
      const uint32_t b = bucket_of(bx[r].lo[0], p.vmin, p.scale, nb);
      atomicAdd(&hist[b], 1u);
      const uint32_t last = bucket_of(bx[r].hi[0], p.vmin, p.scale, nb);
      for (uint32_t j = b + 1; j <= last; ++j) atomicAdd(&bs_size[j], 1u);
    }
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < nb; b += kThreads) C[(size_t)blockIdx.x * nb + b] = hist[b];
  err = (__ballot(err & kErrNaN) ? kErrNaN : 0u) | (__ballot(err & kErrOrder) ? kErrOrder : 0u);
  if (err && lane_id() == 0) atomicOr(&hdr->err, err);
}

// out[c][r] = in[r][c] for a rows x cols row-major matrix, 64x64 LDS tiles.
__global__ __launch_bounds__(256) void transpose_kernel(const uint32_t *__restrict__ in,
                                                        uint32_t *__restrict__ out, uint32_t rows,
                                                        uint32_t cols) {
  __shared__ uint32_t tile[64][65];
  const uint32_t c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  const uint32_t tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (uint32_t j = ty; j < 64; j += 4) {
    const uint32_t r = r0 + j, c = c0 + tx;
    if (r < rows && c < cols) tile[j][tx] = in[(size_t)r * cols + c];
  }
  __syncthreads();
  for (uint32_t j = ty; j < 64; j += 4) {
    const uint32_t c = c0 + j, r = r0 + tx;
    if (c < cols && r < rows) out[(size_t)c * rows + r] = tile[tx][j];
  }
}

// ---------------------------------------------------------- scatter pass

// Record: word 0 = encoded lower key (swept axis), 1 = encoded upper key,
// 2 = region index (updates first), 3 = 0, then lo/hi of each other axis.
template <int D>
__device__ __forceinline__ void write_record(uint32_t *__restrict__ dst, const Box<D> &b,
                                             uint32_t r) {
  constexpr int RW = D == 1 ? 4 : 8;
  uint32_t w[8];
  w[0] = encode_coord(b.lo[0]);
  w[1] = encode_coord(b.hi[0]);
  w[2] = r;
  w[3] = 0;
#pragma unroll
  for (int k = 4; k < 8; ++k) w[k] = 0;
#pragma unroll
  for (int k = 1; k < D; ++k) {
    w[4 + 2 * (k - 1)] = __float_as_uint(b.lo[k]);
    w[5 + 2 * (k - 1)] = __float_as_uint(b.hi[k]);
  }
  uint4 *d4 = reinterpret_cast<uint4 *>(dst);
  d4[0] = make_uint4(w[0], w[1], w[2], w[3]);
  if (RW == 8) d4[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

template <int D>
__global__ __launch_bounds__(kThreads) void bk_scatter_kernel(
    const float *__restrict__ ulo, const float *__restrict__ uhi, const float *__restrict__ slo,
    const float *__restrict__ shi, uint32_t n, uint32_t m, int vec,
    const BucketParams *__restrict__ P, uint32_t gpb, Offsets O, const uint32_t *__restrict__ SB,
    uint32_t *__restrict__ bs_cur, uint32_t bs_cap, uint32_t *__restrict__ rec,
    uint32_t *__restrict__ bs_rec) {
  constexpr int RW = D == 1 ? 4 : 8;
  extern __shared__ uint32_t cur[];
  const BucketParams p = *P;
  const uint32_t nb = O.nb;
  for (uint32_t b = threadIdx.x; b < nb; b += kThreads) cur[b] = SB[(size_t)blockIdx.x * nb + b];
  __syncthreads();
  const uint32_t Gu = (n + 3) / 4, G = Gu + (m + 3) / 4;
  const uint32_t g0 = blockIdx.x * gpb, g1 = min(G, g0 + gpb);
#pragma unroll 2
  for (uint32_t g = g0 + threadIdx.x; g < g1; g += kThreads) {
    const Group q = group_of(g, Gu, ulo, uhi, slo, shi, n, m);
    Box<D> bx[4];
    load_group<D>(q, vec != 0, bx);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if ((uint32_t)r >= q.rows) continue;
      bool empty;
      (void)box_errors<D>(bx[r], empty);
      if (empty) continue;
      const uint32_t b = bucket_of(bx[r].lo[0], p.vmin, p.scale, nb);
      const uint32_t slot = atomicAdd(&cur[b], 1u);
      write_record<D>(rec + (size_t)slot * RW, bx[r], q.r0 + r);
      const uint32_t last = bucket_of(bx[r].hi[0], p.vmin, p.scale, nb);
      for (uint32_t j = b + 1; j <= last; ++j) {
        const uint32_t pos = O.bs_begin(j) + atomicAdd(&bs_cur[j], 1u);
        if (pos < bs_cap) write_record<D>(bs_rec + (size_t)pos * RW, bx[r], q.r0 + r);
      }
    }
  }
}

// ------------------------------------------------------------ sweep pass

// Inverse of encode_coord (for non-NaN codes; -0 comes back as +0).
__device__ __forceinline__ float decode_coord(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

__device__ __forceinline__ uint32_t fine_of(float x, float vmin, float fscale) {
  float t = (x - vmin) * fscale;
  t = fminf(fmaxf(t, 0.0f), (float)(kFine - 1));
  return (uint32_t)t;
}

// Walk of region y over other-kind entries [j, jend) of the bucket: keeps x
// when lo_x comes after lo_y (strictly, or on equal keys when y is the update
// and x the subscription; "after" always holds for boundary-state regions) and
// lo_x < hi_y, and the boxes overlap on the other axes.
template <int DM1, int MODE>
__device__ __forceinline__ uint32_t walk(const uint32_t *__restrict__ KLO,
                                         const uint32_t *__restrict__ RID,
                                         const float *__restrict__ CO, uint32_t j, uint32_t jend,
                                         const uint32_t *y, uint32_t after_key, uint32_t n,
                                         unsigned long long &hits,
                                         int32_t *__restrict__ per_update,
                                         const unsigned long long *__restrict__ pair_off,
                                         uint32_t *__restrict__ cursor, uint32_t *__restrict__ out_u,
                                         uint32_t *__restrict__ out_s) {
  // x counts iff after_key <= KLO[x] < khi, where after_key is klo_y for an
  // update y, klo_y + 1 for a subscription y and 0 for the boundary state.
  constexpr int CW = DM1 == 0 ? 1 : 2 * DM1;
  const uint32_t khi = y[1];
  const uint32_t ry = y[2];
  const bool y_upd = ry < n;
  float ylo[2] = {0.f, 0.f}, yhi[2] = {0.f, 0.f};
#pragma unroll
  for (int c = 0; c < DM1; ++c) {
    ylo[c] = __uint_as_float(y[4 + 2 * c]);
    yhi[c] = __uint_as_float(y[5 + 2 * c]);
  }
  uint32_t own = 0;
  for (; j < jend; j += 4) {
    uint32_t idx[4];
    bool hit[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      idx[u] = j + u < jend ? j + u : jend - 1;
      const uint32_t k = KLO[idx[u]];
      hit[u] = (j + u < jend) && k >= after_key && k < khi;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (DM1 == 1) {
        const float2 xc = *reinterpret_cast<const float2 *>(&CO[idx[u] * CW]);
        hit[u] = hit[u] && ylo[0] < xc.y && xc.x < yhi[0];
      } else if (DM1 == 2) {
        const float4 xc = *reinterpret_cast<const float4 *>(&CO[idx[u] * CW]);
        hit[u] = hit[u] && ylo[0] < xc.y && xc.x < yhi[0] && ylo[1] < xc.w && xc.z < yhi[1];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!hit[u]) continue;
      ++hits;
      if (MODE == 1) {
        if (y_upd)
          ++own;
        else
          atomicAdd(&per_update[RID[idx[u]]], 1);
      } else if (MODE == 2) {
        const uint32_t rx = RID[idx[u]];
        const uint32_t uu = y_upd ? ry : rx;
        const uint32_t sid = (y_upd ? rx : ry) - n;
        const unsigned long long slot = pair_off[uu] + atomicAdd(&cursor[uu], 1u);
        out_u[slot] = uu;
        out_s[slot] = sid;
      }
    }
  }
  return own;
}

template <int DM1, int MODE, int CAP, int THREADS>
__global__ __launch_bounds__(THREADS) void bk_sweep_kernel(
    const uint32_t *__restrict__ rec, Offsets O, const uint32_t *__restrict__ bs_rec,
    uint32_t bs_cap, uint32_t n, Header *__restrict__ hdr, int32_t *__restrict__ per_update,
    const unsigned long long *__restrict__ pair_off, uint32_t *__restrict__ cursor,
    uint32_t *__restrict__ out_u, uint32_t *__restrict__ out_s,
    unsigned long long *__restrict__ total) {
  constexpr int RW = DM1 == 0 ? 4 : 8;
  constexpr int NC = 2 * DM1;            // other-axis words per record
  constexpr int CW = DM1 == 0 ? 1 : NC;  // LDS words per element for coords
  constexpr int ITEMS = CAP / THREADS;
  constexpr int W = THREADS / kWave;
  constexpr int NBINS = 2 * kFine;
  constexpr int BPT = NBINS / THREADS;   // bins per thread in the scan
  static_assert(NBINS % THREADS == 0, "bins must split evenly over the threads");
  // the bucket in LDS, in fine-bin order (updates first): lower key, region
  // index and the other axes' lo/hi of every region
  __shared__ uint32_t KLO[CAP];
  __shared__ uint32_t RID[CAP];
  __shared__ __align__(16) float CO[DM1 == 0 ? 4 : CAP * CW];
  __shared__ uint32_t BIN[NBINS];
  __shared__ float redf[2 * W + 2];
  __shared__ uint32_t red[W + 2];
  __shared__ unsigned long long red64[W];

  const uint32_t b = blockIdx.x;
  const uint32_t nbs_total = O.bs_begin(O.nb);
  const uint32_t start = O.bucket_begin(b);
  const uint32_t C = O.bucket_end(b) - start;
  if (nbs_total > bs_cap || C > (uint32_t)CAP) {  // uniform: the host falls back
    if (threadIdx.x == 0) atomicOr(&hdr->pad[0], 1u);
    return;
  }
  const uint32_t bs_begin = O.bs_begin(b);
  const uint32_t nbs = O.bs_begin(b + 1) - bs_begin;
  const int t = threadIdx.x;

  // 1. own records into registers (slot s = t + i * THREADS); value range
  uint32_t rk[ITEMS][RW];
  float vmn = __int_as_float(0x7f800000), vmx = -__int_as_float(0x7f800000);
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t s = t + i * THREADS;
    if (s < C) {
      const uint4 *src = reinterpret_cast<const uint4 *>(rec + (size_t)(start + s) * RW);
      const uint4 a = src[0];
      rk[i][0] = a.x;
      rk[i][1] = a.y;
      rk[i][2] = a.z;
      rk[i][3] = a.w;
      if (RW == 8) {
        const uint4 c = src[1];
        rk[i][4 % RW] = c.x;
        rk[i][5 % RW] = c.y;
        rk[i][6 % RW] = c.z;
        rk[i][7 % RW] = c.w;
      }
      const float x = decode_coord(rk[i][0]);
      vmn = fminf(vmn, x);
      vmx = fmaxf(vmx, x);
    } else {
#pragma unroll
      for (int k = 0; k < RW; ++k) rk[i][k] = 0;
    }
  }
  vmn = wave_min(vmn);
  vmx = wave_max(vmx);
  if (lane_id() == 0) {
    redf[2 * (t / kWave)] = vmn;
    redf[2 * (t / kWave) + 1] = vmx;
  }
  for (int k = t; k < NBINS; k += THREADS) BIN[k] = 0;
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
    fscale = (float)kFine / (vmx - vmn);
    if (!(fscale <= 3.0e38f)) fscale = 0.f;
  }

  // 2. counting sort into fine bins, updates first: bin = kind * kFine + fine(lo)
  uint32_t key[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t s = t + i * THREADS;
    if (s < C) {
      key[i] = (rk[i][2] >= n ? kFine : 0u) + fine_of(decode_coord(rk[i][0]), vmn, fscale);
      atomicAdd(&BIN[key[i]], 1u);
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
      const uint32_t q = atomicAdd(&BIN[key[i]], 1u);
      KLO[q] = rk[i][0];
      RID[q] = rk[i][2];
#pragma unroll
      for (int c = 0; c < NC; ++c) CO[q * CW + c] = __uint_as_float(rk[i][4 + c]);
    }
  }
  __syncthreads();
  // BIN[k] is now the end of fine bin k; bin k starts at BIN[k - 1] (0 for k = 0)
  auto bin_begin = [&](uint32_t k) { return k ? BIN[k - 1] : 0u; };

  // 3. the walks: every region of the bucket, then the boundary state
  unsigned long long hits = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t s = t + i * THREADS;
    if (s < C) {
      const bool y_upd = rk[i][2] < n;
      const uint32_t fl = fine_of(decode_coord(rk[i][0]), vmn, fscale);
      const uint32_t fh = fine_of(decode_coord(rk[i][1]), vmn, fscale);
      const uint32_t other = y_upd ? kFine : 0u;
      const uint32_t own = walk<DM1, MODE>(KLO, RID, CO, bin_begin(other + fl), BIN[other + fh],
                                           rk[i], y_upd ? rk[i][0] : rk[i][0] + 1u, n, hits,
                                           per_update, pair_off, cursor, out_u, out_s);
      if (MODE == 1 && own) atomicAdd(&per_update[rk[i][2]], (int)own);
    }
  }
  for (uint32_t k = t; k < nbs; k += THREADS) {
    uint32_t y[8];
    const uint4 *src = reinterpret_cast<const uint4 *>(bs_rec + (size_t)(bs_begin + k) * RW);
    const uint4 a = src[0];
    y[0] = a.x;
    y[1] = a.y;
    y[2] = a.z;
    y[3] = a.w;
    y[4] = y[5] = y[6] = y[7] = 0;
    if (RW == 8) {
      const uint4 c = src[1];
      y[4] = c.x;
      y[5] = c.y;
      y[6] = c.z;
      y[7] = c.w;
    }
    const bool y_upd = y[2] < n;
    const uint32_t fh = fine_of(decode_coord(y[1]), vmn, fscale);
    const uint32_t other = y_upd ? kFine : 0u;
    const uint32_t own = walk<DM1, MODE>(KLO, RID, CO, bin_begin(other), BIN[other + fh], y, 0u,
                                         n, hits, per_update, pair_off, cursor, out_u, out_s);
    if (MODE == 1 && own) atomicAdd(&per_update[y[2]], (int)own);
  }
  hits = wave_sum(hits);
  if (lane_id() == 0) red64[t / kWave] = hits;
  __syncthreads();
  if (t == 0) {
    unsigned long long tot = 0;
    for (int i = 0; i < W; ++i) tot += red64[i];
    if (tot) atomicAdd(total, tot);
  }
}

struct Ptrs {
  BucketParams *P;
  float4 *part;
  uint32_t *C, *T, *S, *SB, *bs_cur, *rec, *bs_rec;
  void *scan_tmp;
  Offsets O;
};

Ptrs pointers(const BucketArgs &a) {
  const BucketLayout &L = a.L;
  char *ws = static_cast<char *>(a.ws);
  Ptrs p;
  p.P = reinterpret_cast<BucketParams *>(ws + L.params);
  p.part = reinterpret_cast<float4 *>(ws + L.sample_part);
  p.C = reinterpret_cast<uint32_t *>(ws + L.counts);
  p.T = reinterpret_cast<uint32_t *>(ws + L.transposed);
  p.S = reinterpret_cast<uint32_t *>(ws + L.offsets);
  p.SB = reinterpret_cast<uint32_t *>(ws + L.block_offsets);
  p.bs_cur = reinterpret_cast<uint32_t *>(ws + L.bs_cur);
  p.rec = reinterpret_cast<uint32_t *>(ws + L.rec);
  p.bs_rec = reinterpret_cast<uint32_t *>(ws + L.bs_rec);
  p.scan_tmp = ws + L.scan_tmp;
  p.O.S = p.S;
  p.O.cells = (size_t)L.nb * L.nblk;
  p.O.nblk = L.nblk;
  p.O.nb = L.nb;
  return p;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <int D>
void prepare_impl(const BucketArgs &a, hipStream_t s) {
  const BucketLayout &L = a.L;
  Ptrs p = pointers(a);
  const size_t cells = p.O.cells;
  const size_t lds = (size_t)L.nb * sizeof(uint32_t);
  const int vec = aligned16(a.ulo) && aligned16(a.uhi) && aligned16(a.slo) && aligned16(a.shi);
  prof::mark(s, "bucket.sample");
  bk_sample_kernel<D><<<kSampleBlocks, kSampleThreads, 0, s>>>(a.ulo, a.uhi, a.slo, a.shi, a.n,
                                                               a.m, p.part);
  bk_plan_kernel<<<1, kSampleThreads, 0, s>>>(p.part, L.nb, p.P);
  prof::mark(s, "bucket.count");
  hipMemsetAsync(p.T + cells, 0, (size_t)(L.nb + 1) * sizeof(uint32_t), s);
  bk_count_kernel<D><<<L.nblk, kThreads, lds, s>>>(a.ulo, a.uhi, a.slo, a.shi, a.n, a.m, vec, p.P,
                                                   L.nb, L.gpb, p.C, p.T + cells, a.hdr);
  prof::mark(s, "bucket.offsets");
  transpose_kernel<<<dim3((L.nb + 63) / 64, (L.nblk + 63) / 64), 256, 0, s>>>(p.C, p.T, L.nblk,
                                                                              L.nb);
  exclusive_scan_u32(p.T, p.S, cells + L.nb + 1, p.scan_tmp, s);
  transpose_kernel<<<dim3((L.nblk + 63) / 64, (L.nb + 63) / 64), 256, 0, s>>>(p.S, p.SB, L.nb,
                                                                              L.nblk);
  prof::mark(s, "bucket.scatter");
  hipMemsetAsync(p.bs_cur, 0, (size_t)L.nb * sizeof(uint32_t), s);
  bk_scatter_kernel<D><<<L.nblk, kThreads, lds, s>>>(a.ulo, a.uhi, a.slo, a.shi, a.n, a.m, vec, p.P,
                                                     L.gpb, p.O, p.SB, p.bs_cur, L.bs_cap, p.rec,
                                                     p.bs_rec);
}

template <int DM1, int MODE>
void sweep_impl(const BucketArgs &a, int32_t *per_update, const unsigned long long *pair_off,
                uint32_t *cursor, uint32_t *out_u, uint32_t *out_s, unsigned long long *total,
                hipStream_t s) {
  Ptrs p = pointers(a);
  bk_sweep_kernel<DM1, MODE, kCap, kSweepThreads><<<a.L.nb, kSweepThreads, 0, s>>>(
      p.rec, p.O, p.bs_rec, a.L.bs_cap, a.n, a.hdr, per_update, pair_off, cursor, out_u, out_s,
      total);
}

}  // namespace

bool bucket_path_supported(int d, int64_t n, int64_t m) {
  if (d < 1 || d > 3) return false;
  const int64_t N = n + m;
  if (N < 1) return false;
  const int64_t nb = (N + kTargetBucket - 1) / kTargetBucket;
  return nb <= (int64_t)kMaxBuckets;
}

BucketLayout bucket_layout(int64_t n, int64_t m, int d) {
  BucketLayout L{};
  const uint64_t N = (uint64_t)(n + m);
  L.nb = (uint32_t)((N + kTargetBucket - 1) / kTargetBucket);
  if (L.nb < 1) L.nb = 1;
  const uint64_t groups = (uint64_t)((n + 3) / 4) + (uint64_t)((m + 3) / 4);
  uint64_t nblk = (groups + kThreads - 1) / kThreads;  // at least one group per thread
  if (nblk > kMaxBlocks) nblk = kMaxBlocks;
  if (nblk < 1) nblk = 1;
  L.nblk = (uint32_t)nblk;
  L.gpb = (uint32_t)((groups + nblk - 1) / nblk);
  L.bs_cap = (uint32_t)(N / 2 + 4096);
  L.rec_words = d == 1 ? 4 : 8;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t o = at;
    at += align256(bytes);
    return o;
  };
  const size_t cells = (size_t)L.nb * L.nblk;
  const size_t scanned = cells + L.nb + 1;  // counts + boundary-state sizes + sentinel
  L.params = take(sizeof(BucketParams));
  L.sample_part = take(kSampleBlocks * sizeof(float4));
  L.counts = take(cells * sizeof(uint32_t));
  L.transposed = take(scanned * sizeof(uint32_t));
  L.offsets = take(scanned * sizeof(uint32_t));
  L.block_offsets = take(cells * sizeof(uint32_t));
  L.scan_tmp = take(scan_temp_bytes(scanned));
  L.bs_cur = take((size_t)L.nb * sizeof(uint32_t));
  L.rec = take((size_t)N * L.rec_words * sizeof(uint32_t));
  L.bs_rec = take((size_t)L.bs_cap * L.rec_words * sizeof(uint32_t));
  L.bytes = at;
  return L;
}

hipError_t bucket_prepare(const BucketArgs &a, hipStream_t s) {
  switch (a.d) {
    case 1: prepare_impl<1>(a, s); break;
    case 2: prepare_impl<2>(a, s); break;
    default: prepare_impl<3>(a, s); break;
  }
  return hipGetLastError();
}

hipError_t bucket_sweep(const BucketArgs &a, int mode, int32_t *per_update,
                        const unsigned long long *pair_off, uint32_t *cursor, uint32_t *out_u,
                        uint32_t *out_s, unsigned long long *total, hipStream_t s) {
  prof::mark(s, mode == 2 ? "bucket.sweep.emit" : "bucket.sweep");
#define DDM_SWEEP(DM1)                                                                     \
  if (mode == 0)                                                                           \
    sweep_impl<DM1, 0>(a, per_update, pair_off, cursor, out_u, out_s, total, s);           \
  else if (mode == 1)                                                                      \
    sweep_impl<DM1, 1>(a, per_update, pair_off, cursor, out_u, out_s, total, s);           \
  else                                                                                     \
    sweep_impl<DM1, 2>(a, per_update, pair_off, cursor, out_u, out_s, total, s);
  switch (a.d) {
    case 1: DDM_SWEEP(0) break;
    case 2: DDM_SWEEP(1) break;
    default: DDM_SWEEP(2) break;
  }
#undef DDM_SWEEP
  return hipGetLastError();
}

}  // namespace ddm

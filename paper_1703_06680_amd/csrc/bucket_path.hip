// Bucketed sort-based matching (see bucket_path.h).
//
//   sample   min / max of the swept-axis lower coordinate over a pseudo-random
//            sample of regions;
//   plan     bucket(x) = clamp(floor((x - vmin) * scale), 0, nb - 1), a monotone
//            non-decreasing map, so every region of bucket b starts strictly
//            before every region of bucket b' > b;
//   count    validates every box, and per block of regions histograms the
//            buckets of the non-empty ones; a region whose upper coordinate
//            maps to a later bucket than its lower one may still be active in
//            the buckets in between (it belongs to their boundary state), and
//            adds +1 / -1 to a difference array at the ends of that range;
//   scan     exclusive prefix sum of the bucket-major (bucket, block) counts
//            gives every block its output slots in every bucket;
//   finalize bucket start offsets; prefix sums of the difference array give
//            the size of every bucket's boundary state (the counts of
//            Algorithm 6's SubSet[p] and UpdSet[p] up to the cut being a
//            bucket boundary), and their prefix sum its offset;
//   scatter  writes one fixed-size record per non-empty region into its
//            bucket, and a copy into the boundary state of every later bucket
//            its interval may reach;
//   sweep    one workgroup per bucket: records to registers, a stable LDS
//            radix sort by lower key, per-kind lists in LDS, then every region
//            walks forward over the later lower endpoints of the other kind
//            while they start before it ends; boundary-state regions walk
//            from the start of the bucket.  Each 1-D pair is met exactly once,
//            at the later of the two lower endpoints (the pair Algorithm 4
//            reports at the earlier upper endpoint), and kept if the boxes
//            overlap on every other axis.
#include "bucket_path.h"
#include "primitives.h"
#include "profile.h"

namespace ddm {
namespace {

constexpr int kThreads = 256;                  // sample / count / scatter
constexpr uint32_t kRegionsPerBlock = 16384;   // count / scatter tile
constexpr int kSampleBlocks = 64;
constexpr int kSamplesPerThread = 4;
constexpr uint32_t kTargetBucket = 1536;       // mean records per bucket

// The sweep workgroup: kCap records at most per bucket.
constexpr int kSweepThreads = 512;
constexpr int kCap = 2048;

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

// err bits, emptiness
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

// ---------------------------------------------------------------- sample

template <int D>
__global__ __launch_bounds__(kThreads) void bk_sample_kernel(
    const float *__restrict__ ulo, const float *__restrict__ uhi, const float *__restrict__ slo,
    const float *__restrict__ shi, uint32_t n, uint32_t m, float4 *__restrict__ part) {
  __shared__ float smin[kThreads / kWave], smax[kThreads / kWave];
  __shared__ uint32_t scnt[kThreads / kWave];
  const uint32_t N = n + m;
  float mn = __int_as_float(0x7f800000), mx = -__int_as_float(0x7f800000);
  uint32_t c = 0;
  for (int j = 0; j < kSamplesPerThread; ++j) {
    const uint32_t i = (blockIdx.x * kThreads + threadIdx.x) * kSamplesPerThread + j;
    const uint32_t r = (uint32_t)(((unsigned long long)mix32(i * 0x9E3779B9u + 0x632BE5ABu) * N) >> 32);
    const Box<D> b = load_box<D>(ulo, uhi, slo, shi, n, r);
    bool empty;
    const uint32_t err = box_errors<D>(b, empty);
    const float x = b.lo[0];
    if (!err && !empty && fabsf(x) <= 3.0e38f) {
      mn = fminf(mn, x);
      mx = fmaxf(mx, x);
      ++c;
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
  if (threadIdx.x == 0) {
    for (int i = 1; i < kThreads / kWave; ++i) {
      mn = fminf(mn, smin[i]);
      mx = fmaxf(mx, smax[i]);
      c += scnt[i];
    }
    part[blockIdx.x] = make_float4(mn, mx, __uint_as_float(c), 0.f);
  }
}

__global__ void bk_plan_kernel(const float4 *__restrict__ part, int nparts, uint32_t nb,
                               BucketParams *__restrict__ P) {
  if (threadIdx.x != 0) return;
  float mn = __int_as_float(0x7f800000), mx = -__int_as_float(0x7f800000);
  uint32_t c = 0;
  for (int i = 0; i < nparts; ++i) {
    const float4 p = part[i];
    const uint32_t pc = __float_as_uint(p.z);
    if (pc) {
      mn = fminf(mn, p.x);
      mx = fmaxf(mx, p.y);
      c += pc;
    }
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

// ------------------------------------------------------------ count pass

template <int D>
__global__ __launch_bounds__(kThreads) void bk_count_kernel(
    const float *__restrict__ ulo, const float *__restrict__ uhi, const float *__restrict__ slo,
    const float *__restrict__ shi, uint32_t n, uint32_t m, const BucketParams *__restrict__ P,
    uint32_t nb, uint32_t *__restrict__ counts, uint32_t nblk, int *__restrict__ bs_diff,
    Header *__restrict__ hdr) {
  extern __shared__ uint32_t hist[];
  const BucketParams p = *P;
  for (uint32_t b = threadIdx.x; b < nb; b += kThreads) hist[b] = 0;
  __syncthreads();
  const uint32_t N = n + m;
  const uint32_t base = blockIdx.x * kRegionsPerBlock;
  const uint32_t end = min(base + kRegionsPerBlock, N);
  uint32_t err = 0;
  for (uint32_t r = base + threadIdx.x; r < end; r += kThreads) {
    const Box<D> bx = load_box<D>(ulo, uhi, slo, shi, n, r);
    bool empty;
    err |= box_errors<D>(bx, empty);
    if (empty) continue;
    const uint32_t b = bucket_of(bx.lo[0], p.vmin, p.scale, nb);
    atomicAdd(&hist[b], 1u);
    const uint32_t last = bucket_of(bx.hi[0], p.vmin, p.scale, nb);
    if (last > b) {
      atomicAdd(&bs_diff[b + 1], 1);
      if (last + 1 < nb) atomicAdd(&bs_diff[last + 1], -1);
    }
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < nb; b += kThreads) counts[(size_t)b * nblk + blockIdx.x] = hist[b];
  err = (__ballot(err & kErrNaN) ? kErrNaN : 0u) | (__ballot(err & kErrOrder) ? kErrOrder : 0u);
  if (err && lane_id() == 0) atomicOr(&hdr->err, err);
}

// One block: bucket starts, non-empty total, boundary-state sizes/offsets.
__global__ __launch_bounds__(kThreads) void bk_finalize_kernel(
    const uint32_t *__restrict__ counts, const uint32_t *__restrict__ offsets, uint32_t nb,
    uint32_t nblk, const int *__restrict__ bs_diff, uint32_t bs_cap, uint32_t *__restrict__ bstart,
    uint32_t *__restrict__ bs_off, uint32_t *__restrict__ bs_cur, Header *__restrict__ hdr) {
  __shared__ uint32_t lds[kThreads / kWave + 1];
  const size_t last = (size_t)nb * nblk - 1;
  const uint32_t total = offsets[last] + counts[last];
  for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
    bstart[b] = offsets[(size_t)b * nblk];
    bs_cur[b] = 0;
  }
  if (threadIdx.x == 0) {
    bstart[nb] = total;
    hdr->nonempty = total;
  }
  // size_j = diff[0] + ... + diff[j]; off_j = size_0 + ... + size_{j-1}
  uint32_t carry_size = 0, carry_off = 0;
  for (uint32_t base = 0; base < nb; base += kThreads) {
    const uint32_t j = base + threadIdx.x;
    const uint32_t dv = j < nb ? (uint32_t)bs_diff[j] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<uint32_t, kThreads>(dv, lds, &tot);
    const uint32_t size = carry_size + ex + dv;
    carry_size += tot;
    const uint32_t sz = j < nb ? size : 0u;
    uint32_t tot2;
    const uint32_t ex2 = block_exclusive_scan<uint32_t, kThreads>(sz, lds, &tot2);
    if (j < nb) bs_off[j] = carry_off + ex2;
    carry_off += tot2;
  }
  if (threadIdx.x == 0) {
    bs_off[nb] = carry_off;
    hdr->bs_total = carry_off;
    if (carry_off > bs_cap) hdr->overflow = 1u;
  }
}

// ---------------------------------------------------------- scatter pass

// Record: word 0 = encoded lower key (swept axis), 1 = encoded upper key,
// 2 = region index (updates first), 3 = 0, then lo/hi of each other axis.
template <int D>
__device__ __forceinline__ void write_record(uint32_t *__restrict__ dst, const Box<D> &b,
                                             uint32_t r) {
  constexpr int RW = D == 1 ? 4 : 8;
  uint32_t w[RW];
  w[0] = encode_coord(b.lo[0]);
  w[1] = encode_coord(b.hi[0]);
  w[2] = r;
  w[3] = 0;
#pragma unroll
  for (int k = 1; k < D; ++k) {
    w[4 + 2 * (k - 1)] = __float_as_uint(b.lo[k]);
    w[5 + 2 * (k - 1)] = __float_as_uint(b.hi[k]);
  }
#pragma unroll
  for (int k = 4 + 2 * (D - 1); k < RW; ++k) w[k] = 0;
  uint4 *d4 = reinterpret_cast<uint4 *>(dst);
  d4[0] = make_uint4(w[0], w[1], w[2], w[3]);
  if (RW == 8) d4[1] = make_uint4(w[4 % RW], w[5 % RW], w[6 % RW], w[7 % RW]);
}

template <int D>
__global__ __launch_bounds__(kThreads) void bk_scatter_kernel(
    const float *__restrict__ ulo, const float *__restrict__ uhi, const float *__restrict__ slo,
    const float *__restrict__ shi, uint32_t n, uint32_t m, const BucketParams *__restrict__ P,
    uint32_t nb, const uint32_t *__restrict__ offsets, uint32_t nblk,
    const uint32_t *__restrict__ bs_off, uint32_t *__restrict__ bs_cur, uint32_t bs_cap,
    uint32_t *__restrict__ rec, uint32_t *__restrict__ bs_rec) {
  constexpr int RW = D == 1 ? 4 : 8;
  extern __shared__ uint32_t cur[];
  const BucketParams p = *P;
  for (uint32_t b = threadIdx.x; b < nb; b += kThreads) cur[b] = offsets[(size_t)b * nblk + blockIdx.x];
  __syncthreads();
  const uint32_t N = n + m;
  const uint32_t base = blockIdx.x * kRegionsPerBlock;
  const uint32_t end = min(base + kRegionsPerBlock, N);
  for (uint32_t r = base + threadIdx.x; r < end; r += kThreads) {
    const Box<D> bx = load_box<D>(ulo, uhi, slo, shi, n, r);
    bool empty;
    (void)box_errors<D>(bx, empty);
    if (empty) continue;
    const uint32_t b = bucket_of(bx.lo[0], p.vmin, p.scale, nb);
    const uint32_t slot = atomicAdd(&cur[b], 1u);
    write_record<D>(rec + (size_t)slot * RW, bx, r);
    const uint32_t last = bucket_of(bx.hi[0], p.vmin, p.scale, nb);
    for (uint32_t j = b + 1; j <= last; ++j) {
      const uint32_t pos = bs_off[j] + atomicAdd(&bs_cur[j], 1u);
      if (pos < bs_cap) write_record<D>(bs_rec + (size_t)pos * RW, bx, r);
    }
  }
}

// ------------------------------------------------------------ sweep pass

// One stable LSD pass over C <= CAP (key, value) pairs in LDS, 8-bit digit
// at ``shift``.  Element order: wave w owns positions [w*64*ITEMS,
// (w+1)*64*ITEMS); item i of lane l is position w*64*ITEMS + i*64 + l.
template <int THREADS, int CAP>
__device__ __forceinline__ void lds_radix_pass(const uint32_t *Kin, const uint32_t *Vin,
                                               uint32_t *Kout, uint32_t *Vout, uint32_t C,
                                               int shift, uint32_t *wcnt, uint32_t *dtot) {
  constexpr int W = THREADS / kWave;
  constexpr int ITEMS = CAP / THREADS;
  const int t = threadIdx.x, w = t / kWave, lane = lane_id();
  for (int i = t; i < W * 256; i += THREADS) wcnt[i] = 0;
  __syncthreads();
  uint32_t key[ITEMS], val[ITEMS], dig[ITEMS], rank[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t pos = (uint32_t)(w * (kWave * ITEMS) + i * kWave + lane);
    const bool valid = pos < C;
    key[i] = valid ? Kin[pos] : 0u;
    val[i] = valid ? Vin[pos] : 0u;
    const uint32_t d = (key[i] >> shift) & 255u;
    dig[i] = d;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t on = __ballot(bit);
      peers &= bit ? on : ~on;
    }
    const uint32_t below = __popcll(peers & lanemask_lt());
    const int leader = valid ? (__ffsll((unsigned long long)peers) - 1) : lane;
    uint32_t old = 0;
    if (valid && lane == leader) old = atomicAdd(&wcnt[w * 256 + d], (uint32_t)__popcll(peers));
    old = __shfl(old, leader, kWave);
    rank[i] = valid ? old + below : 0xFFFFFFFFu;
  }
  __syncthreads();
  if (t < 256) {
    uint32_t run = 0;
#pragma unroll
    for (int ww = 0; ww < W; ++ww) {
      const uint32_t c = wcnt[ww * 256 + t];
      wcnt[ww * 256 + t] = run;
      run += c;
    }
    dtot[t] = run;
  }
  __syncthreads();
  if (t < kWave) {
    // exclusive scan of the 256 digit totals, 4 digits per lane
    uint32_t v0 = dtot[4 * t], v1 = dtot[4 * t + 1], v2 = dtot[4 * t + 2], v3 = dtot[4 * t + 3];
    const uint32_t s = v0 + v1 + v2 + v3;
    const uint32_t ex = wave_inclusive_scan(s) - s;
    dtot[4 * t] = ex;
    dtot[4 * t + 1] = ex + v0;
    dtot[4 * t + 2] = ex + v0 + v1;
    dtot[4 * t + 3] = ex + v0 + v1 + v2;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    if (rank[i] != 0xFFFFFFFFu) {
      const uint32_t np = dtot[dig[i]] + wcnt[w * 256 + dig[i]] + rank[i];
      Kout[np] = key[i];
      Vout[np] = val[i];
    }
  }
  __syncthreads();
}

template <int THREADS>
__device__ __forceinline__ uint32_t block_min_u32(uint32_t v, uint32_t *lds) {
  v = wave_min(v);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) lds[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < THREADS / kWave; ++i) v = lds[i] < v ? lds[i] : v;
    lds[THREADS / kWave] = v;
  }
  __syncthreads();
  v = lds[THREADS / kWave];
  __syncthreads();
  return v;
}

template <int THREADS>
__device__ __forceinline__ uint32_t block_max_u32(uint32_t v, uint32_t *lds) {
  v = wave_max(v);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) lds[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < THREADS / kWave; ++i) v = lds[i] > v ? lds[i] : v;
    lds[THREADS / kWave] = v;
  }
  __syncthreads();
  v = lds[THREADS / kWave];
  __syncthreads();
  return v;
}

template <int DM1, int MODE, int CAP, int THREADS>
__global__ __launch_bounds__(THREADS) void bk_sweep_kernel(
    const uint32_t *__restrict__ rec, const uint32_t *__restrict__ bstart,
    const uint32_t *__restrict__ bs_rec, const uint32_t *__restrict__ bs_off, uint32_t n,
    Header *__restrict__ hdr, int32_t *__restrict__ per_update,
    const unsigned long long *__restrict__ pair_off, uint32_t *__restrict__ cursor,
    uint32_t *__restrict__ out_u, uint32_t *__restrict__ out_s,
    unsigned long long *__restrict__ total) {
  constexpr int RW = DM1 == 0 ? 4 : 8;
  constexpr int NC = 2 * DM1;               // other-axis words per record
  constexpr int CW = DM1 == 0 ? 1 : NC;     // LDS words per element for coords
  constexpr int ITEMS = CAP / THREADS;
  constexpr int W = THREADS / kWave;
  constexpr int SOA = (3 + CW) * CAP;
  constexpr int MAIN = SOA > 4 * CAP ? SOA : 4 * CAP;
  constexpr int AUX = (W * 256) > CAP ? (W * 256) : CAP;
  __shared__ __align__(16) uint32_t sm[MAIN];
  __shared__ uint32_t aux[AUX];
  __shared__ uint32_t dtot[256];
  __shared__ uint32_t red[W + 2];
  __shared__ unsigned long long red64[W];

  if (hdr->overflow) return;  // boundary state did not fit (set before launch)
  const uint32_t b = blockIdx.x;
  const uint32_t start = bstart[b];
  const uint32_t C = bstart[b + 1] - start;
  if (C > (uint32_t)CAP) {
    if (threadIdx.x == 0) atomicOr(&hdr->pad[0], 1u);
    return;
  }
  const uint32_t bs_begin = bs_off[b];
  const uint32_t nbs = bs_off[b + 1] - bs_begin;
  const int t = threadIdx.x;

  // 1. own records into registers (slot s = t + i * THREADS)
  uint32_t rk[ITEMS][RW];
  uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
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
      kmin = rk[i][0] < kmin ? rk[i][0] : kmin;
      kmax = rk[i][0] > kmax ? rk[i][0] : kmax;
    } else {
#pragma unroll
      for (int k = 0; k < RW; ++k) rk[i][k] = 0;
    }
  }
  kmin = block_min_u32<THREADS>(kmin, red);
  kmax = block_max_u32<THREADS>(kmax, red);

  // 2. stable LDS radix sort by (lower key - kmin); value = slot | kind << 31
  uint32_t *K0 = sm, *V0 = sm + CAP, *K1 = sm + 2 * CAP, *V1 = sm + 3 * CAP;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t s = t + i * THREADS;
    if (s < C) {
      K0[s] = rk[i][0] - kmin;
      V0[s] = s | ((rk[i][2] >= n) ? 0x80000000u : 0u);
    }
  }
  __syncthreads();
  const uint32_t range = C ? kmax - kmin : 0u;
  const int bits = range ? 32 - __clz(range) : 0;
  const int passes = (bits + 7) / 8;
  uint32_t *Kc = K0, *Vc = V0, *Kn = K1, *Vn = V1;
  for (int p = 0; p < passes; ++p) {
    lds_radix_pass<THREADS, CAP>(Kc, Vc, Kn, Vn, C, 8 * p, aux, dtot);
    uint32_t *tk = Kc, *tv = Vc;
    Kc = Kn;
    Vc = Vn;
    Kn = tk;
    Vn = tv;
  }

  // 3. per-kind lists: updates at [0, Cu), subscriptions at [Cu, C), both in
  //    sorted order; DEST/STO (in the free buffers) give each slot its list
  //    index and the first index of the other kind after it.
  uint32_t *DEST = Kn, *STO = Vn;
  uint32_t vq[ITEMS];
  uint32_t nupd = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t q = t * ITEMS + i;  // blocked order for the scan
    vq[i] = q < C ? Vc[q] : 0x80000000u;
    nupd += (q < C && !(vq[i] >> 31)) ? 1u : 0u;
  }
  uint32_t Cu;
  uint32_t iu = block_exclusive_scan<uint32_t, THREADS>(nupd, red, &Cu);
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t q = t * ITEMS + i;
    if (q < C) {
      const uint32_t slot = vq[i] & 0x7FFFFFFFu;
      const bool sub = vq[i] >> 31;
      const uint32_t is = q - iu;  // subscriptions before q
      DEST[slot] = sub ? Cu + is : iu;
      STO[slot] = sub ? iu : Cu + is;
      if (!sub) ++iu;
    }
  }
  __syncthreads();
  uint32_t dest[ITEMS], sto[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t s = t + i * THREADS;
    dest[i] = s < C ? DEST[s] : 0u;
    sto[i] = s < C ? STO[s] : 0u;
  }
  __syncthreads();
  uint32_t *KLO = sm, *KHI = sm + CAP, *RID = sm + 2 * CAP, *CO = sm + 3 * CAP;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t s = t + i * THREADS;
    if (s < C) {
      const uint32_t q = dest[i];
      KLO[q] = rk[i][0];
      KHI[q] = rk[i][1];
      RID[q] = rk[i][2];
#pragma unroll
      for (int c = 0; c < NC; ++c) CO[q * CW + c] = rk[i][4 + c];
    }
  }
  uint32_t *RC = aux;  // received matches per update list entry
  for (uint32_t j = t; j < (uint32_t)CAP; j += THREADS) RC[j] = 0;
  __syncthreads();

  // 4. the sweep
  unsigned long long hits = 0;
  auto scan = [&](const uint32_t *y, uint32_t j, uint32_t jend, bool from_bs) {
    const uint32_t khi = y[1];
    const uint32_t ry = y[2];
    const bool y_upd = ry < n;
    float ylo[DM1 > 0 ? DM1 : 1], yhi[DM1 > 0 ? DM1 : 1];
#pragma unroll
    for (int c = 0; c < DM1; ++c) {
      ylo[c] = __uint_as_float(y[4 + 2 * c]);
      yhi[c] = __uint_as_float(y[5 + 2 * c]);
    }
    uint32_t own = 0;
    for (; j < jend; ++j) {
      if (KLO[j] >= khi) break;
      bool hit = true;
      if (DM1 == 1) {
        const float2 xc = *reinterpret_cast<const float2 *>(&CO[j * CW]);
        hit = ylo[0] < xc.y && xc.x < yhi[0];
      } else if (DM1 == 2) {
        const float4 xc = *reinterpret_cast<const float4 *>(&CO[j * CW]);
        hit = ylo[0] < xc.y && xc.x < yhi[0] && ylo[DM1 - 1] < xc.w && xc.z < yhi[DM1 - 1];
      }
      if (!hit) continue;
      ++hits;
      if (MODE == 1) {
        if (y_upd)
          ++own;
        else
          atomicAdd(&RC[j], 1u);
      } else if (MODE == 2) {
        const uint32_t rx = RID[j];
        const uint32_t u = y_upd ? ry : rx;
        const uint32_t sid = (y_upd ? rx : ry) - n;
        const unsigned long long slot = pair_off[u] + atomicAdd(&cursor[u], 1u);
        out_u[slot] = u;
        out_s[slot] = sid;
      }
    }
    return own;
  };

  uint32_t own_upd[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    own_upd[i] = 0;
    const uint32_t s = t + i * THREADS;
    if (s < C) {
      const bool y_upd = rk[i][2] < n;
      own_upd[i] = scan(rk[i], sto[i], y_upd ? C : Cu, false);
    }
  }
  for (uint32_t k = t; k < nbs; k += THREADS) {
    uint32_t y[RW];
    const uint4 *src = reinterpret_cast<const uint4 *>(bs_rec + (size_t)(bs_begin + k) * RW);
    const uint4 a = src[0];
    y[0] = a.x;
    y[1] = a.y;
    y[2] = a.z;
    y[3] = a.w;
    if (RW == 8) {
      const uint4 c = src[1];
      y[4 % RW] = c.x;
      y[5 % RW] = c.y;
      y[6 % RW] = c.z;
      y[7 % RW] = c.w;
    }
    const bool y_upd = y[2] < n;
    const uint32_t own = scan(y, y_upd ? Cu : 0u, y_upd ? C : Cu, true);
    if (MODE == 1 && own) atomicAdd(&per_update[y[2]], (int)own);
  }
  if (MODE == 1) {
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
      if (own_upd[i]) atomicAdd(&RC[dest[i]], own_upd[i]);
    __syncthreads();
    for (uint32_t j = t; j < Cu; j += THREADS) {
      const uint32_t c = RC[j];
      if (c) atomicAdd(&per_update[RID[j]], (int)c);
    }
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

template <int D>
void prepare_impl(const BucketArgs &a, hipStream_t s) {
  const BucketLayout &L = a.L;
  char *ws = static_cast<char *>(a.ws);
  auto P = reinterpret_cast<BucketParams *>(ws + L.params);
  auto part = reinterpret_cast<float4 *>(ws + L.sample_part);
  auto counts = reinterpret_cast<uint32_t *>(ws + L.counts);
  auto offsets = reinterpret_cast<uint32_t *>(ws + L.offsets);
  auto bstart = reinterpret_cast<uint32_t *>(ws + L.bstart);
  auto bs_diff = reinterpret_cast<int *>(ws + L.bs_diff);
  auto bs_off = reinterpret_cast<uint32_t *>(ws + L.bs_off);
  auto bs_cur = reinterpret_cast<uint32_t *>(ws + L.bs_cur);
  auto rec = reinterpret_cast<uint32_t *>(ws + L.rec);
  auto bs_rec = reinterpret_cast<uint32_t *>(ws + L.bs_rec);
  const size_t lds = (size_t)L.nb * sizeof(uint32_t);

  prof::mark(s, "bucket.sample");
  bk_sample_kernel<D><<<kSampleBlocks, kThreads, 0, s>>>(a.ulo, a.uhi, a.slo, a.shi, a.n, a.m, part);
  bk_plan_kernel<<<1, 64, 0, s>>>(part, kSampleBlocks, L.nb, P);
  prof::mark(s, "bucket.count");
  hipMemsetAsync(bs_diff, 0, (size_t)(L.nb + 1) * sizeof(int), s);
  bk_count_kernel<D><<<L.nblk, kThreads, lds, s>>>(a.ulo, a.uhi, a.slo, a.shi, a.n, a.m, P, L.nb,
                                                   counts, L.nblk, bs_diff, a.hdr);
  exclusive_scan_u32(counts, offsets, (size_t)L.nb * L.nblk, ws + L.scan_tmp, s);
  prof::mark(s, "bucket.finalize");
  bk_finalize_kernel<<<1, kThreads, 0, s>>>(counts, offsets, L.nb, L.nblk, bs_diff, L.bs_cap,
                                            bstart, bs_off, bs_cur, a.hdr);
  prof::mark(s, "bucket.scatter");
  bk_scatter_kernel<D><<<L.nblk, kThreads, lds, s>>>(a.ulo, a.uhi, a.slo, a.shi, a.n, a.m, P, L.nb,
                                                     offsets, L.nblk, bs_off, bs_cur, L.bs_cap, rec,
                                                     bs_rec);
}

template <int DM1, int MODE>
void sweep_impl(const BucketArgs &a, int32_t *per_update, const unsigned long long *pair_off,
                uint32_t *cursor, uint32_t *out_u, uint32_t *out_s, unsigned long long *total,
                hipStream_t s) {
  const BucketLayout &L = a.L;
  char *ws = static_cast<char *>(a.ws);
  bk_sweep_kernel<DM1, MODE, kCap, kSweepThreads><<<L.nb, kSweepThreads, 0, s>>>(
      reinterpret_cast<const uint32_t *>(ws + L.rec), reinterpret_cast<const uint32_t *>(ws + L.bstart),
      reinterpret_cast<const uint32_t *>(ws + L.bs_rec), reinterpret_cast<const uint32_t *>(ws + L.bs_off),
      a.n, a.hdr, per_update, pair_off, cursor, out_u, out_s, total);
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
  L.nblk = (uint32_t)((N + kRegionsPerBlock - 1) / kRegionsPerBlock);
  if (L.nblk < 1) L.nblk = 1;
  L.bs_cap = (uint32_t)(N / 2 + 4096);
  L.rec_words = d == 1 ? 4 : 8;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t o = at;
    at += align256(bytes);
    return o;
  };
  const size_t cells = (size_t)L.nb * L.nblk;
  L.params = take(sizeof(BucketParams));
  L.sample_part = take(kSampleBlocks * sizeof(float4));
  L.counts = take(cells * sizeof(uint32_t));
  L.offsets = take(cells * sizeof(uint32_t));
  L.scan_tmp = take(scan_temp_bytes(cells));
  L.bstart = take((size_t)(L.nb + 1) * sizeof(uint32_t));
  L.bs_diff = take((size_t)(L.nb + 1) * sizeof(int));
  L.bs_off = take((size_t)(L.nb + 1) * sizeof(uint32_t));
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

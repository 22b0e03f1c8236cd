// Sort-based matching kernels that work directly on device-wide arrays.
//
// Pipeline (Algorithm 4 of the paper, reorganised for a GPU):
//   1. keys_kernel   validate every box (NaN, lo > hi), mark empty boxes and
//                    write, per region r, the encoded lower and upper
//                    coordinate on the swept axis (regions 0..n-1 are updates,
//                    n..n+m-1 subscriptions, so region order is the
//                    (kind, id) tie order);
//   2. radix sort of the lower keys with the region index as value (stable,
//      so equal coordinates stay in (kind, id) order);
//   3. gather_kernel copies, for every sorted lower endpoint, the upper key
//                    and the coordinates on the other axes into sorted order;
//   4. sweep_kernel  one thread per sorted lower endpoint y walks forward over
//                    the lower endpoints x that follow it while x.lo < y.hi.
//
// Why step 4 reports exactly Algorithm 4's pairs: in the sorted endpoint list
// an interval is active at a point when its lower endpoint has been passed
// and its upper endpoint has not.  Algorithm 4 reports a pair at the first of
// the two upper endpoints, where the other interval is active; equivalently
// the pair is found at the later of the two lower endpoints, where the earlier
// interval is still active.  With upper endpoints ordered before lower ones
// at equal coordinates, "y is still active at x's lower endpoint" is
// enc(x.lo) < enc(y.hi), so no upper endpoint needs to be materialised.  The
// pair is then kept iff the boxes also overlap on every other axis (the AND
// over axes of Sec. 3).
//
// Closed intervals [lo, hi] (Algorithm 1's own tests) differ in two places
// only: no box is empty, and the stored upper key is enc(hi) + 1, because on
// integer keys x <= enc(hi) is x < enc(hi) + 1; the other axes use <=.
#include "common.h"
#include "match_global.h"
#include "profile.h"

namespace ddm {

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void keys_kernel(
    const float *__restrict__ ulo, const float *__restrict__ uhi, uint32_t n,
    const float *__restrict__ slo, const float *__restrict__ shi, uint32_t m, int d, int axis,
    uint32_t closed, uint32_t *__restrict__ klo, uint32_t *__restrict__ khi,
    uint4 *__restrict__ partial) {
  __shared__ uint32_t red[4][kThreads / kWave];
  const uint32_t N = n + m;
  uint32_t err = 0, nonempty = 0, kmin = 0xFFFFFFFFu, kmax = 0u;
  for (uint32_t r = blockIdx.x * kThreads + threadIdx.x; r < N; r += gridDim.x * kThreads) {
    const bool is_upd = r < n;
    const size_t row = (size_t)(is_upd ? r : r - n) * d;
    const float *lo = (is_upd ? ulo : slo) + row;
    const float *hi = (is_upd ? uhi : shi) + row;
    bool empty = false;
    float alo = 0.f, ahi = 0.f;
    for (int k = 0; k < d; ++k) {
      const float l = lo[k], h = hi[k];
      if (l != l || h != h) err |= kErrNaN;
      if (l > h) err |= kErrOrder;
      if (l == h && !closed) empty = true;
      if (k == axis) {
        alo = l;
        ahi = h;
      }
    }
    const uint32_t el = encode_coord(alo);
    klo[r] = empty ? kSentinel : el;
    khi[r] = encode_coord(ahi) + closed;
    if (!empty) {
      ++nonempty;
      kmin = el < kmin ? el : kmin;
      kmax = el > kmax ? el : kmax;
    }
  }
  // block reduction, one atomic per block and field
  err = (__ballot(err & kErrNaN) ? kErrNaN : 0u) | (__ballot(err & kErrOrder) ? kErrOrder : 0u);
  nonempty = wave_sum(nonempty);
  kmin = wave_min(kmin);
  kmax = wave_max(kmax);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    red[0][w] = err;
    red[1][w] = nonempty;
    red[2][w] = kmin;
    red[3][w] = kmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kThreads / kWave; ++i) {
      err |= red[0][i];
      nonempty += red[1][i];
      kmin = red[2][i] < kmin ? red[2][i] : kmin;
      kmax = red[3][i] > kmax ? red[3][i] : kmax;
    }
    partial[blockIdx.x] = make_uint4(err, nonempty, kmin, kmax);
  }
}

// One block folds the per-block partials of keys_kernel into the header.
__global__ __launch_bounds__(kThreads) void keys_finalize_kernel(const uint4 *__restrict__ partial,
                                                                 unsigned nparts,
                                                                 Header *__restrict__ hdr) {
  __shared__ uint32_t red[4][kThreads / kWave];
  uint32_t err = 0, nonempty = 0, kmin = 0xFFFFFFFFu, kmax = 0u;
  for (unsigned i = threadIdx.x; i < nparts; i += kThreads) {
    const uint4 p = partial[i];
    err |= p.x;
    nonempty += p.y;
    if (p.y) {
      kmin = p.z < kmin ? p.z : kmin;
      kmax = p.w > kmax ? p.w : kmax;
    }
  }
  err = (__ballot(err & kErrNaN) ? kErrNaN : 0u) | (__ballot(err & kErrOrder) ? kErrOrder : 0u);
  nonempty = wave_sum(nonempty);
  kmin = wave_min(kmin);
  kmax = wave_max(kmax);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    red[0][w] = err;
    red[1][w] = nonempty;
    red[2][w] = kmin;
    red[3][w] = kmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kThreads / kWave; ++i) {
      err |= red[0][i];
      nonempty += red[1][i];
      kmin = red[2][i] < kmin ? red[2][i] : kmin;
      kmax = red[3][i] > kmax ? red[3][i] : kmax;
    }
    hdr->err = err;
    hdr->nonempty = nonempty;
    hdr->kmin = kmin;
    hdr->kmax = kmax;
  }
}

__global__ __launch_bounds__(kThreads) void gather_kernel(
    const uint32_t *__restrict__ sidx, uint32_t count, const uint32_t *__restrict__ khi,
    const float *__restrict__ ulo, const float *__restrict__ uhi, uint32_t n,
    const float *__restrict__ slo, const float *__restrict__ shi, int d, int axis,
    uint32_t *__restrict__ s_khi, float *__restrict__ s_other, size_t stride) {
  for (uint32_t q = blockIdx.x * kThreads + threadIdx.x; q < count; q += gridDim.x * kThreads) {
    const uint32_t r = sidx[q];
    s_khi[q] = khi[r];
    const bool is_upd = r < n;
    const size_t row = (size_t)(is_upd ? r : r - n) * d;
    const float *lo = (is_upd ? ulo : slo) + row;
    const float *hi = (is_upd ? uhi : shi) + row;
    int j = 0;
    for (int k = 0; k < d; ++k) {
      if (k == axis) continue;
      s_other[(size_t)(2 * j) * stride + q] = lo[k];
      s_other[(size_t)(2 * j + 1) * stride + q] = hi[k];
      ++j;
    }
  }
}

// kMode: 0 = count only, 1 = count + per-update counts, 2 = write pairs.
// kDm1 = number of other axes when known at compile time (0, 1, 2), else -1.
template <int kMode, int kDm1>
__global__ __launch_bounds__(kThreads) void sweep_kernel(
    const uint32_t *__restrict__ skey, const uint32_t *__restrict__ sidx,
    const uint32_t *__restrict__ s_khi, const float *__restrict__ s_other, size_t stride,
    uint32_t count, uint32_t n, int dm1_rt, uint32_t closed, int32_t *__restrict__ per_update,
    const unsigned long long *__restrict__ offsets, uint32_t *__restrict__ cursor,
    uint32_t *__restrict__ out_u, uint32_t *__restrict__ out_s,
    unsigned long long *__restrict__ total) {
  constexpr int kMaxOther = 15;
  const int dm1 = kDm1 >= 0 ? kDm1 : dm1_rt;
  unsigned long long found = 0;
  for (uint32_t q = blockIdx.x * kThreads + threadIdx.x; q < count; q += gridDim.x * kThreads) {
    const uint32_t hi_y = s_khi[q];
    const uint32_t ry = sidx[q];
    const bool y_upd = ry < n;
    float ylo[kMaxOther], yhi[kMaxOther];
#pragma unroll
    for (int j = 0; j < (kDm1 >= 0 ? kDm1 : kMaxOther); ++j) {
      if (j < dm1) {
        ylo[j] = s_other[(size_t)(2 * j) * stride + q];
        yhi[j] = s_other[(size_t)(2 * j + 1) * stride + q];
      }
    }
    uint32_t own = 0;
    for (uint32_t q2 = q + 1; q2 < count && skey[q2] < hi_y; ++q2) {
      const uint32_t rx = sidx[q2];
      if ((rx < n) == y_upd) continue;
      bool hit = true;
#pragma unroll
      for (int j = 0; j < (kDm1 >= 0 ? kDm1 : kMaxOther); ++j) {
        if (j < dm1 && hit) {
          const float xlo = s_other[(size_t)(2 * j) * stride + q2];
          const float xhi = s_other[(size_t)(2 * j + 1) * stride + q2];
          hit = (ylo[j] < xhi || (closed && ylo[j] == xhi)) &&
                (xlo < yhi[j] || (closed && xlo == yhi[j]));
        }
      }
      if (!hit) continue;
      ++found;
      const uint32_t u = y_upd ? ry : rx;
      const uint32_t s = (y_upd ? rx : ry) - n;
      if (kMode == 1) {
        if (y_upd)
          ++own;
        else
          atomicAdd(&per_update[u], 1);
      } else if (kMode == 2) {
        const unsigned long long slot = offsets[u] + atomicAdd(&cursor[u], 1u);
        if (out_u) out_u[slot] = u;  // null: rows are implied by the offsets
        out_s[slot] = s;
      }
    }
    if (kMode == 1 && own) atomicAdd(&per_update[ry], (int)own);
  }
  found = wave_sum(found);
  if (lane_id() == 0 && found) atomicAdd(total, found);
}

__global__ void interleave_kernel(const uint32_t *__restrict__ u, const uint32_t *__restrict__ s,
                                  int32_t *__restrict__ out, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x) {
    int2 v;
    v.x = (int32_t)u[i];
    v.y = (int32_t)s[i];
    reinterpret_cast<int2 *>(out)[i] = v;
  }
}

// Orders every row of an emitted pair list: row u holds the cnt[u]
// subscription ids of update u at in[off[u] ..), in the order the sweep found
// them.  One wave per row: the row is staged in the wave's LDS slice and
// every id goes to off[u] + (number of ids of the row below it); ids in a
// row are distinct (every pair is found once), so the ranks are a
// permutation.  Rows of at most kRowMax ids.
constexpr int kRowWaves = kThreads / kWave;

template <bool kPairs>
__global__ __launch_bounds__(kThreads) void row_sort_kernel(
    const unsigned long long *__restrict__ off, const int32_t *__restrict__ cnt,
    const uint32_t *__restrict__ in, uint32_t n, uint32_t *__restrict__ ids,
    int2 *__restrict__ pairs, const uint32_t *__restrict__ done) {
  __shared__ __align__(16) uint32_t stage[kRowWaves][kRowMax];
  const int w = threadIdx.x / kWave, lane = lane_id();
  uint32_t *row = stage[w];
  // each wave takes 64 consecutive rows at a time, finds with one ballot the
  // ones with work and orders those one after the other
  const uint32_t step = gridDim.x * kRowWaves * kWave;
  for (uint32_t u0 = (blockIdx.x * kRowWaves + w) * kWave; u0 < n; u0 += step) {
    const uint32_t mine = u0 + (uint32_t)lane;
    bool work = false;
    if (mine < n) {
      const uint32_t c = (uint32_t)cnt[mine];
      // longer rows are never passed here; done rows are already in order
      work = c != 0 && c <= kRowMax && !(done && done[mine] == c);
    }
    uint64_t todo = __ballot(work);
    while (todo) {
      const uint32_t u = u0 + (uint32_t)(__ffsll((unsigned long long)todo) - 1);
      todo &= todo - 1;
      const uint32_t L = (uint32_t)cnt[u];
      const unsigned long long base = off[u];
      if (L == 1) {
        if (lane == 0) {
          if (kPairs)
            pairs[base] = make_int2((int32_t)u, (int32_t)in[base]);
          else
            ids[base] = in[base];
        }
        continue;
      }
      const uint32_t L4 = (L + 3) & ~3u;  // padded with ids above every real one
      for (uint32_t i = lane; i < L4; i += kWave) row[i] = i < L ? in[base + i] : 0xFFFFFFFFu;
      __builtin_amdgcn_wave_barrier();
      // up to 128 ids: sorted across the wave in registers; longer rows: ranks
      int2 *prow = kPairs ? pairs : nullptr;
      if (L <= kWave)
        sort_row<1>(row, L, lane, u, base, ids, prow);
      else if (L <= 2 * kWave)
        sort_row<2>(row, L, lane, u, base, ids, prow);
      else
        for (uint32_t i0 = 0; i0 < L; i0 += 4 * kWave)
          rank_row<4>(row, L, L4, i0, lane, u, base, ids, prow);
      __builtin_amdgcn_wave_barrier();  // every lane done with the row before the next one
    }
  }
}

inline unsigned grid_for(size_t count, unsigned cap = 8192) {
  size_t g = (count + kThreads - 1) / kThreads;
  if (g < 1) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

template <int kMode>
void launch_sweep(const SweepArgs &a, hipStream_t s) {
  const unsigned grid = grid_for(a.count, 1u << 20);
  switch (a.dm1) {
    case 0:
      sweep_kernel<kMode, 0><<<grid, kThreads, 0, s>>>(a.skey, a.sidx, a.s_khi, a.s_other, a.stride,
                                                       a.count, a.n, a.dm1, a.closed, a.per_update, a.offsets,
                                                       a.cursor, a.out_u, a.out_s, a.total);
      break;
    case 1:
      sweep_kernel<kMode, 1><<<grid, kThreads, 0, s>>>(a.skey, a.sidx, a.s_khi, a.s_other, a.stride,
                                                       a.count, a.n, a.dm1, a.closed, a.per_update, a.offsets,
                                                       a.cursor, a.out_u, a.out_s, a.total);
      break;
    case 2:
      sweep_kernel<kMode, 2><<<grid, kThreads, 0, s>>>(a.skey, a.sidx, a.s_khi, a.s_other, a.stride,
                                                       a.count, a.n, a.dm1, a.closed, a.per_update, a.offsets,
                                                       a.cursor, a.out_u, a.out_s, a.total);
      break;
    default:
      sweep_kernel<kMode, -1><<<grid, kThreads, 0, s>>>(a.skey, a.sidx, a.s_khi, a.s_other,
                                                        a.stride, a.count, a.n, a.dm1, a.closed, a.per_update,
                                                        a.offsets, a.cursor, a.out_u, a.out_s,
                                                        a.total);
      break;
  }
}

}  // namespace

unsigned keys_grid(size_t regions) { return grid_for(regions, kKeysMaxBlocks); }

void launch_keys(const float *ulo, const float *uhi, uint32_t n, const float *slo,
                 const float *shi, uint32_t m, int d, int axis, uint32_t closed, uint32_t *klo,
                 uint32_t *khi, uint4 *partial, Header *hdr, hipStream_t s) {
  const unsigned grid = keys_grid((size_t)n + m);
  prof::mark(s, "keys");
  keys_kernel<<<grid, kThreads, 0, s>>>(ulo, uhi, n, slo, shi, m, d, axis, closed, klo, khi,
                                        partial);
  prof::mark(s, "keys.finalize");
  keys_finalize_kernel<<<1, kThreads, 0, s>>>(partial, grid, hdr);
}

void launch_gather(const uint32_t *sidx, uint32_t count, const uint32_t *khi, const float *ulo,
                   const float *uhi, uint32_t n, const float *slo, const float *shi, int d,
                   int axis, uint32_t *s_khi, float *s_other, size_t stride, hipStream_t s) {
  if (!count) return;
  prof::mark(s, "gather");
  gather_kernel<<<grid_for(count), kThreads, 0, s>>>(sidx, count, khi, ulo, uhi, n, slo, shi, d,
                                                     axis, s_khi, s_other, stride);
}

void launch_sweep(int mode, const SweepArgs &a, hipStream_t s) {
  if (!a.count) return;
  prof::mark(s, mode == 2 ? "sweep.emit" : "sweep.count");
  if (mode == 0)
    launch_sweep<0>(a, s);
  else if (mode == 1)
    launch_sweep<1>(a, s);
  else
    launch_sweep<2>(a, s);
}

void launch_interleave(const uint32_t *u, const uint32_t *sidx, int32_t *out, size_t count,
                       hipStream_t s) {
  if (!count) return;
  prof::mark(s, "pairs.interleave");
  interleave_kernel<<<grid_for(count), kThreads, 0, s>>>(u, sidx, out, count);
}

void launch_row_sort(const unsigned long long *off, const int32_t *cnt, const uint32_t *in,
                     uint32_t n, uint32_t *ids, int32_t *pairs, hipStream_t s,
                     const uint32_t *done) {
  if (!n) return;
  prof::mark(s, "pairs.rowsort");
  const unsigned grid = grid_for((size_t)n / kRowWaves, 4096);
  if (pairs)
    row_sort_kernel<true><<<grid, kThreads, 0, s>>>(off, cnt, in, n, nullptr,
                                                    reinterpret_cast<int2 *>(pairs), done);
  else
    row_sort_kernel<false><<<grid, kThreads, 0, s>>>(off, cnt, in, n, ids, nullptr, done);
}

}  // namespace ddm

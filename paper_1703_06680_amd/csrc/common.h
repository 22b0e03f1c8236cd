// Device-side helpers shared by the libddm kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddm {

constexpr int kWave = 64;
// Key of an empty region's lower endpoint: above every encoded coordinate
// (only a NaN could encode to it, and NaN is rejected).
constexpr uint32_t kSentinel = 0xFFFFFFFFu;

// Device-detected input errors (bit flags in Header::err).
constexpr uint32_t kErrNaN = 1u;
constexpr uint32_t kErrOrder = 2u;

// Header::pad[1] bits of the bucketed path: why it could not finish.
constexpr uint32_t kSplittable = 1u;    // slab buckets overflowed (their totals can split them)
constexpr uint32_t kUnsplittable = 2u;  // something else overflowed

// Small device-resident header at the start of every workspace.
struct Header {
  uint32_t err;        // OR of kErr* flags
  uint32_t nonempty;   // regions that are non-empty on every axis
  uint32_t kmin;       // min encoded lower key over non-empty regions
  uint32_t kmax;       // max encoded lower key over non-empty regions
  // bucketed path: boundary-state copies claimed so far by boxes reaching
  // more than one later cell (checked against the buffer's capacity)
  unsigned long long bs_copies;
  uint32_t pad[2];     // pad[0]: the bucketed path cannot finish; pad[1]: kSplittable |
                       // kUnsplittable, why
  unsigned long long total;  // number of intersecting pairs
  unsigned long long aux[3];
  uint32_t split_nb;   // buckets after overfull ones were split (0: they cannot be)
  uint32_t spare;
};

// Order-preserving map of a non-NaN float32 onto uint32: a < b (IEEE)
// iff enc(a) < enc(b) (unsigned), and enc(-0) == enc(+0).
__device__ __forceinline__ uint32_t encode_coord(float x) {
  uint32_t b = __float_as_uint(x);
  if ((b << 1) == 0u) b = 0u;  // -0.0 -> +0.0
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (uint64_t(1) << lane_id()) - 1;
}

// Sum over the 64 lanes of a wave (result in every lane).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, kWave);
    v = w < v ? w : v;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, kWave);
    v = w > v ? w : v;
  }
  return v;
}

// Inclusive prefix sum over the lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = lane_id();
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(v, o, kWave);
    if (lane >= o) v += y;
  }
  return v;
}

// Value of lane (lane ^ J) of a wave: DPP quad permutes for J = 1, 2,
// ds_swizzle (bitmask mode, within 32-lane halves) for J = 4, 8, 16, a
// lane permute for 32.
template <uint32_t J>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
  if constexpr (J == 1)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
  else if constexpr (J == 2)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
  else if constexpr (J == 4 || J == 8 || J == 16)
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (J << 10));
  else
    return (uint32_t)__shfl_xor((int)v, (int)J, kWave);
}

// One compare-exchange stage of the bitonic network (partner distance J
// below 64, block size K).
template <int NPER, uint32_t K, uint32_t J>
__device__ __forceinline__ void bitonic_stage(uint32_t (&v)[NPER], uint32_t lane) {
#pragma unroll
  for (int r = 0; r < NPER; ++r) {
    const uint32_t e = lane + 64u * (uint32_t)r;
    const uint32_t p = lane_xor<J>(v[r]);
    // element e keeps the smaller value iff (e & K == 0) == (e & J == 0)
    const bool keep_min = ((e & K) == 0) == ((e & J) == 0);
    v[r] = keep_min ? min(v[r], p) : max(v[r], p);
  }
}

template <int NPER, uint32_t K, uint32_t J>
__device__ __forceinline__ void bitonic_merge(uint32_t (&v)[NPER], uint32_t lane) {
  if constexpr (J >= 64) {  // partner in the other register of the same lane
    const uint32_t lo = min(v[0], v[NPER - 1]), hi = max(v[0], v[NPER - 1]);
    const bool up0 = (lane & K) == 0;
    v[0] = up0 ? lo : hi;
    v[NPER - 1] = up0 ? hi : lo;
  } else {
    bitonic_stage<NPER, K, J>(v, lane);
  }
  if constexpr (J > 1) bitonic_merge<NPER, K, J / 2>(v, lane);
}

template <int NPER, uint32_t K>
__device__ __forceinline__ void bitonic_from(uint32_t (&v)[NPER], uint32_t lane) {
  bitonic_merge<NPER, K, K / 2>(v, lane);
  if constexpr (K < 64u * NPER) bitonic_from<NPER, 2 * K>(v, lane);
}

// Ascending bitonic sort of the 64 * NPER values held by a wave, element e
// in lane e % 64 of register e / 64 (NPER = 1 or 2).  After the call the
// same layout holds the sorted sequence.
template <int NPER>
__device__ __forceinline__ void wave_bitonic_sort(uint32_t (&v)[NPER]) {
  static_assert(NPER == 1 || NPER == 2, "64 or 128 values");
  bitonic_from<NPER, 2>(v, (uint32_t)lane_id());
}

// Ordering one row of a pair list (update u's subscription ids, all
// distinct) that a wave has staged in LDS: the ids go to
// ids[base + position] (CSR), or, with pairs non-null, to
// pairs[base + position] = (u, id).
//
// sort_row: a row of L <= 64 * NPER ids, sorted across the wave in
// registers and written in order (coalesced).
template <int NPER>
__device__ __forceinline__ void sort_row(const uint32_t *stage, uint32_t L, int lane, uint32_t u,
                                         unsigned long long base, uint32_t *ids, int2 *pairs) {
  uint32_t v[NPER];
#pragma unroll
  for (int r = 0; r < NPER; ++r) {
    const uint32_t e = (uint32_t)lane + 64u * (uint32_t)r;
    v[r] = e < L ? stage[e] : 0xFFFFFFFFu;
  }
  wave_bitonic_sort<NPER>(v);
#pragma unroll
  for (int r = 0; r < NPER; ++r) {
    const uint32_t e = (uint32_t)lane + 64u * (uint32_t)r;
    if (e < L) {
      if (pairs)
        pairs[base + e] = make_int2((int32_t)u, (int32_t)v[r]);
      else
        ids[base + e] = v[r];
    }
  }
}

// rank_row: the ids at positions i0 .. i0 + 64 kPer of a row of L ids,
// staged with padding above every id up to L4 (a multiple of four); each
// goes to its rank, the number of the row's ids below it.
template <int kPer>
__device__ __forceinline__ void rank_row(const uint32_t *stage, uint32_t L, uint32_t L4,
                                         uint32_t i0, int lane, uint32_t u, unsigned long long base,
                                         uint32_t *ids, int2 *pairs) {
  uint32_t v[kPer], rank[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint32_t i = i0 + k * kWave + lane;
    v[k] = i < L ? stage[i] : 0xFFFFFFFFu;
    rank[k] = 0;
  }
  for (uint32_t j = 0; j < L4; j += 4) {
    const uint4 q = *reinterpret_cast<const uint4 *>(stage + j);  // same address in every lane
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      rank[k] += (uint32_t)(q.x < v[k]) + (uint32_t)(q.y < v[k]) + (uint32_t)(q.z < v[k]) +
                 (uint32_t)(q.w < v[k]);
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint32_t i = i0 + k * kWave + lane;
    if (i < L) {
      if (pairs)
        pairs[base + rank[k]] = make_int2((int32_t)u, (int32_t)v[k]);
      else
        ids[base + rank[k]] = v[k];
    }
  }
}

// Exclusive prefix sum over a block of THREADS threads.  ``lds`` must hold
// THREADS/64 + 1 elements.  Returns the exclusive prefix of ``v`` and writes
// the block total to ``*total``.  Contains barriers: every thread must call.
template <typename T, int THREADS>
__device__ __forceinline__ T block_exclusive_scan(T v, T *lds, T *total) {
  constexpr int W = THREADS / kWave;
  const int w = threadIdx.x / kWave;
  T x = wave_inclusive_scan(v);
  if (lane_id() == kWave - 1) lds[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = 0;
    for (int i = 0; i < W; ++i) {
      T t = lds[i];
      lds[i] = acc;
      acc += t;
    }
    lds[W] = acc;
  }
  __syncthreads();
  T res = lds[w] + x - v;
  *total = lds[W];
  __syncthreads();
  return res;
}

}  // namespace ddm

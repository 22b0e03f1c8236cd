// Device-wide primitives: exclusive prefix sums (reduce-then-scan) and a
// stable least-significant-digit radix sort of (uint32 key, uint32 value)
// pairs.
//
// The sort is the "sort T in non-decreasing order" step of sort-based
// matching (Algorithm 4; Sec. 4 asks for a parallel sort).  Each pass takes an
// 8-bit digit: an up-sweep kernel histograms every 4096-element tile, a
// device-wide exclusive scan over the digit-major histogram matrix turns the
// counts into output offsets, and a down-sweep kernel ranks every element
// inside its tile (wave-level digit match with ballots, per-wave running
// counters in LDS) and scatters it.  Ranks follow input order within a tile
// and tiles follow input order within a digit, so every pass is stable.
#include <algorithm>

#include "common.h"
#include "primitives.h"
#include "profile.h"

namespace ddm {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kScanThreads * kScanItems;

__host__ __device__ inline size_t div_up(size_t a, size_t b) { return (a + b - 1) / b; }
__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ------------------------------------------------------------------- scans

// Inputs of type TI (count of them; zero past the end) summed as TO; with
// max_out, the largest input is also folded into *max_out (atomic maximum).
template <typename TI, typename TO>
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const TI *__restrict__ in,
                                                                   size_t count,
                                                                   TO *__restrict__ block_sums,
                                                                   TO *__restrict__ max_out) {
  __shared__ TO part[kScanThreads / kWave];
  const size_t base = (size_t)blockIdx.x * kScanChunk;
  TO acc = 0, most = 0;
  for (int i = 0; i < kScanItems; ++i) {
    size_t idx = base + (size_t)i * kScanThreads + threadIdx.x;
    if (idx < count) {
      const TO v = (TO)in[idx];
      acc += v;
      most = v > most ? v : most;
    }
  }
  acc = wave_sum(acc);
  if (lane_id() == 0) part[threadIdx.x / kWave] = acc;
  if (max_out) {
    most = wave_max(most);
    // a read first: most waves see a larger maximum already and skip the atomic
    if (lane_id() == 0 && most > *(volatile TO *)max_out) atomicMax(max_out, most);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    TO t = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) t += part[w];
    block_sums[blockIdx.x] = t;
  }
}

// One block scans the per-block sums (any length) with a running carry.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_block_sums_kernel(T *__restrict__ sums,
                                                                       size_t nblocks) {
  __shared__ T lds[kScanThreads / kWave + 1];
  T carry = 0;
  for (size_t base = 0; base < nblocks; base += kScanThreads) {
    size_t idx = base + threadIdx.x;
    T v = idx < nblocks ? sums[idx] : T(0);
    T total;
    T ex = block_exclusive_scan<T, kScanThreads>(v, lds, &total);
    if (idx < nblocks) sums[idx] = carry + ex;
    carry += total;
  }
}

__device__ __forceinline__ int padded(int i) { return i + (i >> 5); }

// Inputs TI[count_in] (zero past the end), exclusive prefix written as
// TO[count_out].
template <typename TI, typename TO>
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const TI *in, TO *out,
                                                                  size_t count_in, size_t count_out,
                                                                  const TO *__restrict__ block_sums) {
  using T = TO;
  __shared__ T tile[kScanChunk + kScanChunk / 32];
  __shared__ T lds[kScanThreads / kWave + 1];
  const size_t base = (size_t)blockIdx.x * kScanChunk;
  for (int i = 0; i < kScanItems; ++i) {
    int j = i * kScanThreads + threadIdx.x;
    size_t idx = base + j;
    tile[padded(j)] = idx < count_in ? (T)in[idx] : T(0);
  }
  __syncthreads();
  T loc[kScanItems];
  T sum = 0;
  for (int i = 0; i < kScanItems; ++i) {
    loc[i] = tile[padded(threadIdx.x * kScanItems + i)];
    sum += loc[i];
  }
  T total;
  T run = block_exclusive_scan<T, kScanThreads>(sum, lds, &total) + block_sums[blockIdx.x];
  for (int i = 0; i < kScanItems; ++i) {
    tile[padded(threadIdx.x * kScanItems + i)] = run;
    run += loc[i];
  }
  __syncthreads();
  for (int i = 0; i < kScanItems; ++i) {
    int j = i * kScanThreads + threadIdx.x;
    size_t idx = base + j;
    if (idx < count_out) out[idx] = tile[padded(j)];
  }
}

// Arrays of at most kSmallScan elements are scanned by one workgroup in one
// launch.  The array passes through LDS so that every device read and write
// is coalesced (consecutive lanes, consecutive elements): it is loaded
// whole, thread t then scans a run of at most kSmallItems consecutive
// elements in LDS, offset by a workgroup scan of the run sums, and the
// result is stored whole.  Every element is read before any is written, so
// out may alias in.  LDS: small_scan_lds(count_out, sizeof(TO)) bytes.
constexpr int kSmallScanThreads = 1024;
constexpr int kSmallItems = 16;
constexpr size_t kSmallScan = (size_t)kSmallItems * kSmallScanThreads;

// one pad element per 32, so that the runs of consecutive threads (a
// stride of up to 16 elements) fall in different banks
__device__ __forceinline__ uint32_t small_pad(uint32_t i) { return i + (i >> 5); }
inline size_t small_scan_lds(size_t count, size_t elem) { return (count + (count >> 5) + 1) * elem; }

template <typename TI, typename TO>
__global__ __launch_bounds__(kSmallScanThreads) void scan_small_kernel(const TI *in, TO *out,
                                                                       uint32_t count_in,
                                                                       uint32_t count_out,
                                                                       TO *max_out) {
  extern __shared__ __align__(16) unsigned char small_smem[];
  TO *tile = reinterpret_cast<TO *>(small_smem);
  __shared__ TO lds[kSmallScanThreads / kWave + 1];
  TO most = 0;
  for (uint32_t i = threadIdx.x; i < count_out; i += kSmallScanThreads) {
    const TO x = i < count_in ? (TO)in[i] : TO(0);
    tile[small_pad(i)] = x;
    most = x > most ? x : most;
  }
  __syncthreads();
  const uint32_t per = (count_out + kSmallScanThreads - 1) / kSmallScanThreads;
  const uint32_t b0 = min(count_out, threadIdx.x * per);
  TO v[kSmallItems], sum = 0;
#pragma unroll
  for (int q = 0; q < kSmallItems; ++q) {
    const uint32_t i = b0 + (uint32_t)q;
    v[q] = (uint32_t)q < per && i < count_out ? tile[small_pad(i)] : TO(0);
    sum += v[q];
  }
  TO total;
  TO run = block_exclusive_scan<TO, kSmallScanThreads>(sum, lds, &total);
#pragma unroll
  for (int q = 0; q < kSmallItems; ++q) {
    const uint32_t i = b0 + (uint32_t)q;
    if ((uint32_t)q < per && i < count_out) tile[small_pad(i)] = run;
    run += v[q];
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < count_out; i += kSmallScanThreads) out[i] = tile[small_pad(i)];
  if (max_out) {
    most = wave_max(most);
    if (lane_id() == 0 && most > *(volatile TO *)max_out) atomicMax(max_out, most);
  }
}

// Exclusive prefix of count_in inputs (zero past the end) into count_out
// outputs, summed in TO; the largest input into *max_out if given.
template <typename TI, typename TO>
hipError_t exclusive_scan_impl(const TI *in, size_t count_in, TO *out, size_t count_out,
                               void *temp, hipStream_t s, TO *max_out = nullptr) {
  if (count_out == 0) return hipSuccess;
  if (count_out <= kSmallScan) {
    scan_small_kernel<TI, TO>
        <<<dim3(1), dim3(kSmallScanThreads), small_scan_lds(count_out, sizeof(TO)), s>>>(
            in, out, (uint32_t)count_in, (uint32_t)count_out, max_out);
    return hipGetLastError();
  }
  size_t nb = div_up(count_out, kScanChunk);
  TO *sums = static_cast<TO *>(temp);
  scan_reduce_kernel<TI, TO><<<dim3((unsigned)nb), dim3(kScanThreads), 0, s>>>(in, count_in, sums,
                                                                               max_out);
  scan_block_sums_kernel<TO><<<dim3(1), dim3(kScanThreads), 0, s>>>(sums, nb);
  scan_apply_kernel<TI, TO><<<dim3((unsigned)nb), dim3(kScanThreads), 0, s>>>(
      in, out, count_in, count_out, sums);
  return hipGetLastError();
}

// ------------------------------------------------------------- radix sort

__device__ __forceinline__ uint32_t transform_key(uint32_t k, KeyTransform xf) {
  if (!xf.reduce) return k;
  return k == kSentinel ? xf.sentinel_code : k - xf.kmin;
}

__device__ __forceinline__ uint32_t live_count(uint32_t count, const uint32_t *count_dev) {
  if (!count_dev) return count;
  const uint32_t c = *count_dev;
  return c < count ? c : count;
}

__global__ __launch_bounds__(kSortThreads) void radix_upsweep_kernel(
    const uint32_t *__restrict__ keys, uint32_t count, KeyTransform xf, int shift,
    uint32_t *__restrict__ counts, uint32_t ntiles, const uint32_t *__restrict__ count_dev) {
  __shared__ uint32_t hist[kRadix];
  count = live_count(count, count_dev);
  for (int i = threadIdx.x; i < kRadix; i += kSortThreads) hist[i] = 0;
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * kSortTile;
  for (int i = 0; i < kSortItems; ++i) {
    size_t idx = base + (size_t)i * kSortThreads + threadIdx.x;
    if (idx < count) {
      uint32_t d = (transform_key(keys[idx], xf) >> shift) & (kRadix - 1);
      atomicAdd(&hist[d], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += kSortThreads)
    counts[(size_t)d * ntiles + blockIdx.x] = hist[d];
}

template <bool kIota>
__global__ __launch_bounds__(kSortThreads) void radix_downsweep_kernel(
    const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in,
    uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out, uint32_t count,
    KeyTransform xf, int shift, const uint32_t *__restrict__ offsets, uint32_t ntiles,
    const uint32_t *__restrict__ count_dev) {
  constexpr int W = kSortThreads / kWave;
  count = live_count(count, count_dev);
  __shared__ uint32_t wcnt[W][kRadix];
  __shared__ uint32_t wbase[W][kRadix];
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int w = tid / kWave;
  for (int i = tid; i < W * kRadix; i += kSortThreads) (&wcnt[0][0])[i] = 0;
  __syncthreads();

  // wave w owns the contiguous slice [w*1024, (w+1)*1024) of the tile;
  // item i of lane l is element i*64 + l of that slice
  const size_t base = (size_t)blockIdx.x * kSortTile + (size_t)w * (kSortItems * kWave);
  uint32_t key[kSortItems], val[kSortItems], rank[kSortItems], dig[kSortItems];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const size_t idx = base + (size_t)i * kWave + lane;
    const bool valid = idx < count;
    const uint32_t k = valid ? keys_in[idx] : 0u;
    key[i] = k;
    val[i] = kIota ? (uint32_t)idx : (valid ? vals_in[idx] : 0u);
    const uint32_t d = (transform_key(k, xf) >> shift) & (kRadix - 1);
    dig[i] = d;
    // lanes holding the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t on = __ballot(bit);
      peers &= bit ? on : ~on;
    }
    const uint32_t below = __popcll(peers & lanemask_lt());
    const int leader = valid ? (__ffsll((unsigned long long)peers) - 1) : lane;
    uint32_t old = 0;
    if (valid && lane == leader) old = atomicAdd(&wcnt[w][d], (uint32_t)__popcll(peers));
    old = __shfl(old, leader, kWave);
    rank[i] = valid ? old + below : 0xFFFFFFFFu;
  }
  __syncthreads();
  for (int d = tid; d < kRadix; d += kSortThreads) {
    uint32_t acc = offsets[(size_t)d * ntiles + blockIdx.x];
#pragma unroll
    for (int ww = 0; ww < W; ++ww) {
      const uint32_t c = wcnt[ww][d];
      wbase[ww][d] = acc;
      acc += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    if (rank[i] != 0xFFFFFFFFu) {
      const uint32_t dst = wbase[w][dig[i]] + rank[i];
      keys_out[dst] = key[i];
      vals_out[dst] = val[i];
    }
  }
}

__global__ void iota_kernel(uint32_t *out, uint32_t count, const uint32_t *count_dev) {
  count = live_count(count, count_dev);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = (uint32_t)i;
}

template <typename T>
__global__ void fill_kernel(T *out, T value, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = value;
}

template <typename T>
hipError_t fill_impl(T *out, T value, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>(div_up(count, 256), 2048);
  fill_kernel<T><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(out, value, count);
  return hipGetLastError();
}

}  // namespace

hipError_t fill_u32(uint32_t *out, uint32_t value, size_t count, hipStream_t s) {
  return fill_impl<uint32_t>(out, value, count, s);
}

hipError_t fill_u64(unsigned long long *out, unsigned long long value, size_t count,
                    hipStream_t s) {
  return fill_impl<unsigned long long>(out, value, count, s);
}

size_t scan_temp_bytes(size_t count) {
  return align256(div_up(count ? count : 1, kScanChunk) * sizeof(unsigned long long));
}

hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, size_t count, void *temp,
                              hipStream_t s) {
  return exclusive_scan_impl<uint32_t, uint32_t>(in, count, out, count, temp, s);
}

hipError_t exclusive_scan_u64(const unsigned long long *in, unsigned long long *out, size_t count,
                              void *temp, hipStream_t s) {
  return exclusive_scan_impl<unsigned long long, unsigned long long>(in, count, out, count, temp,
                                                                     s);
}

hipError_t exclusive_scan_widen(const uint32_t *in, size_t count, unsigned long long *out,
                                size_t out_count, void *temp, hipStream_t s,
                                unsigned long long *max_out) {
  return exclusive_scan_impl<uint32_t, unsigned long long>(in, count, out, out_count, temp, s,
                                                           max_out);
}

size_t radix_sort_temp_bytes(uint32_t count) {
  size_t ntiles = div_up(count ? count : 1, kSortTile);
  size_t hist = (size_t)kRadix * ntiles;
  return align256(hist * sizeof(uint32_t)) + scan_temp_bytes(hist);
}

hipError_t radix_sort_pairs(uint32_t *keys_a, uint32_t *vals_a, uint32_t *keys_b, uint32_t *vals_b,
                            uint32_t count, int bits, bool vals_iota, KeyTransform xf, void *temp,
                            hipStream_t s, int *in_b, const uint32_t *count_dev) {
  *in_b = 0;
  if (count == 0) return hipSuccess;
  const int passes = (bits + kRadixBits - 1) / kRadixBits;
  if (passes == 0) {
    prof::mark(s, "sort.iota");
    if (vals_iota) iota_kernel<<<dim3(1024), dim3(256), 0, s>>>(vals_a, count, count_dev);
    return hipGetLastError();
  }
  const uint32_t ntiles = (uint32_t)div_up(count, kSortTile);
  const size_t hist = (size_t)kRadix * ntiles;
  uint32_t *counts = static_cast<uint32_t *>(temp);
  void *scan_tmp = static_cast<char *>(temp) + align256(hist * sizeof(uint32_t));
  uint32_t *ck = keys_a, *cv = vals_a, *ok = keys_b, *ov = vals_b;
  bool iota = vals_iota;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * kRadixBits;
    prof::mark(s, "sort.upsweep");
    radix_upsweep_kernel<<<dim3(ntiles), dim3(kSortThreads), 0, s>>>(ck, count, xf, shift, counts,
                                                                     ntiles, count_dev);
    hipError_t e = exclusive_scan_u32(counts, counts, hist, scan_tmp, s);
    if (e != hipSuccess) return e;
    prof::mark(s, "sort.downsweep");
    if (iota)
      radix_downsweep_kernel<true><<<dim3(ntiles), dim3(kSortThreads), 0, s>>>(
          ck, cv, ok, ov, count, xf, shift, counts, ntiles, count_dev);
    else
      radix_downsweep_kernel<false><<<dim3(ntiles), dim3(kSortThreads), 0, s>>>(
          ck, cv, ok, ov, count, xf, shift, counts, ntiles, count_dev);
    iota = false;
    uint32_t *tk = ck, *tv = cv;
    ck = ok;
    cv = ov;
    ok = tk;
    ov = tv;
  }
  *in_b = passes & 1;
  return hipGetLastError();
}

}  // namespace ddm

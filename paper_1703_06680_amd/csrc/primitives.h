// Host-side interface of the device-wide primitives in primitives.hip:
// exclusive prefix sums and a stable LSD radix sort of (uint32 key, uint32
// value) pairs.  All work is enqueued on the given stream; temporaries live in
// caller-provided device memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ddm {

// Exclusive prefix sum out[i] = in[0] + ... + in[i-1] (out may alias in).
size_t scan_temp_bytes(size_t count);
hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, size_t count, void *temp,
                              hipStream_t s);
hipError_t exclusive_scan_u64(const unsigned long long *in, unsigned long long *out,
                              size_t count, void *temp, hipStream_t s);
// The same over count 32-bit inputs (zero past the end) into out_count
// (count or count + 1) 64-bit outputs, without a separate widening pass; with
// max_out (cleared beforehand), the largest input is folded into it.  temp
// holds scan_temp_bytes(out_count) bytes.
hipError_t exclusive_scan_widen(const uint32_t *in, size_t count, unsigned long long *out,
                                size_t out_count, void *temp, hipStream_t s,
                                unsigned long long *max_out = nullptr);

// out[i] = value for i < count, by a kernel (so that it may be recorded into a
// graph, unlike a memset node).
hipError_t fill_u32(uint32_t *out, uint32_t value, size_t count, hipStream_t s);
hipError_t fill_u64(unsigned long long *out, unsigned long long value, size_t count, hipStream_t s);

// Optional range reduction applied to keys before digits are taken:
// key' = (key == 0xFFFFFFFF) ? sentinel_code : key - kmin.
struct KeyTransform {
  uint32_t reduce;  // 0: use raw keys
  uint32_t kmin;
  uint32_t sentinel_code;
};

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;

size_t radix_sort_temp_bytes(uint32_t count);

// Stable sort of count pairs by the low ``bits`` bits of the (transformed)
// key, ping-ponging between buffer A and buffer B.  If ``vals_iota`` the
// values of A are not read and value i is taken to be i.  ``*in_b`` is set
// to 1 if the sorted result is in B, 0 if it is in A.  bits == 0 leaves the
// data in A (and materialises the iota values if asked).  If ``count_dev`` is
// not null, the number of pairs is min(count, *count_dev), read on the device
// (launch sizes follow ``count``, which is then a capacity).
hipError_t radix_sort_pairs(uint32_t *keys_a, uint32_t *vals_a, uint32_t *keys_b, uint32_t *vals_b,
                            uint32_t count, int bits, bool vals_iota, KeyTransform xf, void *temp,
                            hipStream_t s, int *in_b, const uint32_t *count_dev = nullptr);

}  // namespace ddm

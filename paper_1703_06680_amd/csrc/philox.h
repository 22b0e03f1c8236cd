// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
// as easy as 1, 2, 3", SC 2011) and the Irwin-Hall normal of the random-walk
// motion, shared by the step kernels of sim.hip and resident.hip so that both
// move a region by the same bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddm {

// One round: the two 32 x 32 -> 64-bit products, each taken whole (one
// v_mad_u64_u32 rather than separate low and high multiplies).
__device__ __forceinline__ uint4 philox_round(uint4 x, uint32_t k0, uint32_t k1) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * x.x;
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * x.z;
  return make_uint4((uint32_t)(p1 >> 32) ^ x.y ^ k0, (uint32_t)p1,
                    (uint32_t)(p0 >> 32) ^ x.w ^ k1, (uint32_t)p0);
}

__device__ __forceinline__ uint4 philox4x32_10(uint4 ctr, uint32_t k0, uint32_t k1) {
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    ctr = philox_round(ctr, k0, k1);
    k0 += W0;
    k1 += W1;
  }
  return ctr;
}

// z for (region, axis, step): twelve 24-bit uniforms from three Philox draws.
__device__ __forceinline__ float irwin_hall12(uint32_t region, uint32_t axis, uint32_t step,
                                              uint32_t k0, uint32_t k1) {
  uint32_t sum = 0;
#pragma unroll
  for (uint32_t j = 0; j < 3; ++j) {
    const uint4 w = philox4x32_10(make_uint4(region, axis, step, j), k0, k1);
    sum += (w.x >> 8) + (w.y >> 8) + (w.z >> 8) + (w.w >> 8);
  }
  // sum < 12 * 2^24 < 2^28: exact in uint32; one rounding to float32
  const float s = __uint2float_rn(sum);
  return s * 5.9604644775390625e-08f - 6.0f;  // 2^-24
}

}  // namespace ddm

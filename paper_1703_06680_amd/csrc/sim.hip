// Random-walk step of a resident simulation (the serving workload's motion).
//
// Every step moves each region's lower corner on every axis by sigma * z and
// resets the upper corner to lo + side, so sides never drift.  z is a
// bounded approximation of a standard normal, the Irwin-Hall sum of twelve
// uniforms minus six, whose uniforms come from the counter-based generator
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): counter = (region, axis, step, draw), key =
// the simulation's 64-bit seed.  Every operation after the integer sum is a
// single IEEE float32 operation (int-to-float conversion, multiplication by a
// power of two, subtraction, multiplication, addition, each rounded to
// nearest), so any implementation that follows the same definition gets the
// same bits.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.h"
#include "sim.h"

namespace ddm {
namespace {

__global__ void walk_kernel(float *__restrict__ lo, float *__restrict__ hi, uint32_t rows, int d,
                            uint32_t region0, float side, float sigma, uint32_t step, uint32_t k0,
                            uint32_t k1) {
  const uint32_t total = rows * (uint32_t)d;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += gridDim.x * blockDim.x) {
    const uint32_t r = i / (uint32_t)d, k = i - r * (uint32_t)d;
    const float z = irwin_hall12(region0 + r, k, step, k0, k1);
    const float moved = __fadd_rn(lo[i], __fmul_rn(sigma, z));
    lo[i] = moved;
    hi[i] = __fadd_rn(moved, side);
  }
}

}  // namespace

hipError_t launch_walk(const WalkArgs &w, hipStream_t s) {
  const uint32_t k0 = (uint32_t)w.seed, k1 = (uint32_t)(w.seed >> 32);
  const uint64_t nu = (uint64_t)w.n * (uint64_t)w.d, nm = (uint64_t)w.m * (uint64_t)w.d;
  if (nu) {
    const unsigned grid = (unsigned)((nu + 255) / 256 < 4096 ? (nu + 255) / 256 : 4096);
    walk_kernel<<<grid, 256, 0, s>>>(w.upd_lo, w.upd_hi, (uint32_t)w.n, w.d, 0u, w.side, w.sigma,
                                     w.step, k0, k1);
  }
  if (nm) {
    const unsigned grid = (unsigned)((nm + 255) / 256 < 4096 ? (nm + 255) / 256 : 4096);
    walk_kernel<<<grid, 256, 0, s>>>(w.sub_lo, w.sub_hi, (uint32_t)w.m, w.d, (uint32_t)w.n,
                                     w.side, w.sigma, w.step, k0, k1);
  }
  return hipGetLastError();
}

}  // namespace ddm

extern "C" int ddm_sim_step(float *upd_lo, float *upd_hi, int64_t n, float *sub_lo,
                            float *sub_hi, int64_t m, int d, float side, float sigma,
                            uint64_t seed, uint32_t step, void *stream) {
  if (n < 0 || m < 0 || d < 1 || d > DDM_MAX_DIMS || (n + m) * (int64_t)d >= (int64_t(1) << 32))
    return DDM_E_INVAL;
  if ((n > 0 && (!upd_lo || !upd_hi)) || (m > 0 && (!sub_lo || !sub_hi))) return DDM_E_INVAL;
  ddm::WalkArgs w{upd_lo, upd_hi, n, sub_lo, sub_hi, m, d, side, sigma, seed, step};
  return ddm::launch_walk(w, static_cast<hipStream_t>(stream)) == hipSuccess ? DDM_OK
                                                                            : DDM_E_DEVICE;
}

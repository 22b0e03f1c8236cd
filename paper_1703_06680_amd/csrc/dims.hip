// Per-axis 1-D candidate counts (declared in include/ddm.h).
//
// For every axis k, K_1D(k) is the number of (update, subscription) pairs
// whose intervals on axis k intersect, among the regions that are non-empty
// on every axis: the pairs a sweep along axis k examines before the other
// axes filter them (Sec. 3, the reduction of d axes to one after Algorithm
// 1).  Each axis is extracted into a one-dimensional problem (regions that
// are empty on some axis become empty intervals, invalid regions get a NaN
// so that the matcher reports them) and counted by the d = 1 matcher.
#include <stddef.h>
#include <stdint.h>

#include "../../include/ddm.h"
#include "internal.h"
#include "common.h"

namespace ddm {
namespace {

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

__global__ void axis_column_kernel(const float *__restrict__ lo, const float *__restrict__ hi,
                                   uint32_t rows, int d, int k, float *__restrict__ out_lo,
                                   float *__restrict__ out_hi) {
  const float nan = __int_as_float(0x7fc00000);
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < rows;
       r += gridDim.x * blockDim.x) {
    bool bad = false, empty = false;
    for (int a = 0; a < d; ++a) {
      const float l = lo[(size_t)r * d + a], h = hi[(size_t)r * d + a];
      bad = bad || l != l || h != h || l > h;
      empty = empty || l == h;
    }
    const float l = lo[(size_t)r * d + k], h = hi[(size_t)r * d + k];
    out_lo[r] = bad ? nan : (empty ? h : l);
    out_hi[r] = h;
  }
}

void launch_column(const float *lo, const float *hi, int64_t rows, int d, int k, float *out_lo,
                   float *out_hi, hipStream_t s) {
  if (rows <= 0) return;
  const unsigned grid = (unsigned)((rows + 255) / 256 < 4096 ? (rows + 255) / 256 : 4096);
  axis_column_kernel<<<grid, 256, 0, s>>>(lo, hi, (uint32_t)rows, d, k, out_lo, out_hi);
}

}  // namespace
}  // namespace ddm

using namespace ddm;

extern "C" size_t ddm_dim_counts_workspace_bytes(int64_t n, int64_t m, int d) {
  if (n < 0 || m < 0 || d < 1 || d > DDM_MAX_DIMS) return 0;
  const size_t inner = ddm_workspace_bytes(n, m, 1, DDM_COUNT, 0);
  if (inner == 0) return 0;
  return 2 * align256((size_t)n * sizeof(float)) + 2 * align256((size_t)m * sizeof(float)) + inner;
}

extern "C" int ddm_dim_counts(const float *upd_lo, const float *upd_hi, int64_t n,
                              const float *sub_lo, const float *sub_hi, int64_t m, int d,
                              void *workspace, size_t ws_bytes, void *stream,
                              uint64_t *counts_host) {
  if (n < 0 || m < 0 || d < 1 || d > DDM_MAX_DIMS || !counts_host) return DDM_E_INVAL;
  if ((n > 0 && (!upd_lo || !upd_hi)) || (m > 0 && (!sub_lo || !sub_hi))) return DDM_E_INVAL;
  const size_t need = ddm_dim_counts_workspace_bytes(n, m, d);
  if (need == 0) return DDM_E_INVAL;
  if (!workspace || ws_bytes < need) return DDM_E_WORKSPACE;
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return DDM_E_INVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *w = static_cast<char *>(workspace);
  float *ul = reinterpret_cast<float *>(w);
  w += align256((size_t)n * sizeof(float));
  float *uh = reinterpret_cast<float *>(w);
  w += align256((size_t)n * sizeof(float));
  float *sl = reinterpret_cast<float *>(w);
  w += align256((size_t)m * sizeof(float));
  float *sh = reinterpret_cast<float *>(w);
  w += align256((size_t)m * sizeof(float));
  const size_t inner = need - (size_t)(w - static_cast<char *>(workspace));
  for (int k = 0; k < d; ++k) {
    launch_column(upd_lo, upd_hi, n, d, k, ul, uh, s);
    launch_column(sub_lo, sub_hi, m, d, k, sl, sh, s);
    if (hipGetLastError() != hipSuccess) return DDM_E_DEVICE;
    uint64_t K = 0;
    const int rc = match_quiet(ul, uh, n, sl, sh, m, 1, DDM_COUNT, w, inner, stream, &K, nullptr,
                             nullptr, 0);
    if (rc != DDM_OK) return rc;
    counts_host[k] = K;
  }
  return DDM_OK;
}

// C interface of libddm (declared in include/ddm.h).
//
// ddm_match() enqueues the whole matching pipeline on the caller's stream and
// synchronises once to learn how many regions are non-empty and the key range
// (which fixes the number of radix passes), and once more at the end to return
// the total; in pair mode it also synchronises after the counting sweep to
// size the pair list.
#include <string.h>

#include "../../include/ddm.h"
#include "common.h"
#include "match_global.h"
#include "primitives.h"
#include "profile.h"

namespace ddm {
namespace {

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of every workspace buffer; size 0 means "not used".
struct Layout {
  size_t hdr, partial, klo, khi, vals_a, keys_b, vals_b, sort_tmp, s_khi, s_other;
  size_t cnt, off, cur, pu, ps, pu2, ps2, scan_tmp, pair_sort_tmp;
  size_t total;
};

Layout make_layout(int64_t n, int64_t m, int d, int mode, int64_t cap) {
  Layout L{};
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t o = at;
    at += align256(bytes);
    return o;
  };
  const size_t N = (size_t)(n + m);
  const size_t u4 = N * sizeof(uint32_t);
  L.hdr = take(sizeof(Header));
  L.partial = take(kKeysMaxBlocks * sizeof(uint4));
  L.klo = take(u4);
  L.khi = take(u4);
  L.vals_a = take(u4);
  L.keys_b = take(u4);
  L.vals_b = take(u4);
  L.sort_tmp = take(radix_sort_temp_bytes((uint32_t)N));
  L.s_khi = take(u4);
  L.s_other = take((size_t)2 * (d - 1) * u4);
  if (mode == DDM_PAIRS) {
    const size_t c = (size_t)(cap > 0 ? cap : 0);
    L.cnt = take((size_t)n * sizeof(int32_t));
    L.off = take((size_t)n * sizeof(unsigned long long));
    L.cur = take((size_t)n * sizeof(uint32_t));
    L.pu = take(c * sizeof(uint32_t));
    L.ps = take(c * sizeof(uint32_t));
    L.pu2 = take(c * sizeof(uint32_t));
    L.ps2 = take(c * sizeof(uint32_t));
    L.scan_tmp = take(scan_temp_bytes((size_t)n));
    L.pair_sort_tmp = take(radix_sort_temp_bytes((uint32_t)(c ? c : 1)));
  }
  L.total = at;
  return L;
}

bool sizes_ok(int64_t n, int64_t m, int d, int mode) {
  if (n < 0 || m < 0) return false;
  if (n + m >= (int64_t(1) << 31)) return false;
  if (d < 1 || d > DDM_MAX_DIMS) return false;
  if (mode != DDM_COUNT && mode != DDM_PER_UPDATE && mode != DDM_PAIRS) return false;
  return true;
}

int bit_length(uint32_t x) { return x ? 32 - __builtin_clz(x) : 0; }

#define DDM_HIP(call)                          \
  do {                                         \
    if ((call) != hipSuccess) return DDM_E_DEVICE; \
  } while (0)

template <typename T>
T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// Sorts (u, s) pair staging buffers lexicographically: stable by s, then
// stable by u.  Returns the buffers holding the result.
hipError_t order_pairs(uint32_t *pu, uint32_t *ps, uint32_t *pu2, uint32_t *ps2, uint32_t K,
                       int64_t n, int64_t m, void *tmp, hipStream_t s, uint32_t **res_u,
                       uint32_t **res_s) {
  KeyTransform raw{0, 0, 0};
  int in_b = 0;
  hipError_t e = radix_sort_pairs(ps, pu, ps2, pu2, K, bit_length((uint32_t)(m > 0 ? m - 1 : 0)),
                                  false, raw, tmp, s, &in_b);
  if (e != hipSuccess) return e;
  uint32_t *sk = in_b ? ps2 : ps, *sv = in_b ? pu2 : pu;  // keys = s, vals = u
  uint32_t *ok = in_b ? ps : ps2, *ov = in_b ? pu : pu2;  // free pair of buffers
  e = radix_sort_pairs(sv, sk, ok, ov, K, bit_length((uint32_t)(n > 0 ? n - 1 : 0)), false, raw,
                       tmp, s, &in_b);
  if (e != hipSuccess) return e;
  *res_u = in_b ? ok : sv;
  *res_s = in_b ? ov : sk;
  return hipSuccess;
}

}  // namespace
}  // namespace ddm

using namespace ddm;

extern "C" size_t ddm_workspace_bytes(int64_t n, int64_t m, int d, int mode,
                                      int64_t pair_capacity) {
  if (!sizes_ok(n, m, d, mode) || pair_capacity < 0) return 0;
  return make_layout(n, m, d, mode, pair_capacity).total;
}

extern "C" const char *ddm_strerror(int code) {
  switch (code) {
    case DDM_OK: return "success";
    case DDM_E_INVAL: return "invalid argument or input (NaN coordinate, lo > hi, bad size or pointer)";
    case DDM_E_CAPACITY: return "pair buffer too small (count_host holds the number of pairs)";
    case DDM_E_WORKSPACE: return "workspace smaller than ddm_workspace_bytes()";
    case DDM_E_DEVICE: return "HIP runtime error";
    case DDM_E_UNSUPPORTED: return "request outside the supported range";
    default: return "unknown error";
  }
}

extern "C" int ddm_match(const float *upd_lo, const float *upd_hi, int64_t n, const float *sub_lo,
                         const float *sub_hi, int64_t m, int d, int mode, void *workspace,
                         size_t ws_bytes, void *stream, uint64_t *count_host, int32_t *per_update,
                         int32_t *pairs, int64_t pair_capacity) {
  // ---------------------------------------------------- host-side checks
  if (!sizes_ok(n, m, d, mode) || !count_host || pair_capacity < 0) return DDM_E_INVAL;
  if ((n > 0 && (!upd_lo || !upd_hi)) || (m > 0 && (!sub_lo || !sub_hi))) return DDM_E_INVAL;
  if (mode == DDM_PER_UPDATE && n > 0 && !per_update) return DDM_E_INVAL;
  if (mode == DDM_PAIRS && pair_capacity > 0 && !pairs) return DDM_E_INVAL;
  const Layout L = make_layout(n, m, d, mode, pair_capacity);
  if (!workspace || ws_bytes < L.total) return DDM_E_WORKSPACE;
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return DDM_E_INVAL;
  *count_host = 0;

  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint32_t un = (uint32_t)n, um = (uint32_t)m, N = un + um;
  Header *hdr = at<Header>(workspace, L.hdr);
  int32_t *cnt = mode == DDM_PAIRS ? (per_update ? per_update : at<int32_t>(workspace, L.cnt))
                                   : per_update;
  const bool want_counts = mode != DDM_COUNT;

  DDM_HIP(hipMemsetAsync(hdr, 0, sizeof(Header), s));
  DDM_HIP(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(&hdr->kmin), 0xFFFFFFFFu, 1, s));
  if (want_counts && n > 0) DDM_HIP(hipMemsetAsync(cnt, 0, (size_t)n * sizeof(int32_t), s));
  if (N == 0) return DDM_OK;

  // ---------------------------------------- 1. validate, encode, empties
  uint32_t *klo = at<uint32_t>(workspace, L.klo);
  uint32_t *khi = at<uint32_t>(workspace, L.khi);
  const int axis = 0;
  launch_keys(upd_lo, upd_hi, un, sub_lo, sub_hi, um, d, axis, klo, khi,
              at<uint4>(workspace, L.partial), hdr, s);
  DDM_HIP(hipGetLastError());
  Header h{};
  prof::end(s);
  DDM_HIP(hipMemcpyAsync(&h, hdr, sizeof(Header), hipMemcpyDeviceToHost, s));
  DDM_HIP(hipStreamSynchronize(s));
  prof::flush();
  if (h.err) return DDM_E_INVAL;
  const uint32_t nne = h.nonempty;
  if (nne == 0 || n == 0 || m == 0) return DDM_OK;  // counts already zeroed

  // ---------------------------------------------------- 2. radix sort
  const bool has_empty = nne < N;
  const uint32_t range = h.kmax - h.kmin;
  KeyTransform xf{1u, h.kmin, range + 1u};
  const int bits = bit_length(has_empty ? range + 1u : range);
  uint32_t *vals_a = at<uint32_t>(workspace, L.vals_a);
  uint32_t *keys_b = at<uint32_t>(workspace, L.keys_b);
  uint32_t *vals_b = at<uint32_t>(workspace, L.vals_b);
  int in_b = 0;
  DDM_HIP(radix_sort_pairs(klo, vals_a, keys_b, vals_b, N, bits, true, xf,
                           at<void>(workspace, L.sort_tmp), s, &in_b));
  const uint32_t *skey = in_b ? keys_b : klo;
  const uint32_t *sidx = in_b ? vals_b : vals_a;

  // --------------------------------------- 3. other axes in sorted order
  uint32_t *s_khi = at<uint32_t>(workspace, L.s_khi);
  float *s_other = at<float>(workspace, L.s_other);
  launch_gather(sidx, nne, khi, upd_lo, upd_hi, un, sub_lo, sub_hi, d, axis, s_khi, s_other, N, s);
  DDM_HIP(hipGetLastError());

  // ------------------------------------------------------- 4. the sweep
  SweepArgs a{};
  a.skey = skey;
  a.sidx = sidx;
  a.s_khi = s_khi;
  a.s_other = s_other;
  a.stride = N;
  a.count = nne;
  a.n = un;
  a.dm1 = d - 1;
  a.per_update = cnt;
  a.total = &hdr->total;
  launch_sweep(want_counts ? 1 : 0, a, s);
  DDM_HIP(hipGetLastError());
  unsigned long long K = 0;
  prof::end(s);
  DDM_HIP(hipMemcpyAsync(&K, &hdr->total, sizeof(K), hipMemcpyDeviceToHost, s));
  DDM_HIP(hipStreamSynchronize(s));
  prof::flush();
  *count_host = K;
  if (mode != DDM_PAIRS || K == 0) return DDM_OK;
  if ((int64_t)K > pair_capacity) return DDM_E_CAPACITY;
  if (K >= (1ull << 32)) return DDM_E_UNSUPPORTED;  // pair staging uses 32-bit positions

  // -------------------------------------- 5. pairs: two-pass compaction
  unsigned long long *off = at<unsigned long long>(workspace, L.off);
  uint32_t *cur = at<uint32_t>(workspace, L.cur);
  uint32_t *pu = at<uint32_t>(workspace, L.pu), *ps = at<uint32_t>(workspace, L.ps);
  uint32_t *pu2 = at<uint32_t>(workspace, L.pu2), *ps2 = at<uint32_t>(workspace, L.ps2);
  launch_widen(cnt, off, (size_t)n, s);
  DDM_HIP(exclusive_scan_u64(off, off, (size_t)n, at<void>(workspace, L.scan_tmp), s));
  prof::mark(s, "pairs.memset");
  DDM_HIP(hipMemsetAsync(cur, 0, (size_t)n * sizeof(uint32_t), s));
  a.offsets = off;
  a.cursor = cur;
  a.out_u = pu;
  a.out_s = ps;
  a.total = &hdr->aux[0];
  launch_sweep(2, a, s);
  DDM_HIP(hipGetLastError());
  uint32_t *ru = nullptr, *rs = nullptr;
  DDM_HIP(order_pairs(pu, ps, pu2, ps2, (uint32_t)K, n, m, at<void>(workspace, L.pair_sort_tmp), s,
                      &ru, &rs));
  launch_interleave(ru, rs, pairs, (size_t)K, s);
  DDM_HIP(hipGetLastError());
  prof::end(s);
  DDM_HIP(hipStreamSynchronize(s));
  prof::flush();
  return DDM_OK;
}

// Per-phase GPU timing with HIP events; see profile.h.
#include <stdio.h>
#include <string.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/ddm.h"
#include "profile.h"

namespace ddm {
namespace prof {
namespace {

struct Mark {
  hipEvent_t ev;
  const char *phase;  // nullptr closes the previous phase
};

struct Totals {
  double ms = 0.0;
  long long launches = 0;
};

bool g_on = false;
std::vector<hipEvent_t> g_pool;
std::vector<Mark> g_marks;
std::map<std::string, Totals> g_totals;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

bool enabled() { return g_on; }

bool swap_enabled(bool on) {
  const bool was = g_on;
  g_on = on;
  return was;
}

void mark(hipStream_t s, const char *phase) {
  if (!g_on) return;
  hipEvent_t e = take_event();
  if (!e) return;
  if (hipEventRecord(e, s) != hipSuccess) {
    g_pool.push_back(e);
    return;
  }
  g_marks.push_back({e, phase});
}

void end(hipStream_t s) { mark(s, nullptr); }

void flush() {
  if (g_marks.empty()) return;
  for (size_t i = 0; i + 1 < g_marks.size(); ++i) {
    if (!g_marks[i].phase) continue;
    float ms = 0.f;
    if (hipEventSynchronize(g_marks[i + 1].ev) == hipSuccess &&
        hipEventElapsedTime(&ms, g_marks[i].ev, g_marks[i + 1].ev) == hipSuccess) {
      Totals &t = g_totals[g_marks[i].phase];
      t.ms += ms;
      t.launches += 1;
    }
  }
  for (auto &m : g_marks) g_pool.push_back(m.ev);
  g_marks.clear();
}

}  // namespace prof
}  // namespace ddm

using namespace ddm;

extern "C" int ddm_profile(int enable) {
  prof::flush();
  if (enable) prof::g_totals.clear();
  prof::g_on = enable != 0;
  return DDM_OK;
}

extern "C" int ddm_profile_report(char *buf, size_t len) {
  prof::flush();
  std::string out = "{";
  bool first = true;
  char tmp[256];
  for (auto &kv : prof::g_totals) {
    snprintf(tmp, sizeof(tmp), "%s\"%s\": {\"ms\": %.6f, \"launches\": %lld}", first ? "" : ", ",
             kv.first.c_str(), kv.second.ms, kv.second.launches);
    out += tmp;
    first = false;
  }
  out += "}";
  if (!buf || len <= out.size()) return (int)out.size() + 1;
  memcpy(buf, out.c_str(), out.size() + 1);
  return DDM_OK;
}

// ------------------------------------------------ achievable bandwidth
//
// A plain device copy: 16-byte loads and stores in a grid-stride loop, eight
// workgroups of 512 threads per CU.  Its rate is the bandwidth a streaming
// kernel can reach on this device, the yardstick beside the published peak.
namespace {

__global__ __launch_bounds__(512) void copy_probe_kernel(uint4 *__restrict__ dst,
                                                         const uint4 *__restrict__ src,
                                                         size_t count) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    dst[i] = src[i];
}

}  // namespace

extern "C" int ddm_copy_probe(void *dst, const void *src, size_t bytes, int reps, void *stream,
                              double *ms_out) {
  if (!dst || !src || !ms_out || reps < 1 || (bytes & 15) ||
      (reinterpret_cast<uintptr_t>(dst) & 15) || (reinterpret_cast<uintptr_t>(src) & 15))
    return DDM_E_INVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t count = bytes / 16;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return DDM_E_DEVICE;
  const unsigned grid = (unsigned)(cus > 0 ? cus * 8 : 2048);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return DDM_E_DEVICE;
  int rc = DDM_OK;
  copy_probe_kernel<<<grid, 512, 0, s>>>(static_cast<uint4 *>(dst),
                                         static_cast<const uint4 *>(src), count);  // warm-up
  if (hipEventRecord(e0, s) != hipSuccess) rc = DDM_E_DEVICE;
  for (int r = 0; rc == DDM_OK && r < reps; ++r)
    copy_probe_kernel<<<grid, 512, 0, s>>>(static_cast<uint4 *>(dst),
                                           static_cast<const uint4 *>(src), count);
  float ms = 0.f;
  if (rc == DDM_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                       hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess))
    rc = DDM_E_DEVICE;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == DDM_OK) *ms_out = (double)ms / reps;
  return rc;
}

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

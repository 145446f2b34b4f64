// qv_timing.hip -- optional per-kernel timing: while enabled, every kernel
// launch of the library is bracketed by two hipEvents recorded on the launch
// stream, and qv_timing_read sums the elapsed times by kernel name.
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qv_internal.h"

namespace qv {

namespace {
struct Rec {
  const char *name;
  int tag;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

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

TimingScope::TimingScope(const char *name, hipStream_t st, int tag)
    : name_(name), st_(st), ev_(nullptr), tag_(tag) {
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_on) return;
  ev_ = take_event();
  if (ev_ && hipEventRecord((hipEvent_t)ev_, st_) != hipSuccess) ev_ = nullptr;
}

TimingScope::~TimingScope() {
  if (!ev_) return;
  std::lock_guard<std::mutex> g(g_mu);
  hipEvent_t e = take_event();
  if (!e) return;
  if (hipEventRecord(e, st_) != hipSuccess) return;
  g_recs.push_back({name_, tag_, (hipEvent_t)ev_, e});
}

}  // namespace qv

using namespace qv;

extern "C" {

int32_t qv_timing_enable(int32_t on) {
  std::lock_guard<std::mutex> g(g_mu);
  g_on = on != 0;
  for (auto &r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  return QV_OK;
}

int32_t qv_timing_read(qv_kernel_time *out, int32_t max_entries, int32_t *n_out) {
  if (!out || max_entries < 0 || !n_out) return QV_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(g_mu);
  int32_t n = 0;
  for (auto &r : g_recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess) return QV_ERR_HIP;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return QV_ERR_HIP;
    // a template name with a comma reaches the launch macro in parentheses
    const char *base = r.name;
    int len = (int)std::strlen(base);
    if (len >= 2 && base[0] == '(' && base[len - 1] == ')') {
      ++base;
      len -= 2;
    }
    char nm[sizeof out[0].name];
    if (r.tag >= 0)
      std::snprintf(nm, sizeof nm, "%.*s@L%d", len, base, r.tag);
    else
      std::snprintf(nm, sizeof nm, "%.*s", len, base);
    int32_t i = 0;
    while (i < n && std::strncmp(out[i].name, nm, sizeof out[i].name) != 0) ++i;
    if (i == n) {
      if (n == max_entries) continue;
      std::memset(&out[n], 0, sizeof out[n]);
      std::strncpy(out[n].name, nm, sizeof out[n].name - 1);
      ++n;
    }
    out[i].launches += 1;
    out[i].total_ms += ms;
  }
  *n_out = n;
  for (auto &r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  return QV_OK;
}

}  // extern "C"

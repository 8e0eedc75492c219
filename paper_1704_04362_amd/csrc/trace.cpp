// Launch tracing: while enabled, every TraceScope records a HIP event pair
// on the caller's stream around the kernels it encloses; the C ABI reports
// per-name call counts and summed durations. Used to time the stages of a
// call inside a caller's own timed region, on the stream the work runs on.
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace tp {
namespace {

struct Rec {
  std::string name;
  hipEvent_t e0, e1;
};

struct Agg {
  std::string name;
  int64_t calls = 0;
  double ms = 0.0;
};

std::mutex g_mu;
int g_mode = 0;  // 0 off, 1 every stage, 2 the slice-product stages only
std::vector<Rec> g_recs;
std::vector<Agg> g_aggs;

void drop_records() {
  for (auto& r : g_recs) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  g_recs.clear();
}

}  // namespace

bool trace_on(const char* name) {
  int mode;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    mode = g_mode;
  }
  if (mode == 1) return true;
  if (mode != 2) return false;
  const std::string n(name);
  return n.size() >= 5 && n.compare(n.size() - 5, 5, ".gemm") == 0;
}

TraceScope::TraceScope(const char* name, hipStream_t st) : name_(name), st_(st) {
  if (!trace_on(name)) return;
  if (hipEventCreate(&e0_) != hipSuccess) return;
  if (hipEventCreate(&e1_) != hipSuccess) {
    (void)hipEventDestroy(e0_);
    return;
  }
  if (hipEventRecord(e0_, st_) != hipSuccess) {
    (void)hipEventDestroy(e0_);
    (void)hipEventDestroy(e1_);
    return;
  }
  live_ = true;
}

TraceScope::~TraceScope() {
  if (!live_) return;
  if (hipEventRecord(e1_, st_) != hipSuccess) {
    (void)hipEventDestroy(e0_);
    (void)hipEventDestroy(e1_);
    return;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_recs.push_back(Rec{name_, e0_, e1_});
}

}  // namespace tp

using namespace tp;

extern "C" {

int tp_trace_enable(int on) {
  if (on < 0 || on > 2) return fail(TP_EINVAL, "trace: mode must be 0, 1 or 2");
  std::lock_guard<std::mutex> lk(g_mu);
  if (on) {
    drop_records();
    g_aggs.clear();
  }
  g_mode = on;
  return TP_OK;
}

int tp_trace_count(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  std::map<std::string, Agg> by;
  for (auto& a : g_aggs) by[a.name] = a;
  for (auto& r : g_recs) {
    if (hipEventSynchronize(r.e1) != hipSuccess) return fail(TP_EHIP, "trace: event synchronize failed");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) return fail(TP_EHIP, "trace: elapsed time failed");
    Agg& a = by[r.name];
    a.name = r.name;
    a.calls += 1;
    a.ms += ms;
  }
  drop_records();
  g_aggs.clear();
  for (auto& kv : by) g_aggs.push_back(kv.second);
  return (int)g_aggs.size();
}

int tp_trace_entry(int i, char* name, size_t name_cap, int64_t* calls, double* total_ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (i < 0 || i >= (int)g_aggs.size()) return fail(TP_EINVAL, "trace: entry index out of range");
  if (name && name_cap > 0) {
    const std::string& n = g_aggs[i].name;
    const size_t len = n.size() < name_cap - 1 ? n.size() : name_cap - 1;
    n.copy(name, len);
    name[len] = '\0';
  }
  if (calls) *calls = g_aggs[i].calls;
  if (total_ms) *total_ms = g_aggs[i].ms;
  return TP_OK;
}

}  // extern "C"

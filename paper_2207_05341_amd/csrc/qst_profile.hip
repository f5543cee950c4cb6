// Optional per-kernel timing: when enabled, each timed scope of the library
// (one kernel, or a fixed short sequence under one name) is bracketed by two
// hipEvents recorded on its launch stream (or, for a single kernel, taken
// by its launch as start and stop events).  The report waits for the events
// and sums the elapsed times per kernel name.
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "qst_kernels.h"

namespace qst {

namespace {

struct Pending {
  std::string name;
  hipEvent_t a, b;
};

struct State {
  std::mutex mu;
  bool enabled = false;
  std::string only;  // empty: every scope
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<long long, double>> totals;  // calls, ms
};

State& state() {
  static State s;
  return s;
}

hipEvent_t take_event(State& st) {
  if (!st.pool.empty()) {
    hipEvent_t e = st.pool.back();
    st.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  // timing-only events: no system-scope fence (cache write-back and
  // invalidate) when they complete
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

ProfScope::ProfScope(const char* name, hipStream_t s, bool in_launch) : s_(s), in_launch_(in_launch) {
  State& st = state();
  std::lock_guard<std::mutex> lock(st.mu);
  if (!st.enabled) return;
  if (!st.only.empty() && st.only != name) return;
  hipEvent_t a = take_event(st), b = take_event(st);
  if (!a || !b) return;
  if (!in_launch && hipEventRecord(a, s) != hipSuccess) return;
  st.pending.push_back({name, a, b});
  idx_ = int(st.pending.size()) - 1;
  if (in_launch) {
    a_ = a;
    b_ = b;
  }
}

ProfScope::~ProfScope() {
  if (idx_ < 0 || in_launch_) return;
  State& st = state();
  std::lock_guard<std::mutex> lock(st.mu);
  if (idx_ < int(st.pending.size())) (void)hipEventRecord(st.pending[idx_].b, s_);
}

}  // namespace qst

extern "C" {

qst_status qst_profile_enable(int on, const char* only) {
  qst::State& st = qst::state();
  std::lock_guard<std::mutex> lock(st.mu);
  st.enabled = on != 0;
  st.only = only ? only : "";
  return QST_OK;
}

size_t qst_profile_report(char* buf, size_t len, int reset) {
  qst::State& st = qst::state();
  std::lock_guard<std::mutex> lock(st.mu);
  for (auto& p : st.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      auto& t = st.totals[p.name];
      t.first += 1;
      t.second += double(ms);
    }
    st.pool.push_back(p.a);
    st.pool.push_back(p.b);
  }
  st.pending.clear();
  std::string out;
  char line[256];
  for (const auto& kv : st.totals) {
    std::snprintf(line, sizeof(line), "%s %lld %.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
    out += line;
  }
  if (reset) st.totals.clear();
  if (buf && len > 0) {
    const size_t n = out.size() < len - 1 ? out.size() : len - 1;
    out.copy(buf, n);
    buf[n] = '\0';
  }
  return out.size() + 1;
}

}  // extern "C"

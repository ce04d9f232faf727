// Opt-in stage timing with HIP events, recorded on the stream each stage is launched on.
//
// When a stage is enabled, the library records an event pair around that stage's launches;
// varlingam_profile_read() waits for the recorded events and returns the accumulated elapsed
// time.  Disabled stages cost one relaxed atomic load per launch site.
#include <atomic>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "profile.hpp"

namespace vl {
namespace {

struct Rec {
  hipEvent_t a, b;
};

struct Stage {
  std::vector<Rec> pending;
  double ms = 0.0;
  int64_t count = 0;
};

std::mutex g_mu;
std::atomic<bool> g_any{false};
std::string g_enabled;                       // comma separated stage names, or "*"
std::unordered_map<std::string, Stage> g_stages;
std::vector<hipEvent_t> g_pool;

bool enabled_locked(const char* name) {
  if (g_enabled == "*") return true;
  const std::string n(name);
  size_t pos = 0;
  while (pos <= g_enabled.size()) {
    size_t e = g_enabled.find(',', pos);
    if (e == std::string::npos) e = g_enabled.size();
    if (g_enabled.compare(pos, e - pos, n) == 0 && e - pos == n.size()) return true;
    pos = e + 1;
  }
  return false;
}

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

void drain_locked(Stage& s) {
  for (Rec& r : s.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      s.ms += ms;
      s.count += 1;
    }
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  s.pending.clear();
}

}  // namespace

ProfileScope::ProfileScope(const char* name, hipStream_t stream) : name_(name), stream_(stream) {
  if (!g_any.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!enabled_locked(name)) return;
  start_ = take_event();
  if (start_ && hipEventRecord(static_cast<hipEvent_t>(start_), stream) != hipSuccess) {
    g_pool.push_back(static_cast<hipEvent_t>(start_));
    start_ = nullptr;
  }
}

ProfileScope::~ProfileScope() {
  if (!start_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t stop = take_event();
  if (!stop || hipEventRecord(stop, stream_) != hipSuccess) {
    g_pool.push_back(static_cast<hipEvent_t>(start_));
    return;
  }
  g_stages[name_].pending.push_back(Rec{static_cast<hipEvent_t>(start_), stop});
}

}  // namespace vl

extern "C" {

void varlingam_profile_enable(const char* stages) {
  std::lock_guard<std::mutex> lk(vl::g_mu);
  for (auto& kv : vl::g_stages) vl::drain_locked(kv.second);
  vl::g_stages.clear();
  vl::g_enabled = stages ? stages : "";
  vl::g_any.store(!vl::g_enabled.empty(), std::memory_order_relaxed);
}

int varlingam_profile_read(const char* stage, double* total_ms, int64_t* count) {
  if (!stage || !total_ms || !count) return VL_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(vl::g_mu);
  auto it = vl::g_stages.find(stage);
  if (it == vl::g_stages.end()) {
    *total_ms = 0.0;
    *count = 0;
    return VL_OK;
  }
  vl::drain_locked(it->second);
  *total_ms = it->second.ms;
  *count = it->second.count;
  return VL_OK;
}

}  // extern "C"

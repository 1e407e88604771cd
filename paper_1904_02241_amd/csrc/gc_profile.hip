// Per-kernel timing with HIP events recorded on the launching stream around
// every launch while profiling is on (gc_profile).

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gc_internal.h"

namespace {

struct Record {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  double total_ms = 0.0;
  int64_t launches = 0;
};

std::mutex g_mu;
bool g_on = false;
std::map<std::string, Record> g_rec;
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

// Waits for all pending event pairs and folds them into the totals.
hipError_t drain() {
  for (auto& kv : g_rec) {
    for (auto& pr : kv.second.pending) {
      hipError_t e = hipEventSynchronize(pr.second);
      if (e != hipSuccess) return e;
      float ms = 0.0f;
      e = hipEventElapsedTime(&ms, pr.first, pr.second);
      if (e != hipSuccess) return e;
      kv.second.total_ms += ms;
      kv.second.launches += 1;
      g_pool.push_back(pr.first);
      g_pool.push_back(pr.second);
    }
    kv.second.pending.clear();
  }
  return hipSuccess;
}

}  // namespace

namespace gcx {

ProfScope::ProfScope(const char* name, hipStream_t s) : name_(name), s_(s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  start_ = take_event();
  stop_ = take_event();
  if (start_ && stop_ && hipEventRecord(start_, s_) == hipSuccess) return;
  start_ = stop_ = nullptr;
}

ProfScope::~ProfScope() {
  if (!start_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (hipEventRecord(stop_, s_) == hipSuccess) g_rec[name_].pending.emplace_back(start_, stop_);
}

}  // namespace gcx

extern "C" {

int gc_profile(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (enable) {
    const hipError_t e = drain();
    g_rec.clear();
    g_on = true;
    return e == hipSuccess ? GC_OK : GC_EHIP;
  }
  g_on = false;
  return drain() == hipSuccess ? GC_OK : GC_EHIP;
}

int gc_profile_count(int32_t* count) {
  if (!count) return GC_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  if (drain() != hipSuccess) return GC_EHIP;
  *count = static_cast<int32_t>(g_rec.size());
  return GC_OK;
}

int gc_profile_get(int32_t index, char* name, int32_t name_len, double* total_ms, int64_t* launches) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (drain() != hipSuccess) return GC_EHIP;
  if (index < 0 || index >= static_cast<int32_t>(g_rec.size())) return GC_EINVAL;
  auto it = g_rec.begin();
  std::advance(it, index);
  if (name && name_len > 0) {
    std::strncpy(name, it->first.c_str(), static_cast<size_t>(name_len) - 1);
    name[name_len - 1] = '\0';
  }
  if (total_ms) *total_ms = it->second.total_ms;
  if (launches) *launches = it->second.launches;
  return GC_OK;
}

}  // extern "C"

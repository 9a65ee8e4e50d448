// la_profile.cpp -- opt-in per-kernel timing with HIP events.
#include "la_profile.h"

#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/la.h"

namespace la {
namespace {

struct Rec {
  const char* name;
  hipEvent_t start, stop;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_free;

}  // namespace

bool profiling_on() { return g_on.load(std::memory_order_relaxed); }

hipEvent_t profile_event() {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_free.empty()) {
    hipEvent_t e = g_free.back();
    g_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void profile_record(const char* name, hipEvent_t start, hipEvent_t stop) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_recs.push_back({name, start, stop});
}

}  // namespace la

extern "C" {

la_status la_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(la::g_mu);
  for (auto& r : la::g_recs) {
    la::g_free.push_back(r.start);
    la::g_free.push_back(r.stop);
  }
  la::g_recs.clear();
  la::g_on.store(on != 0);
  return LA_OK;
}

la_status la_profile_read(la_kernel_stat* out, int32_t capacity, int32_t* count) {
  if (!count || capacity < 0 || (capacity > 0 && !out)) return LA_ERR_INVALID_ARG;
  std::vector<la::Rec> recs;
  {
    std::lock_guard<std::mutex> lk(la::g_mu);
    recs = la::g_recs;
  }
  std::map<std::string, std::pair<int64_t, double>> agg;
  std::vector<std::string> order;
  for (const auto& r : recs) {
    if (hipEventSynchronize(r.stop) != hipSuccess) return LA_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return LA_ERR_HIP;
    auto it = agg.find(r.name);
    if (it == agg.end()) {
      order.push_back(r.name);
      agg[r.name] = {1, ms};
    } else {
      it->second.first += 1;
      it->second.second += ms;
    }
  }
  int32_t n = 0;
  for (const auto& name : order) {
    if (n < capacity) {
      std::memset(&out[n], 0, sizeof(la_kernel_stat));
      std::strncpy(out[n].name, name.c_str(), sizeof(out[n].name) - 1);
      out[n].launches = agg[name].first;
      out[n].total_ms = agg[name].second;
    }
    ++n;
  }
  *count = n;
  return LA_OK;
}

}  // extern "C"

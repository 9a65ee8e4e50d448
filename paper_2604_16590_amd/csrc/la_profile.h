// la_profile.h -- opt-in per-kernel timing with HIP events (internal).
//
// When enabled through la_profile_enable(), every kernel launch of the
// library is bracketed by two events recorded on the launch stream, so the
// measured duration is that kernel's own on the stream it runs on.
#pragma once
#include <hip/hip_runtime.h>

namespace la {

bool profiling_on();
void profile_record(const char* name, hipEvent_t start, hipEvent_t stop);
hipEvent_t profile_event();

class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t s) : name_(name), s_(s) {
    if (profiling_on()) {
      start_ = profile_event();
      stop_ = profile_event();
      if (start_ && stop_) (void)hipEventRecord(start_, s_);
    }
  }
  ~ProfScope() {
    if (start_ && stop_) {
      (void)hipEventRecord(stop_, s_);
      profile_record(name_, start_, stop_);
    }
  }
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  const char* name_;
  hipStream_t s_;
  hipEvent_t start_ = nullptr, stop_ = nullptr;
};

}  // namespace la

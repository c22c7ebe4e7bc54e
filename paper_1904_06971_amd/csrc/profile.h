// Phase timer used around kernel launches (active only when profiling is on).
#pragma once

#include <hip/hip_runtime.h>

namespace igs {

bool profiling();

class PhaseTimer {
 public:
  PhaseTimer(const char* name, hipStream_t s);
  ~PhaseTimer();
  void stop();
  PhaseTimer(const PhaseTimer&) = delete;
  PhaseTimer& operator=(const PhaseTimer&) = delete;

 private:
  const char* name_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

}  // namespace igs

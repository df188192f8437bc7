// Scoped kernel-phase timer (see profile.cpp).
#pragma once

#include "common.hpp"

namespace skls {

bool profiling_on();

class PhaseTimer {
 public:
  PhaseTimer(const char* name, hipStream_t s);
  ~PhaseTimer();
  PhaseTimer(const PhaseTimer&) = delete;
  PhaseTimer& operator=(const PhaseTimer&) = delete;

 private:
  const char* name_;
  hipStream_t s_;
  hipEvent_t start_ = nullptr, stop_ = nullptr;
  bool active_ = false;
};

}  // namespace skls

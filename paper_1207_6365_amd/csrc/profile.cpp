// Kernel-phase timing: when enabled, each phase the library launches is
// bracketed by HIP events recorded on the caller's stream, and the elapsed
// times are accumulated per phase name when they are read back.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "profile.hpp"

namespace skls {
namespace {

struct Phase {
  std::string name;
  int64_t launches = 0;
  double total_ms = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Phase> g_phases;

Phase& phase_of(const char* name) {
  for (auto& p : g_phases)
    if (p.name == name) return p;
  g_phases.push_back(Phase{});
  g_phases.back().name = name;
  return g_phases.back();
}

void resolve(Phase& p) {
  for (auto& e : p.pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(e.second) == hipSuccess && hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) {
      p.total_ms += ms;
      ++p.launches;
    }
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  p.pending.clear();
}

void clear_all() {
  for (auto& p : g_phases) {
    for (auto& e : p.pending) {
      (void)hipEventSynchronize(e.second);
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  }
  g_phases.clear();
}

}  // namespace

bool profiling_on() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_on;
}

PhaseTimer::PhaseTimer(const char* name, hipStream_t s) : name_(name), s_(s) {
  if (!profiling_on()) return;
  if (hipEventCreate(&start_) != hipSuccess) return;
  if (hipEventCreate(&stop_) != hipSuccess) {
    (void)hipEventDestroy(start_);
    return;
  }
  if (hipEventRecord(start_, s_) != hipSuccess) {
    (void)hipEventDestroy(start_);
    (void)hipEventDestroy(stop_);
    return;
  }
  active_ = true;
}

PhaseTimer::~PhaseTimer() {
  if (!active_) return;
  if (hipEventRecord(stop_, s_) != hipSuccess) {
    (void)hipEventDestroy(start_);
    (void)hipEventDestroy(stop_);
    return;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  phase_of(name_).pending.emplace_back(start_, stop_);
}

}  // namespace skls

using namespace skls;

extern "C" {

int32_t skls_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_mu);
  clear_all();
  g_on = on != 0;
  return SKLS_OK;
}

int32_t skls_profile_count(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  return static_cast<int32_t>(g_phases.size());
}

int32_t skls_profile_get(int32_t index, const char** name, int64_t* launches, double* total_ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (index < 0 || index >= static_cast<int32_t>(g_phases.size()) || name == nullptr || launches == nullptr ||
      total_ms == nullptr) {
    set_error("profile index out of range or NULL output");
    return SKLS_ERR_ARG;
  }
  Phase& p = g_phases[static_cast<size_t>(index)];
  resolve(p);
  *name = p.name.c_str();
  *launches = p.launches;
  *total_ms = p.total_ms;
  return SKLS_OK;
}

}  // extern "C"

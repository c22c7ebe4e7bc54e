// Opt-in, thread-local phase profiler: HIP events around kernel launches.
#include <cstring>
#include <string>
#include <vector>

#include "igs_internal.h"
#include "profile.h"

namespace igs {

namespace {
struct Rec {
  std::string name;
  hipEvent_t a, b;
};
struct State {
  bool on = false;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
thread_local State g_state;
}  // namespace

bool profiling() { return g_state.on; }

PhaseTimer::PhaseTimer(const char* name, hipStream_t s) : name_(name), s_(s) {
  if (!g_state.on) return;
  a_ = g_state.get();
  b_ = g_state.get();
  if (a_ && b_) (void)hipEventRecord(a_, s_);
}

PhaseTimer::~PhaseTimer() { stop(); }

void PhaseTimer::stop() {
  if (!a_ || !b_) return;
  (void)hipEventRecord(b_, s_);
  g_state.recs.push_back(Rec{name_, a_, b_});
  a_ = b_ = nullptr;
}

}  // namespace igs

extern "C" {

igs_status igs_profile_enable(int32_t on) {
  igs::g_state.on = on != 0;
  return IGS_OK;
}

igs_status igs_profile_read(igs_profile* out) {
  if (!out) return IGS_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  igs_status st = IGS_OK;
  for (auto& r : igs::g_state.recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) st = IGS_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) st = IGS_ERR_HIP;
    int k = 0;
    while (k < out->nphase && std::strncmp(out->phase[k].name, r.name.c_str(), 31) != 0) ++k;
    if (k == out->nphase) {
      if (out->nphase == IGS_PROFILE_MAX_PHASES) continue;
      std::strncpy(out->phase[k].name, r.name.c_str(), 31);
      out->nphase++;
    }
    out->phase[k].launches++;
    out->phase[k].ms += ms;
    igs::g_state.pool.push_back(r.a);
    igs::g_state.pool.push_back(r.b);
  }
  igs::g_state.recs.clear();
  return st;
}

}  // extern "C"

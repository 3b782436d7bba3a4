// Host-side runtime state: the per-thread GEMM arithmetic mode and the launch
// probes (HIP event pairs around individual kernel launches).
#include <mutex>
#include <vector>

#include "common.h"

namespace gep {
namespace {

thread_local MathMode t_mode = MathMode::Fp64;
bool g_force_timeout = false;
bool g_force_eig_failure = false;

struct ProbeRecord {
  hipEvent_t start, stop;
  double flops;
};

std::mutex g_probe_mu;
bool g_probe_on = false;
std::vector<ProbeRecord> g_records[PROBE_COUNT];
std::vector<hipEvent_t> g_free_events;

hipEvent_t take_event() {
  if (!g_free_events.empty()) {
    hipEvent_t e = g_free_events.back();
    g_free_events.pop_back();
    return e;
  }
  hipEvent_t e;
  GEP_HIP(hipEventCreate(&e));
  return e;
}

}  // namespace

MathMode math_mode() { return t_mode; }

void set_force_wait_timeout(bool on) { g_force_timeout = on; }
bool force_wait_timeout() { return g_force_timeout; }
void set_force_eig_failure(bool on) { g_force_eig_failure = on; }
bool force_eig_failure() { return g_force_eig_failure; }

uint64_t wait_limit_ticks() {
  int dev = 0, rate_khz = 0;
  GEP_HIP(hipGetDevice(&dev));
  GEP_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
  if (rate_khz <= 0) rate_khz = 100000;
  return (uint64_t)rate_khz * 1000ull * 10ull;
}

MathScope::MathScope(MathMode m) : saved(t_mode) { t_mode = m; }
MathScope::~MathScope() { t_mode = saved; }

void probe_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_probe_mu);
  g_probe_on = on;
}

ProbeScope::ProbeScope(int id_, hipStream_t s_, double flops_)
    : id(id_), s(s_), flops(flops_), start(nullptr), stop(nullptr) {
  std::lock_guard<std::mutex> lk(g_probe_mu);
  on = g_probe_on && id >= 0 && id < PROBE_COUNT;
  if (!on) return;
  start = take_event();
  stop = take_event();
  GEP_HIP(hipEventRecord(start, s));
}

ProbeScope::~ProbeScope() {
  if (!on) return;
  // The scope owns its event pair, so launches from several host threads stay
  // paired.  A destructor does not throw: a failed record shows up when the
  // events are read.
  (void)hipEventRecord(stop, s);
  std::lock_guard<std::mutex> lk(g_probe_mu);
  g_records[id].push_back(ProbeRecord{start, stop, flops});
}

bool probe_read(int id, int64_t* launches, double* ms, double* flops) {
  if (id < 0 || id >= PROBE_COUNT) return false;
  std::lock_guard<std::mutex> lk(g_probe_mu);
  int64_t n = 0;
  double t = 0.0, f = 0.0;
  for (const ProbeRecord& r : g_records[id]) {
    GEP_HIP(hipEventSynchronize(r.stop));
    float e = 0.0f;
    GEP_HIP(hipEventElapsedTime(&e, r.start, r.stop));
    t += e;
    f += r.flops;
    ++n;
    g_free_events.push_back(r.start);
    g_free_events.push_back(r.stop);
  }
  g_records[id].clear();
  if (launches) *launches = n;
  if (ms) *ms = t;
  if (flops) *flops = f;
  return true;
}

}  // namespace gep

// Optional per-launch timing with HIP events (instrumentation for measurement).
//
// When enabled, every product launch made by the library is bracketed by two
// events recorded on the launch's stream and tagged with its class. Reading
// the totals waits for the recorded events and releases them to a pool.
#include <mutex>
#include <vector>

#include "common.hpp"

namespace sc {

namespace {
struct Rec { int kind; hipEvent_t a, b; };
std::mutex mu;
bool enabled = false;
std::vector<Rec> recs;
std::vector<hipEvent_t> pool;

hipEvent_t take() {
  if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool timing_on() { return enabled; }

TimingMark timing_begin(int kind, hipStream_t stream) {
  TimingMark m{kind, nullptr};
  if (!enabled) return m;
  std::lock_guard<std::mutex> g(mu);
  m.a = take();
  if (m.a && hipEventRecord((hipEvent_t)m.a, stream) != hipSuccess) {   // measurement only: skip it
    pool.push_back((hipEvent_t)m.a);
    m.a = nullptr;
  }
  return m;
}

void timing_end(const TimingMark& m, hipStream_t stream) {
  if (!enabled || !m.a) return;
  std::lock_guard<std::mutex> g(mu);
  hipEvent_t b = take();
  if (!b) {
    pool.push_back((hipEvent_t)m.a);
    return;
  }
  if (hipEventRecord(b, stream) != hipSuccess) {
    pool.push_back((hipEvent_t)m.a);
    pool.push_back(b);
    return;
  }
  recs.push_back(Rec{m.kind, (hipEvent_t)m.a, b});
}

}  // namespace sc

using namespace sc;

extern "C" {

sincosm_status sincosm_timing_enable(int on) {
  std::lock_guard<std::mutex> g(mu);
  for (auto& r : recs) { pool.push_back(r.a); pool.push_back(r.b); }
  recs.clear();
  enabled = on != 0;
  return SINCOSM_OK;
}

sincosm_status sincosm_timing_read(int kind, double* total_ms, int64_t* count) {
  if (!total_ms || !count) return SINCOSM_E_ARG;
  std::lock_guard<std::mutex> g(mu);
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto& r : recs) {
    if (r.kind != kind) continue;
    SC_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    SC_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *count = cnt;
  return SINCOSM_OK;
}

}  // extern "C"

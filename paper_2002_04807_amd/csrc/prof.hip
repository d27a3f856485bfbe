// Per-class kernel timing with HIP events (see prof.hpp).
#include <vector>

#include "prof.hpp"

namespace mf {

namespace {
struct Rec {
  int cls;
  double flops, bytes;
  int a, b;  // event indices
};
// per host thread: calls on different handles may run from different threads
thread_local bool g_on = false;
thread_local std::vector<hipEvent_t> g_events;
thread_local int g_next = 0;
thread_local std::vector<Rec> g_recs;
thread_local bool g_coop = true;

int take_event() {
  if (g_next >= (int)g_events.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    g_events.push_back(e);
  }
  return g_next++;
}
}  // namespace

bool prof_on() { return g_on; }

bool coop_allowed() { return g_coop; }
void set_coop_allowed(bool on) { g_coop = on; }

void prof_enable(bool on) {
  g_on = on;
  g_next = 0;
  g_recs.clear();
}

int prof_begin(hipStream_t s) {
  if (!g_on) return -1;
  const int a = take_event();
  if (a >= 0) (void)hipEventRecord(g_events[a], s);
  return a;
}

void prof_end(int token, hipStream_t s, int cls, double flops, double bytes) {
  if (!g_on || token < 0) return;
  const int b = take_event();
  if (b < 0) return;
  (void)hipEventRecord(g_events[b], s);
  g_recs.push_back({cls, flops, bytes, token, b});
}

void prof_collect(double* out) {
  for (const Rec& r : g_recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_events[r.a], g_events[r.b]) != hipSuccess) continue;
    out[r.cls * 4 + 0] += 1.0;
    out[r.cls * 4 + 1] += ms;
    out[r.cls * 4 + 2] += r.flops;
    out[r.cls * 4 + 3] += r.bytes;
  }
  g_recs.clear();
  g_next = 0;
}

}  // namespace mf

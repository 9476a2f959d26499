// Optional per-kernel timing with HIP events recorded on the launching
// stream (enabled by tg_set_timing or the TG_TIMING environment variable).
// Results appear in tg_last_stats() as "<kernel>_ms" (summed duration),
// "<kernel>_n" (launches) and "<kernel>_busy_ms": the length of the union of
// the launches' intervals, measured from one reference event per call, so
// that launches overlapping on several streams count once.
#include <stdlib.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <string>
#include <vector>

#include "tg_internal.h"

namespace tg {
namespace {

struct Pending {
  const char *name;
  size_t a, b;
};

struct TimerState {
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Pending> pending;
  KTimes t;
  hipEvent_t own_ref = nullptr;  // this thread's reference event
  hipEvent_t ref = nullptr;      // the call's reference (own_ref or a parent thread's)
};

thread_local TimerState g_t;

hipEvent_t take() {
  if (g_t.used == g_t.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_t.pool.push_back(e);
  }
  return g_t.pool[g_t.used++];
}

double union_length(std::vector<std::pair<float, float>> iv) {
  std::sort(iv.begin(), iv.end());
  double len = 0.0;
  float lo = 0.f, hi = -1.f;
  for (const auto &x : iv) {
    if (x.first > hi) {
      if (hi > lo) len += hi - lo;
      lo = x.first;
      hi = x.second;
    } else {
      hi = std::max(hi, x.second);
    }
  }
  if (hi > lo) len += hi - lo;
  return len;
}

std::atomic<int> g_timing{-1};  // -1: not yet read from TG_TIMING

}  // namespace

bool timing_enabled() {
  int v = g_timing.load(std::memory_order_relaxed);
  if (v < 0) {
    const char *e = getenv("TG_TIMING");
    v = (e != nullptr && e[0] != '0') ? 1 : 0;
    int expect = -1;
    g_timing.compare_exchange_strong(expect, v);
    v = g_timing.load(std::memory_order_relaxed);
  }
  return v == 1;
}

void set_timing(bool on) { g_timing.store(on ? 1 : 0, std::memory_order_relaxed); }

hipEvent_t ktimer_ensure_ref(hipStream_t s) {
  if (!timing_enabled()) return nullptr;
  if (!g_t.ref) {
    // the call's reference: recorded before its first timed launch
    if (!g_t.own_ref && hipEventCreate(&g_t.own_ref) != hipSuccess) return nullptr;
    TG_QUIET(hipEventRecord(g_t.own_ref, s));
    g_t.ref = g_t.own_ref;
  }
  return g_t.ref;
}

int ktimer_start(hipStream_t s) {
  if (!timing_enabled()) return -1;
  if (!ktimer_ensure_ref(s)) return -1;
  hipEvent_t e = take();
  if (!e) return -1;
  TG_QUIET(hipEventRecord(e, s));
  return (int)(g_t.used - 1);
}

void ktimer_set_ref(hipEvent_t ref) { g_t.ref = ref; }

void ktimer_stop(int start, hipStream_t s, const char *name) {
  if (start < 0) return;
  hipEvent_t e = take();
  if (!e) return;
  TG_QUIET(hipEventRecord(e, s));
  g_t.pending.push_back({name, (size_t)start, g_t.used - 1});
}

void ktimer_flush() {
  if (!timing_enabled()) return;
  for (const Pending &p : g_t.pending) {
    float ms = 0.f, t0 = 0.f, t1 = 0.f;
    if (hipEventSynchronize(g_t.pool[p.b]) == hipSuccess &&
        hipEventElapsedTime(&ms, g_t.pool[p.a], g_t.pool[p.b]) == hipSuccess) {
      auto &a = g_t.t.acc[p.name];
      a.first += ms;
      a.second += 1;
      if (g_t.ref && hipEventElapsedTime(&t0, g_t.ref, g_t.pool[p.a]) == hipSuccess &&
          hipEventElapsedTime(&t1, g_t.ref, g_t.pool[p.b]) == hipSuccess)
        g_t.t.iv[p.name].push_back({std::max(t0, 0.f), std::max(t1, 0.f)});
    }
  }
  g_t.pending.clear();
  g_t.used = 0;
}

void ktimer_reset() {
  ktimer_flush();
  g_t.t.acc.clear();
  g_t.t.iv.clear();
  g_t.ref = nullptr;
}

KTimes ktimer_export() {
  ktimer_flush();
  KTimes out = std::move(g_t.t);
  g_t.t = KTimes();
  return out;
}

void ktimer_import(const KTimes &k) {
  for (const auto &kv : k.acc) {
    auto &a = g_t.t.acc[kv.first];
    a.first += kv.second.first;
    a.second += kv.second.second;
  }
  for (const auto &kv : k.iv) {
    auto &v = g_t.t.iv[kv.first];
    v.insert(v.end(), kv.second.begin(), kv.second.end());
  }
}

void ktimer_emit() {
  ktimer_flush();
  for (auto &kv : g_t.t.acc) {
    stats_add((kv.first + "_ms").c_str(), kv.second.first);
    stats_add((kv.first + "_n").c_str(), (double)kv.second.second);
    const auto it = g_t.t.iv.find(kv.first);
    if (it != g_t.t.iv.end()) stats_add((kv.first + "_busy_ms").c_str(), union_length(it->second));
  }
  g_t.t.acc.clear();
  g_t.t.iv.clear();
  g_t.ref = nullptr;
}

}  // namespace tg

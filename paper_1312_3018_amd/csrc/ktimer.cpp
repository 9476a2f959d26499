// Optional per-kernel timing with HIP events recorded on the launching
// stream (enabled by the TG_TIMING environment variable).  Results appear in
// tg_last_stats() as "<kernel>_ms" (summed duration) and "<kernel>_n"
// (launches).
#include <stdlib.h>

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
  std::map<std::string, std::pair<double, long long>> acc;
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

}  // namespace

namespace {
std::atomic<int> g_timing{-1};  // -1: not yet read from TG_TIMING
}

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

int ktimer_start(hipStream_t s) {
  if (!timing_enabled()) return -1;
  hipEvent_t e = take();
  if (!e) return -1;
  TG_QUIET(hipEventRecord(e, s));
  return (int)(g_t.used - 1);
}

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
    float ms = 0.f;
    if (hipEventSynchronize(g_t.pool[p.b]) == hipSuccess &&
        hipEventElapsedTime(&ms, g_t.pool[p.a], g_t.pool[p.b]) == hipSuccess) {
      auto &a = g_t.acc[p.name];
      a.first += ms;
      a.second += 1;
    }
  }
  g_t.pending.clear();
  g_t.used = 0;
}

void ktimer_reset() {
  ktimer_flush();
  g_t.acc.clear();
}

std::vector<std::pair<std::string, std::pair<double, long long>>> ktimer_export() {
  ktimer_flush();
  std::vector<std::pair<std::string, std::pair<double, long long>>> out(g_t.acc.begin(), g_t.acc.end());
  g_t.acc.clear();
  return out;
}

void ktimer_import(const std::vector<std::pair<std::string, std::pair<double, long long>>> &acc) {
  for (const auto &kv : acc) {
    auto &a = g_t.acc[kv.first];
    a.first += kv.second.first;
    a.second += kv.second.second;
  }
}

void ktimer_emit() {
  ktimer_flush();
  for (auto &kv : g_t.acc) {
    stats_add((kv.first + "_ms").c_str(), kv.second.first);
    stats_add((kv.first + "_n").c_str(), (double)kv.second.second);
  }
  g_t.acc.clear();
}

}  // namespace tg

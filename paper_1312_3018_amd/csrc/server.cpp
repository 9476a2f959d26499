// Query server with continuous batching.  Graphs stay resident on the
// device; BFS and SSSP queries are queued per (graph, kind) and admitted into
// the 64-slot engine of that graph as slots and memory free up, at superstep
// boundaries, so queries that arrive while others run join the next
// superstep instead of waiting for the batch to drain.  One worker thread
// enqueues one superstep on every engine that has work (each engine has its
// own stream, so different graphs' supersteps overlap on the device), then
// completes them, retires finished slots (results are in the caller's buffer)
// and admits waiting queries.
//
// SSSP on a large graph with hubs is served by solo searches instead: the
// slot engine relaxes every active (vertex, query) pair each superstep,
// which costs more than the delta-stepping schedule of a single search once
// the graph is large and its degrees are skewed (the step schedule settles
// a hub's neighbourhood once instead of at every superstep); on a large
// graph without hubs the slot engine stays ahead.  Such a lane has its own host threads (up to the partition's
// sssp_lanes, at most max_slots), each running one query at a time with the
// single-search schedule on its own workspace and stream.
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <system_error>
#include <thread>
#include <unordered_map>
#include <vector>

#include "slots.h"

using namespace tg;

namespace {

using clk = std::chrono::steady_clock;

struct Query {
  uint64_t ticket;
  int32_t graph, kind, root;
  int32_t *out;
  clk::time_point arrival, done_at;
  bool done = false;
  int status = TG_OK;
  std::string err;
  int64_t bytes = 0;
  bool held = false;  // admitted: its bytes count in mem_used
};

struct Lane {  // one (graph, kind) engine
  tg_partition *p = nullptr;
  int kind = 0;
  hipStream_t stream = nullptr;
  std::unique_ptr<SlotEngine> eng;
  std::deque<Query *> waiting;
  Query *slot_q[kSlots] = {};
  bool launched = false;
  int64_t engine_bytes = 0;
  // solo SSSP lane: its queries run as single searches on these threads
  bool solo = false;
  std::vector<std::thread> solo_workers;
};

bool json_num(const char *json, const char *key, double *out) {
  if (!json) return false;
  std::string k = std::string("\"") + key + "\"";
  const char *p = strstr(json, k.c_str());
  if (!p) return false;
  p += k.size();
  while (*p == ' ' || *p == ':' || *p == '\t' || *p == '\n') ++p;
  char *end = nullptr;
  const double v = strtod(p, &end);
  if (end == p) return false;
  *out = v;
  return true;
}

}  // namespace

struct tg_server {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<std::unique_ptr<Lane>> lanes;  // index = graph * 2 + kind
  std::vector<tg_partition *> graphs;
  std::unordered_map<uint64_t, std::unique_ptr<Query>> queries;
  uint64_t next_ticket = 1;
  int max_slots = kSlots;
  // SSSP lanes of graphs at least this large, whose largest out-degree is at
  // least solo_min_skew times the mean, run solo searches
  int64_t solo_min_n = int64_t(1) << 22;
  double solo_min_skew = 16.0;
  int64_t mem_cap = INT64_MAX;
  int64_t mem_used = 0;
  int64_t held = 0;  // queries admitted and not yet finished
  int device = 0;
  bool stop = false;
  std::thread worker;
  // statistics (supersteps: completion passes of the worker)
  int64_t completed = 0, supersteps = 0, max_concurrent = 0;

  void run();
  void solo_worker(Lane *L);
};

namespace {

// Device bytes a query holds while it runs (the per-query share of the
// space formula of section 4.3.3: per-vertex state for one source).
int64_t query_bytes(const tg_partition *p, int kind) {
  const int64_t n = p->gpu.n;
  return kind == kSlotBfs ? (3 * n + 7) / 8 : 4 * n + (2 * n + 7) / 8;
}

void finish(tg_server *S, Query *q, int status, const std::string &err) {
  q->status = status;
  q->err = err;
  q->done_at = clk::now();
  q->done = true;
  if (q->held) {  // queries that fail before admission never held memory
    S->mem_used -= q->bytes;
    --S->held;
  }
  ++S->completed;
}

void admit(tg_server *S, Query *q) {
  S->mem_used += q->bytes;
  q->held = true;
  if (++S->held > S->max_concurrent) S->max_concurrent = S->held;
}

}  // namespace

// One thread of a solo SSSP lane: take the next waiting query that fits the
// memory cap, run it as a single search, write its distances, repeat.
void tg_server::solo_worker(Lane *L) {
  TG_QUIET(hipSetDevice(device));
  tg_partition *p = L->p;
  Workspace ws;
  hipStream_t st = nullptr;
  int setup = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess
                  ? TG_OK
                  : set_error(TG_EDEVICE, "server: hipStreamCreateWithFlags failed");
  if (setup == TG_OK) setup = ws.ensure(p->gpu, 0);
  const std::string setup_err = setup == TG_OK ? "" : tg_last_error();
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_work.wait(lk, [&] {
      return stop || (!L->waiting.empty() && (setup != TG_OK || mem_used + L->waiting.front()->bytes <= mem_cap));
    });
    if (stop) break;
    Query *q = L->waiting.front();
    L->waiting.pop_front();
    if (setup != TG_OK) {
      finish(this, q, setup, setup_err);
      cv_done.notify_all();
      continue;
    }
    admit(this, q);
    const int32_t root = p->h_l_of_g[q->root];
    lk.unlock();
    int64_t rounds = 0, pulls = 0;
    int rc = gpu_sssp(p, ws, root, st, &rounds, &pulls);
    if (rc == TG_OK) rc = collect_i32(p->gpu, ws.state, q->out, st);
    if (rc == TG_OK && hipStreamSynchronize(st) != hipSuccess)
      rc = set_error(TG_EDEVICE, "server: hipStreamSynchronize failed");
    const std::string err = rc == TG_OK ? "" : tg_last_error();
    ktimer_flush();
    lk.lock();
    finish(this, q, rc, err);
    cv_done.notify_all();
    cv_work.notify_all();  // memory freed: other lanes may admit
  }
  lk.unlock();
  if (st) {
    TG_QUIET(hipStreamSynchronize(st));
    TG_QUIET(hipStreamDestroy(st));
  }
}

void tg_server::run() {
  TG_QUIET(hipSetDevice(device));
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // 1. every idle lane: admit waiting queries into free slots (within the
    //    memory cap), then start its next superstep if it has running slots
    bool in_flight = false;
    for (auto &lp : lanes) {
      Lane &L = *lp;
      if (!L.p || L.solo) continue;
      if (L.launched) {
        in_flight = true;
        continue;
      }
      while (!L.waiting.empty()) {
        Query *q = L.waiting.front();
        if (!L.eng) {
          L.eng.reset(new SlotEngine());
          int rc = L.eng->init(L.p, L.kind, L.stream);
          if (rc != TG_OK) {
            std::string e = tg_last_error();
            for (Query *w : L.waiting) finish(this, w, rc, e);
            L.waiting.clear();
            L.eng.reset();
            cv_done.notify_all();
            break;
          }
        }
        int used = 0;
        for (int k = 0; k < kSlots; ++k) used += L.slot_q[k] != nullptr;
        const int slot = L.eng->free_slot();
        if (slot < 0 || used >= max_slots || mem_used + q->bytes > mem_cap) break;
        L.waiting.pop_front();
        admit(this, q);
        L.slot_q[slot] = q;
        int rc = L.eng->join(slot, L.p->h_l_of_g[q->root], L.kind == kSlotBfs ? q->out : nullptr);
        if (rc != TG_OK) {
          L.slot_q[slot] = nullptr;
          L.eng->busy &= ~(1ull << slot);
          finish(this, q, rc, tg_last_error());
          cv_done.notify_all();
        }
      }
      if (L.eng && L.eng->busy) {
        if (L.eng->launch_step() == TG_OK) {
          L.launched = true;
          in_flight = true;
        }
      }
    }
    if (!in_flight) {
      if (stop) break;
      cv_work.wait(lk);
      continue;
    }
    // 2. complete whichever lanes' supersteps are done; lanes advance
    //    independently, so a slow graph does not hold back the others.
    //    server_add_graph may grow `lanes` meanwhile: walk a copy of the
    //    lane pointers taken under the lock (each Lane stays where it is).
    std::vector<Lane *> snap;
    snap.reserve(lanes.size());
    for (auto &lp : lanes) snap.push_back(lp.get());
    lk.unlock();
    std::vector<std::pair<Lane *, unsigned long long>> fin;
    bool progressed = false;
    for (Lane *lp : snap) {
      Lane &L = *lp;
      if (!L.launched || hipStreamQuery(L.stream) != hipSuccess) continue;
      (void)hipGetLastError();  // hipStreamQuery reports "not ready" through the error state
      L.launched = false;
      progressed = true;
      unsigned long long f = 0;
      if (L.eng->finish_step(&f) == TG_OK && f) {
        if (L.kind == kSlotSssp)
          for (int k = 0; k < kSlots; ++k)
            if ((f >> k) & 1ull) L.eng->tab.out[k] = L.slot_q[k]->out;
        unsigned long long ovf = 0;
        const int rc = L.eng->retire(f, &ovf);
        fin.emplace_back(&L, f);
        for (int k = 0; k < kSlots; ++k)
          if ((f >> k) & 1ull) {
            if (rc != TG_OK) L.slot_q[k]->status = rc;
            else if ((ovf >> k) & 1ull) L.slot_q[k]->status = TG_ERANGE;
          }
      }
    }
    (void)hipGetLastError();
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    lk.lock();
    if (progressed) ++supersteps;
    for (auto &pr : fin) {
      Lane &L = *pr.first;
      for (int k = 0; k < kSlots; ++k)
        if ((pr.second >> k) & 1ull) {
          Query *q = L.slot_q[k];
          L.slot_q[k] = nullptr;
          const int st = q->status;
          finish(this, q, st,
                 st == TG_ERANGE ? "sssp: a shortest-path distance does not fit below INT32_MAX" : "");
        }
    }
    if (!fin.empty()) cv_done.notify_all();
  }
}

extern "C" int server_create(const char *opts_json, tg_server **out) {
  clear_error();
  if (!out) return set_error(TG_EINVAL, "server_create: out is NULL");
  auto *S = new (std::nothrow) tg_server();
  if (!S) return set_error(TG_ENOMEM, "server_create: out of host memory");
  double v;
  if (json_num(opts_json, "max_slots", &v)) S->max_slots = (int)v;
  if (json_num(opts_json, "memory_cap_bytes", &v)) S->mem_cap = (int64_t)v;
  if (json_num(opts_json, "sssp_solo_min_vertices", &v)) S->solo_min_n = (int64_t)v;
  if (json_num(opts_json, "sssp_solo_min_skew", &v)) S->solo_min_skew = v;
  if (S->max_slots < 1 || S->max_slots > kSlots) {
    delete S;
    return set_error(TG_EINVAL, "server_create: max_slots must be in [1, 64]");
  }
  if (S->mem_cap < 0) {
    delete S;
    return set_error(TG_EINVAL, "server_create: memory_cap_bytes < 0");
  }
  if (S->solo_min_n < 0) {
    delete S;
    return set_error(TG_EINVAL, "server_create: sssp_solo_min_vertices < 0");
  }
  if (!(S->solo_min_skew >= 0.0)) {
    delete S;
    return set_error(TG_EINVAL, "server_create: sssp_solo_min_skew must be >= 0");
  }
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return set_error(TG_EDEVICE, "server_create: no HIP device");
  }
  S->worker = std::thread([S] { S->run(); });
  *out = S;
  return TG_OK;
}

extern "C" int server_add_graph(tg_server *S, const tg_partition *p, int32_t *graph_id) {
  clear_error();
  if (!S || !p || !graph_id) return set_error(TG_EINVAL, "server_add_graph: NULL argument");
  if (p->alpha > 0.0) return set_error(TG_EUNSUPPORTED, "server_add_graph: hybrid partitions are not served");
  std::lock_guard<std::mutex> lk(S->mu);
  tg_partition *pm = const_cast<tg_partition *>(p);
  // degree skew: largest local out-degree (local ids run by decreasing
  // out-degree) over the mean
  const double mean_deg = p->gpu.n > 0 ? (double)p->gpu.out.m / (double)p->gpu.n : 0.0;
  const double skew = mean_deg > 0.0 && !p->gpu.h_deg.empty() ? (double)p->gpu.h_deg[0] / mean_deg : 0.0;
  const bool solo = p->g->has_w && p->gpu.n >= S->solo_min_n && skew >= S->solo_min_skew;
  if (solo) {
    // the layouts the single-search schedule reads, built before its
    // threads share the partition
    hipStream_t st = nullptr;
    TG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    int rc = sssp_prepare(pm, st);
    if (hipStreamSynchronize(st) != hipSuccess && rc == TG_OK)
      rc = set_error(TG_EDEVICE, "server_add_graph: hipStreamSynchronize failed");
    TG_QUIET(hipStreamDestroy(st));
    if (rc != TG_OK) return rc;
  }
  // the graph is registered only once both lanes exist: a lane is found
  // at index 2 * id + kind
  std::unique_ptr<Lane> made[2];
  for (int kind = 0; kind < 2; ++kind) {
    made[kind].reset(new Lane());
    made[kind]->p = pm;
    made[kind]->kind = kind;
    made[kind]->solo = solo && kind == kSlotSssp;
    const hipError_t e = hipStreamCreateWithFlags(&made[kind]->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (auto &L : made)
        if (L && L->stream) TG_QUIET(hipStreamDestroy(L->stream));
      return set_error(TG_EDEVICE, "server_add_graph: hipStreamCreateWithFlags failed: %s", hipGetErrorString(e));
    }
  }
  const int32_t id = (int32_t)S->graphs.size();
  S->graphs.push_back(pm);
  for (auto &L : made) S->lanes.push_back(std::move(L));
  Lane *SL = S->lanes.back().get();
  if (SL->solo) {
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(p->tune.sssp_lanes, S->max_slots));
    try {
      for (int i = 0; i < nt; ++i) SL->solo_workers.emplace_back([S, SL] { S->solo_worker(SL); });
    } catch (const std::system_error &) {
      // fewer threads than asked for serve the lane; with none, its slot
      // engine does
    }
    if (SL->solo_workers.empty()) SL->solo = false;
  }
  *graph_id = id;
  return TG_OK;
}

extern "C" int server_submit(tg_server *S, int32_t graph_id, int32_t kind, int32_t root, int32_t *out,
                             uint64_t *ticket) {
  clear_error();
  if (!S || !out || !ticket) return set_error(TG_EINVAL, "server_submit: NULL argument");
  if (kind != TG_QUERY_BFS && kind != TG_QUERY_SSSP) return set_error(TG_EINVAL, "server_submit: unknown kind %d", kind);
  std::lock_guard<std::mutex> lk(S->mu);
  if (graph_id < 0 || graph_id >= (int32_t)S->graphs.size())
    return set_error(TG_EINVAL, "server_submit: unknown graph %d", graph_id);
  tg_partition *p = S->graphs[graph_id];
  if (root < 0 || root >= p->g->n) return set_error(TG_EINVAL, "server_submit: root %d out of range", root);
  if (kind == TG_QUERY_SSSP && !p->g->has_w)
    return set_error(TG_EUNSUPPORTED, "server_submit: graph %d has no weights", graph_id);
  const int k = kind == TG_QUERY_BFS ? kSlotBfs : kSlotSssp;
  const int64_t bytes = query_bytes(p, k);
  if (bytes > S->mem_cap)
    return set_error(TG_ENOMEM, "server_submit: a query needs %lld bytes, above the cap", (long long)bytes);
  std::unique_ptr<Query> q(new Query());
  q->ticket = S->next_ticket++;
  q->graph = graph_id;
  q->kind = k;
  q->root = root;
  q->out = out;
  q->arrival = clk::now();
  q->bytes = bytes;
  S->lanes[(size_t)graph_id * 2 + k]->waiting.push_back(q.get());
  *ticket = q->ticket;
  S->queries.emplace(q->ticket, std::move(q));
  S->cv_work.notify_all();
  return TG_OK;
}

extern "C" int server_wait(tg_server *S, uint64_t ticket, int64_t timeout_us, double *latency_us) {
  clear_error();
  if (!S) return set_error(TG_EINVAL, "server_wait: server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->queries.find(ticket);
  if (it == S->queries.end()) return set_error(TG_EINVAL, "server_wait: unknown ticket %llu", (unsigned long long)ticket);
  Query *q = it->second.get();
  auto ready = [q] { return q->done; };
  if (timeout_us < 0) {
    S->cv_done.wait(lk, ready);
  } else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return set_error(TG_ETIMEOUT, "server_wait: ticket %llu not done within %lld us", (unsigned long long)ticket,
                     (long long)timeout_us);
  }
  if (latency_us) *latency_us = std::chrono::duration<double, std::micro>(q->done_at - q->arrival).count();
  const int st = q->status;
  const std::string err = q->err;
  S->queries.erase(it);
  if (st != TG_OK) return set_error(st, "%s", err.c_str());
  return TG_OK;
}

extern "C" int server_stats(tg_server *S, char *json, size_t cap) {
  clear_error();
  if (!S) return set_error(TG_EINVAL, "server_stats: server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  int64_t waiting = 0;
  for (auto &lp : S->lanes) waiting += (int64_t)lp->waiting.size();
  char buf[512];
  const int n = snprintf(buf, sizeof(buf),
                         "{\"completed\":%lld,\"supersteps\":%lld,\"max_concurrent\":%lld,\"waiting\":%lld,"
                         "\"memory_in_use\":%lld,\"max_slots\":%d}",
                         (long long)S->completed, (long long)S->supersteps, (long long)S->max_concurrent,
                         (long long)waiting, (long long)S->mem_used, S->max_slots);
  if (json && cap) {
    const size_t k = std::min(cap - 1, (size_t)n);
    memcpy(json, buf, k);
    json[k] = 0;
  }
  return n;
}

extern "C" void server_destroy(tg_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    // queries still waiting are abandoned; running ones finish first
    for (auto &lp : S->lanes) lp->waiting.clear();
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (auto &lp : S->lanes)
    for (auto &t : lp->solo_workers)
      if (t.joinable()) t.join();
  for (auto &lp : S->lanes) {
    lp->eng.reset();
    if (lp->stream) TG_QUIET(hipStreamDestroy(lp->stream));
  }
  delete S;
}

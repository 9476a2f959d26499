// C ABI entry points, graph loading and validation, partition by degree
// centrality (section 6.2), device memory and error reporting.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <omp.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <string>
#include <thread>
#include <vector>

#include "hybrid.h"
#include "slots.h"
#include "tg_internal.h"

using namespace tg;

// ---------------------------------------------------------------- errors
namespace {
thread_local std::string g_err;
thread_local std::string g_stats;
}  // namespace

namespace tg {

int set_error(int code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

// Also drop any HIP error left pending by an earlier unchecked runtime call
// (so that a launch check reports only its own launch); with TG_DEBUG set,
// name it on stderr.
void debug_hip(hipError_t e, const char *what) {
  static const bool dbg = getenv("TG_DEBUG") != nullptr;
  if (e != hipSuccess) {
    if (dbg) fprintf(stderr, "[tg] %s: %s\n", what, hipGetErrorName(e));
    (void)hipGetLastError();
  }
}

void clear_error() {
  g_err.clear();
  const hipError_t stale = hipGetLastError();
  static const bool dbg = getenv("TG_DEBUG") != nullptr;
  if (stale != hipSuccess && dbg) fprintf(stderr, "[tg] pending HIP error at API entry: %s\n", hipGetErrorName(stale));
}

void stats_reset(const char *algo) {
  g_stats = std::string("{\"algorithm\":\"") + algo + "\"";
}

void stats_add(const char *key, double value) {
  char buf[128];
  snprintf(buf, sizeof(buf), ",\"%s\":%.17g", key, value);
  g_stats += buf;
}

// --------------------------------------------------------- device memory
int DevArena::alloc(void **p, size_t n) {
  if (n == 0) n = 256;
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return set_error(TG_ENOMEM, "hipMalloc(%zu bytes) failed: %s", n, hipGetErrorString(e));
  }
  ptrs.push_back(q);
  bytes += n;
  *p = q;
  return TG_OK;
}

int HostMappedArena::upload(void **dev, const void *src, size_t n) {
  void *h = nullptr;
  const size_t sz = n ? n : 256;
  if (hipHostMalloc(&h, sz, hipHostMallocMapped) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(TG_ENOMEM, "hipHostMalloc(%zu bytes, mapped) failed", sz);
  }
  ptrs.push_back(h);
  bytes += sz;
  if (n) memcpy(h, src, n);
  TG_HIP(hipHostGetDevicePointer(dev, h, 0));
  return TG_OK;
}

HostMappedArena::~HostMappedArena() {
  for (void *h : ptrs) TG_QUIET(hipHostFree(h));
}

void DevArena::release_one(void *p) {
  for (size_t i = 0; i < ptrs.size(); ++i)
    if (ptrs[i] == p) {
      TG_QUIET(hipFree(p));
      ptrs.erase(ptrs.begin() + (long)i);
      return;
    }
}

void DevArena::release() {
  for (void *q : ptrs) TG_QUIET(hipFree(q));
  ptrs.clear();
  bytes = 0;
}

void Workspace::drop_graphs() {
  for (GraphChunk &c : graphs) TG_QUIET(hipGraphExecDestroy(c.exec));
  graphs.clear();
}

Workspace::~Workspace() {
  drop_graphs();
  if (h_plan) TG_QUIET(hipHostFree(h_plan));
  if (h_flags) TG_QUIET(hipHostFree(h_flags));
  if (h_work) TG_QUIET(hipHostFree(h_work));
  if (h_stat) TG_QUIET(hipHostFree(h_stat));
  if (h_ctl) TG_QUIET(hipHostFree(h_ctl));
}

int Workspace::ensure(const GpuPart &g, int64_t hub_chunks_needed) {
  const int64_t hubs_needed = g.max_out_hubs + 1;
  if (cap_n == g.n && hub_chunks_needed <= hub_chunks_cap && hubs_needed <= hubs_cap) return TG_OK;
  drop_graphs();
  ++gen;
  arena.release();
  fd = nullptr;
  pull_part = nullptr;
  buckets = nullptr;
  buckets_k = 0;
  pull_part_cap = 0;
  const int64_t n = g.n;
  nwords = ((n + 31) / 32 + 1023) / 1024 * 1024;
  if (nwords == 0) nwords = 1024;
  TG_TRY(dalloc(arena, &bits_a, nwords));
  TG_TRY(dalloc(arena, &bits_b, nwords));
  TG_TRY(dalloc(arena, &bits_c, nwords));
  TG_TRY(dalloc(arena, &queue, n + 1));
  TG_TRY(dalloc(arena, &state, n + 1));
  TG_TRY(dalloc(arena, &settled, n + 1));
  TG_TRY(dalloc(arena, &cbuf[0], n + 1));
  TG_TRY(dalloc(arena, &cbuf[1], n + 1));
  TG_TRY(dalloc(arena, &sigma, n + 1));
  TG_TRY(dalloc(arena, &delta, n + 1));
  TG_TRY(dalloc(arena, &bc_acc, n + 1));
  partials_cap = 16384;
  TG_TRY(dalloc(arena, &partials, partials_cap));
  // frontier hub chunks are bounded by E / chunk + (hub vertices)
  // (hub_chunk >= 256, so a frontier has at most E/256 + hubs chunks)
  int64_t chunks = std::max<int64_t>(hub_chunks_needed, g.m / 256 + g.max_out_hubs + 1);
  hub_chunks_cap = chunks;
  TG_TRY(dalloc(arena, &hub_partials, chunks));
  const int64_t hubs = hubs_needed;
  hubs_cap = hubs;
  TG_TRY(dalloc(arena, &hubpref, hubs + 1));
  TG_TRY(dalloc(arena, &scalars, 16));
  TG_TRY(dalloc(arena, &counters, 64));
  TG_TRY(dalloc(arena, &work, (size_t)tgk::STAT_COUNTERS * tgk::STAT_SPAN));
  TG_TRY(dalloc(arena, &bcount, nwords / 1024 + 1));
  TG_TRY(dalloc(arena, &plan, 1));
  TG_TRY(dalloc(arena, &ctl, 1));
  TG_HIP(hipMemset(bits_a, 0, nwords * sizeof(uint32_t)));
  TG_HIP(hipMemset(bits_b, 0, nwords * sizeof(uint32_t)));
  TG_HIP(hipMemset(bits_c, 0, nwords * sizeof(uint32_t)));
  TG_HIP(hipMemset(counters, 0, 64 * sizeof(uint32_t)));
  TG_HIP(hipMemset(work, 0, (size_t)tgk::STAT_COUNTERS * tgk::STAT_SPAN * sizeof(unsigned long long)));
  // the clears above run on the null stream, which is not ordered before
  // work on the lanes' non-blocking streams: let them finish first
  TG_HIP(hipDeviceSynchronize());
  if (!h_plan) TG_HIP(hipHostMalloc((void **)&h_plan, sizeof(Plan), hipHostMallocDefault));
  if (!h_flags) TG_HIP(hipHostMalloc((void **)&h_flags, 64 * sizeof(uint32_t), hipHostMallocDefault));
  if (!h_ctl) TG_HIP(hipHostMalloc((void **)&h_ctl, sizeof(tgk::BfsCtl), hipHostMallocDefault));
  if (!h_work) TG_HIP(hipHostMalloc((void **)&h_work, 8 * sizeof(unsigned long long), hipHostMallocDefault));
  if (!h_stat)
    TG_HIP(hipHostMalloc((void **)&h_stat, (size_t)tgk::STAT_COUNTERS * tgk::STAT_SPAN * sizeof(unsigned long long),
                         hipHostMallocDefault));
  cap_n = n;
  return TG_OK;
}

namespace {
// The pieces of a device-resident BFS workspace, each 256-byte aligned.
struct BfsPieces {
  size_t bits, queue, state, bcount, plan, hubpref, work, ctl;
  size_t total() const { return 3 * bits + queue + state + bcount + plan + hubpref + work + ctl; }
};
size_t al256(size_t n) { return (n + 255) & ~(size_t)255; }
BfsPieces bfs_pieces(const GpuPart &g, int64_t nwords) {
  BfsPieces b;
  b.bits = al256((size_t)nwords * sizeof(uint32_t));
  b.queue = al256((size_t)(g.n + 1) * sizeof(int32_t));
  b.state = al256((size_t)(g.n + 1) * sizeof(int32_t));
  b.bcount = al256((size_t)(nwords / 1024 + 1) * sizeof(uint32_t));
  b.plan = al256(sizeof(Plan));
  b.hubpref = al256((size_t)(g.max_out_hubs + 2) * sizeof(int64_t));
  b.work = al256((size_t)tgk::STAT_COUNTERS * tgk::STAT_SPAN * sizeof(unsigned long long));
  b.ctl = al256(sizeof(tgk::BfsCtl));
  return b;
}
int64_t bitmap_words(int64_t n) {
  const int64_t w = ((n + 31) / 32 + 1023) / 1024 * 1024;
  return w == 0 ? 1024 : w;
}
}  // namespace

size_t bfs_scratch_bytes(const GpuPart &g) { return bfs_pieces(g, bitmap_words(g.n)).total(); }

int Workspace::bind_bfs(const GpuPart &g, void *base, size_t bytes) {
  const int64_t nw = bitmap_words(g.n);
  const BfsPieces b = bfs_pieces(g, nw);
  if (b.total() > bytes)
    return set_error(TG_ENOMEM, "the partition's BFS needs %zu bytes of scratch; %zu are available", b.total(),
                     bytes);
  uint8_t *p = static_cast<uint8_t *>(base);
  auto take = [&p](size_t n) {
    void *r = p;
    p += n;
    return r;
  };
  nwords = nw;
  bits_a = static_cast<uint32_t *>(take(b.bits));
  bits_b = static_cast<uint32_t *>(take(b.bits));
  bits_c = static_cast<uint32_t *>(take(b.bits));
  queue = static_cast<int32_t *>(take(b.queue));
  state = static_cast<int32_t *>(take(b.state));
  bcount = static_cast<uint32_t *>(take(b.bcount));
  plan = static_cast<Plan *>(take(b.plan));
  hubpref = static_cast<int64_t *>(take(b.hubpref));
  work = static_cast<unsigned long long *>(take(b.work));
  ctl = static_cast<tgk::BfsCtl *>(take(b.ctl));
  hubs_cap = g.max_out_hubs + 1;
  cap_n = -1;  // never taken for an allocated workspace by ensure()
  return TG_OK;
}

int lane_workspace(tg_partition *p, int i, Workspace **out) {
  if (i == 0) {
    *out = &p->ws;
    return TG_OK;
  }
  if (i < 0 || i >= MAX_LANES) return set_error(TG_EINVAL, "lane %d outside [0, %d)", i, MAX_LANES);
  if (!p->lane_ws[i - 1]) {
    p->lane_ws[i - 1].reset(new (std::nothrow) Workspace());
    if (!p->lane_ws[i - 1]) return set_error(TG_ENOMEM, "out of host memory");
  }
  *out = p->lane_ws[i - 1].get();
  return TG_OK;
}

int graph_stream(tg_partition *p, int i, hipStream_t *out) {
  if (i < 0 || i >= MAX_LANES) return set_error(TG_EINVAL, "lane %d outside [0, %d)", i, MAX_LANES);
  if (!p->graph_stream[i]) TG_HIP(hipStreamCreateWithFlags(&p->graph_stream[i], hipStreamNonBlocking));
  *out = p->graph_stream[i];
  return TG_OK;
}

int lane_stream(tg_partition *p, int i, hipStream_t s, hipStream_t *out) {
  if (i == 0) {
    *out = s;
    return TG_OK;
  }
  if (i < 0 || i >= MAX_LANES) return set_error(TG_EINVAL, "lane %d outside [0, %d)", i, MAX_LANES);
  if (!p->lane_stream[i - 1]) TG_HIP(hipStreamCreateWithFlags(&p->lane_stream[i - 1], hipStreamNonBlocking));
  *out = p->lane_stream[i - 1];
  return TG_OK;
}

int stat_zero(Workspace &ws, int k, hipStream_t s) {
  TG_HIP(hipMemsetAsync(tgk::stat_counter(ws.work, k), 0, tgk::STAT_SPAN * sizeof(unsigned long long), s));
  return TG_OK;
}

int stat_zero_all(Workspace &ws, hipStream_t s) {
  TG_HIP(hipMemsetAsync(ws.work, 0, (size_t)tgk::STAT_COUNTERS * tgk::STAT_SPAN * sizeof(unsigned long long), s));
  return TG_OK;
}

int stat_fetch(Workspace &ws, int k, hipStream_t s) {
  TG_HIP(hipMemcpyAsync(tgk::stat_counter(ws.h_stat, k), tgk::stat_counter(ws.work, k), tgk::STAT_SPAN * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, s));
  return TG_OK;
}

unsigned long long stat_sum(const Workspace &ws, int k) {
  const unsigned long long *c = tgk::stat_counter(ws.h_stat, k);
  unsigned long long t = 0;
  for (int i = 0; i < tgk::STAT_SLOTS; ++i) t += c[(size_t)i * tgk::STAT_STRIDE];
  return t;
}

// ----------------------------------------------------------------- tuning
Tuning default_tuning() {
  Tuning t;
  t.min_deg[tgk::BIN_HUB] = 8192;
  t.min_deg[tgk::BIN_BLOCK] = 512;
  t.min_deg[tgk::BIN_WAVE] = 48;
  t.min_deg[tgk::BIN_G16] = 12;
  t.min_deg[tgk::BIN_G4] = 3;
  t.hub_chunk = 4096;
  t.pr_lds_verts = 40960;  // as many as fit next to the row blocks
  t.pr_grid = 256;         // one workgroup per CU
  t.bfs_lds_words = 4096;
  t.bfs_grid = 2048;
  t.bfs_lds_min_vblocks = 4096;
  t.sssp_delta = 32;
  t.sssp_lds_verts = 0;
  t.sssp_grid = 2048;
  t.pr_xcd = 1;
  t.pr_rows = 512;
  t.bfs_do = 1;
  t.bfs_alpha = 14;
  t.bfs_beta = 24;
  t.sssp_xcd = 0;  // measured slower than the plain relax (8 x the per-vertex work)
  t.bfs_lanes = 2;
  t.bfs_td_grid = 1024;
  t.bfs_bu_grid = 4096;
  t.sssp_pull = 0;  // measured slower on R-MAT (pull steps lose the chaining of push steps)
  t.sssp_lanes = 4;
  t.sssp_packed = 1;
  t.sssp_ring = 1;
  t.sssp_split = 1;
  t.sssp_hpull = 100;
  t.bfs_graph = 0;  // replaying captured chunks measured 1-2% slower than direct launches
  t.mapped_edges = 0;
  return t;
}

static bool json_int(const char *json, const char *key, int64_t *out) {
  std::string k = std::string("\"") + key + "\"";
  const char *p = strstr(json, k.c_str());
  if (!p) return false;
  p += k.size();
  while (*p == ' ' || *p == '\t' || *p == '\n' || *p == ':') ++p;
  char *end = nullptr;
  long long v = strtoll(p, &end, 10);
  if (end == p) return false;
  *out = v;
  return true;
}

int parse_tuning(const char *json, Tuning *t) {
  *t = default_tuning();
  if (!json) return TG_OK;
  const char *keys[5] = {"hub_min_deg", "block_min_deg", "wave_min_deg", "g16_min_deg", "g4_min_deg"};
  for (int b = 0; b < 5; ++b) {
    int64_t v;
    if (json_int(json, keys[b], &v)) t->min_deg[b] = v;
  }
  int64_t v;
  if (json_int(json, "hub_chunk", &v)) t->hub_chunk = v;
  if (json_int(json, "pr_lds_verts", &v)) t->pr_lds_verts = v;
  if (json_int(json, "pr_grid", &v)) t->pr_grid = v;
  if (json_int(json, "bfs_lds_words", &v)) t->bfs_lds_words = v;
  if (json_int(json, "bfs_grid", &v)) t->bfs_grid = v;
  if (json_int(json, "bfs_lds_min_vblocks", &v)) t->bfs_lds_min_vblocks = v;
  if (json_int(json, "sssp_delta", &v)) t->sssp_delta = v;
  if (json_int(json, "sssp_lds_verts", &v)) t->sssp_lds_verts = v;
  if (json_int(json, "sssp_grid", &v)) t->sssp_grid = v;
  if (json_int(json, "pr_xcd", &v)) t->pr_xcd = v;
  if (json_int(json, "pr_rows", &v)) t->pr_rows = v;
  if (json_int(json, "bfs_do", &v)) t->bfs_do = v;
  if (json_int(json, "bfs_alpha", &v)) t->bfs_alpha = v;
  if (json_int(json, "bfs_beta", &v)) t->bfs_beta = v;
  if (json_int(json, "sssp_xcd", &v)) t->sssp_xcd = v;
  if (json_int(json, "bfs_lanes", &v)) t->bfs_lanes = v;
  if (json_int(json, "bfs_td_grid", &v)) t->bfs_td_grid = v;
  if (json_int(json, "bfs_bu_grid", &v)) t->bfs_bu_grid = v;
  if (json_int(json, "sssp_pull", &v)) t->sssp_pull = v;
  if (json_int(json, "sssp_lanes", &v)) t->sssp_lanes = v;
  if (json_int(json, "sssp_packed", &v)) t->sssp_packed = v;
  if (json_int(json, "sssp_ring", &v)) t->sssp_ring = v;
  if (json_int(json, "sssp_split", &v)) t->sssp_split = v;
  if (json_int(json, "sssp_hpull", &v)) t->sssp_hpull = v;
  if (json_int(json, "bfs_graph", &v)) t->bfs_graph = v;
  if (json_int(json, "mapped_edges", &v)) t->mapped_edges = v;
  if (t->mapped_edges != 0 && t->mapped_edges != 1) return set_error(TG_EINVAL, "tuning: mapped_edges must be 0 or 1");
  if (t->bfs_graph != 0 && t->bfs_graph != 1) return set_error(TG_EINVAL, "tuning: bfs_graph must be 0 or 1");
  if (t->sssp_pull < 0 || t->sssp_pull > 100) return set_error(TG_EINVAL, "tuning: sssp_pull must be in [0, 100]");
  if (t->sssp_lanes < 1 || t->sssp_lanes > MAX_LANES)
    return set_error(TG_EINVAL, "tuning: sssp_lanes outside [1, %d]", MAX_LANES);
  if (t->sssp_packed != 0 && t->sssp_packed != 1) return set_error(TG_EINVAL, "tuning: sssp_packed must be 0 or 1");
  if (t->sssp_ring != 0 && t->sssp_ring != 1) return set_error(TG_EINVAL, "tuning: sssp_ring must be 0 or 1");
  if (t->sssp_split != 0 && t->sssp_split != 1) return set_error(TG_EINVAL, "tuning: sssp_split must be 0 or 1");
  if (t->sssp_hpull < 0 || t->sssp_hpull > 100000)
    return set_error(TG_EINVAL, "tuning: sssp_hpull must be in [0, 100000]");
  if (t->bfs_lanes < 1 || t->bfs_lanes > MAX_BFS_LANES)
    return set_error(TG_EINVAL, "tuning: bfs_lanes outside [1, %d]", MAX_BFS_LANES);
  if (t->bfs_td_grid < 1 || t->bfs_td_grid > 16384 || t->bfs_bu_grid < 2 || t->bfs_bu_grid > 16384)
    return set_error(TG_EINVAL, "tuning: bfs_td_grid must be in [1, 16384] and bfs_bu_grid in [2, 16384]");
  if (t->sssp_xcd != 0 && t->sssp_xcd != 1) return set_error(TG_EINVAL, "tuning: sssp_xcd must be 0 or 1");
  if (t->bfs_do != 0 && t->bfs_do != 1) return set_error(TG_EINVAL, "tuning: bfs_do must be 0 or 1");
  if (t->bfs_alpha < 1 || t->bfs_alpha > 1000000 || t->bfs_beta < 1 || t->bfs_beta > 1000000)
    return set_error(TG_EINVAL, "tuning: bfs_alpha and bfs_beta must be in [1, 10^6]");
  if (t->pr_xcd != 0 && t->pr_xcd != 1) return set_error(TG_EINVAL, "tuning: pr_xcd must be 0 or 1");
  if (t->pr_rows != 256 && t->pr_rows != 512) return set_error(TG_EINVAL, "tuning: pr_rows must be 256 or 512");
  if (t->sssp_delta < 0 || t->sssp_delta > INT32_MAX / 2) return set_error(TG_EINVAL, "tuning: sssp_delta outside [0, 2^30]");
  if (t->sssp_lds_verts < 0 || t->sssp_lds_verts > 14336) return set_error(TG_EINVAL, "tuning: sssp_lds_verts outside [0, 14336]");
  if (t->sssp_grid < 1 || t->sssp_grid > 16384) return set_error(TG_EINVAL, "tuning: sssp_grid outside [1, 16384]");
  if (t->pr_lds_verts < 0 || t->pr_lds_verts > 40960) return set_error(TG_EINVAL, "tuning: pr_lds_verts outside [0, 40960]");
  if (t->bfs_lds_words < 0 || t->bfs_lds_words > 14336) return set_error(TG_EINVAL, "tuning: bfs_lds_words outside [0, 14336]");
  if (t->pr_grid < 1 || t->pr_grid > 16384 || t->bfs_grid < 1 || t->bfs_grid > 16384)
    return set_error(TG_EINVAL, "tuning: grids must be in [1, 16384]");
  if (t->bfs_lds_min_vblocks < 0) return set_error(TG_EINVAL, "tuning: bfs_lds_min_vblocks < 0");
  for (int b = 0; b < 5; ++b)
    if (t->min_deg[b] < 1) return set_error(TG_EINVAL, "tuning: %s must be >= 1", keys[b]);
  for (int b = 0; b + 1 < 5; ++b)
    if (t->min_deg[b] < t->min_deg[b + 1])
      return set_error(TG_EINVAL, "tuning: degree thresholds must be non-increasing");
  if (t->hub_chunk < 256) return set_error(TG_EINVAL, "tuning: hub_chunk must be >= 256");
  return TG_OK;
}

}  // namespace tg

// ------------------------------------------------------------ graph load
namespace {

int validate_graph(const tg_graph &g, bool check_sym) {
  const int64_t n = g.n, m = g.m;
  if (g.off[0] != 0) return set_error(TG_EINVAL, "row_offsets[0] = %lld, expected 0", (long long)g.off[0]);
  if (g.off[n] != m)
    return set_error(TG_EINVAL, "row_offsets[V] = %lld, expected num_edges = %lld", (long long)g.off[n],
                     (long long)m);
  for (int64_t v = 0; v < n; ++v)
    if (g.off[v + 1] < g.off[v])
      return set_error(TG_EINVAL, "row_offsets decrease at vertex %lld", (long long)v);
  int64_t bad = -1;
#pragma omp parallel for schedule(static) reduction(max : bad)
  for (int64_t e = 0; e < m; ++e)
    if (g.col[e] < 0 || g.col[e] >= n) bad = std::max(bad, e);
  if (bad >= 0) return set_error(TG_EINVAL, "col_indices[%lld] = %d is out of range", (long long)bad, g.col[bad]);
  if (g.has_w) {
    bad = -1;
#pragma omp parallel for schedule(static) reduction(max : bad)
    for (int64_t e = 0; e < m; ++e)
      if (g.w[e] < 1) bad = std::max(bad, e);
    if (bad >= 0) return set_error(TG_EINVAL, "weights[%lld] = %d must be >= 1", (long long)bad, g.w[bad]);
  }
  if (check_sym) {
    // every (u, v, w) needs a (v, u, w): look it up in a sorted copy of row v
    std::vector<int64_t> key((size_t)m);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t u = 0; u < n; ++u) {
      for (int64_t e = g.off[u]; e < g.off[u + 1]; ++e)
        key[e] = ((int64_t)g.col[e] << 32) | (uint32_t)(g.has_w ? g.w[e] : 0);
      std::sort(key.begin() + g.off[u], key.begin() + g.off[u + 1]);
    }
    int64_t miss = -1;
#pragma omp parallel for schedule(dynamic, 1024) reduction(max : miss)
    for (int64_t u = 0; u < n; ++u) {
      for (int64_t e = g.off[u]; e < g.off[u + 1]; ++e) {
        const int32_t v = g.col[e];
        const int64_t want = ((int64_t)u << 32) | (uint32_t)(g.has_w ? g.w[e] : 0);
        if (!std::binary_search(key.begin() + g.off[v], key.begin() + g.off[v + 1], want))
          miss = std::max(miss, e);
      }
    }
    if (miss >= 0)
      return set_error(TG_EINVAL, "graph flagged symmetric but edge %lld has no reverse edge of equal weight",
                       (long long)miss);
  }
  return TG_OK;
}

}  // namespace

extern "C" int graph_load_csr(int64_t num_vertices, int64_t num_edges, const int64_t *row_offsets,
                              const int32_t *col_indices, const int32_t *weights, uint32_t flags,
                              void *stream, tg_graph **out) {
  clear_error();
  if (!out) return set_error(TG_EINVAL, "graph_load_csr: out is NULL");
  *out = nullptr;
  if (num_vertices < 0 || num_vertices > INT32_MAX)
    return set_error(TG_EINVAL, "num_vertices = %lld outside [0, INT32_MAX]", (long long)num_vertices);
  if (num_edges < 0) return set_error(TG_EINVAL, "num_edges = %lld < 0", (long long)num_edges);
  if (!row_offsets) return set_error(TG_EINVAL, "row_offsets is NULL");
  if (num_edges > 0 && !col_indices) return set_error(TG_EINVAL, "col_indices is NULL");
  tg_graph *g = new (std::nothrow) tg_graph();
  if (!g) return set_error(TG_ENOMEM, "graph_load_csr: out of host memory");
  try {
    g->n = num_vertices;
    g->m = num_edges;
    g->symmetric = (flags & TG_SYMMETRIC) != 0;
    g->has_w = weights != nullptr;
    g->off.resize((size_t)num_vertices + 1);
    g->col.resize((size_t)num_edges);
    if (g->has_w) g->w.resize((size_t)num_edges);
  } catch (...) {
    delete g;
    return set_error(TG_ENOMEM, "graph_load_csr: out of host memory for %lld edges", (long long)num_edges);
  }
  if (flags & TG_PTRS_DEVICE) {
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(g->off.data(), row_offsets, (num_vertices + 1) * sizeof(int64_t),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && num_edges)
      e = hipMemcpyAsync(g->col.data(), col_indices, num_edges * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && g->has_w && num_edges)
      e = hipMemcpyAsync(g->w.data(), weights, num_edges * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      delete g;
      return set_error(TG_EDEVICE, "graph_load_csr: device copy failed: %s", hipGetErrorString(e));
    }
  } else {
    memcpy(g->off.data(), row_offsets, (num_vertices + 1) * sizeof(int64_t));
    if (num_edges) memcpy(g->col.data(), col_indices, num_edges * sizeof(int32_t));
    if (g->has_w && num_edges) memcpy(g->w.data(), weights, num_edges * sizeof(int32_t));
  }
  if (flags & TG_VALIDATE) {
    int rc = validate_graph(*g, g->symmetric);
    if (rc != TG_OK) {
      delete g;
      return rc;
    }
  } else if (g->off[0] != 0 || g->off[num_vertices] != num_edges) {
    delete g;
    return set_error(TG_EINVAL, "row_offsets do not span [0, num_edges]");
  }
  *out = g;
  return TG_OK;
}

extern "C" void graph_free(tg_graph *g) { delete g; }

// -------------------------------------------------- partition by degree
namespace {

// Bin boundaries over a sequence whose degrees are non-increasing.
BinBounds bins_of(const std::vector<int64_t> &deg_in_order, const Tuning &t) {
  BinBounds bb;
  const int64_t n = (int64_t)deg_in_order.size();
  int64_t i = 0;
  for (int b = 0; b < NBIN; ++b) {
    while (i < n && bin_of_degree(deg_in_order[i], t) < b) ++i;
    bb.bstart[b] = i;
  }
  bb.bstart[NBIN] = n;
  return bb;
}

// The same boundaries from unsorted degrees (positions they would have after
// a sort by decreasing degree).
BinBounds bins_of_unsorted(const std::vector<int64_t> &deg, const Tuning &t) {
  int64_t cnt[NBIN] = {};
  for (int64_t d : deg) cnt[bin_of_degree(d, t)]++;
  BinBounds bb;
  int64_t acc = 0;
  for (int b = 0; b < NBIN; ++b) {
    bb.bstart[b] = acc;
    acc += cnt[b];
  }
  bb.bstart[NBIN] = acc;
  return bb;
}

}  // namespace

namespace tg {

// Stable counting sort of `ids` by key descending (keys >= 0).
void sort_desc_by_key(const std::vector<int64_t> &key, std::vector<int32_t> &ids) {
  if (ids.empty()) return;
  int64_t maxk = 0;
  for (int32_t v : ids) maxk = std::max(maxk, key[v]);
  std::vector<int64_t> cnt((size_t)maxk + 2, 0);
  for (int32_t v : ids) cnt[(size_t)(maxk - key[v]) + 1]++;
  for (size_t i = 1; i < cnt.size(); ++i) cnt[i] += cnt[i - 1];
  std::vector<int32_t> outv(ids.size());
  for (int32_t v : ids) outv[(size_t)cnt[(size_t)(maxk - key[v])]++] = v;
  ids.swap(outv);
}

// In-edges of a CSR over n vertices: rows sorted ascending (deterministic).
void transpose_csr(int64_t n, const std::vector<int64_t> &off, const std::vector<int32_t> &col,
                   std::vector<int64_t> &ioff, std::vector<int32_t> &icol) {
  const int64_t m = off[n];
  std::vector<int64_t> cnt((size_t)n + 1, 0);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) __atomic_fetch_add(&cnt[(size_t)col[e] + 1], (int64_t)1, __ATOMIC_RELAXED);
  ioff.assign((size_t)n + 1, 0);
  for (int64_t i = 0; i < n; ++i) ioff[i + 1] = ioff[i] + cnt[i + 1];
  icol.resize((size_t)m);
  std::vector<int64_t> cur(ioff.begin(), ioff.end() - 1);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t u = 0; u < n; ++u)
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      const int64_t k = __atomic_fetch_add(&cur[col[e]], (int64_t)1, __ATOMIC_RELAXED);
      icol[(size_t)k] = (int32_t)u;
    }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v) std::sort(icol.begin() + ioff[v], icol.begin() + ioff[v + 1]);
}

}  // namespace tg

namespace {

template <typename T>
int upload(tg::DevArena &a, T **dst, const T *src, size_t count) {
  TG_TRY(dalloc(a, dst, count));
  if (count) TG_HIP(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
  return TG_OK;
}

}  // namespace

namespace tg {

// Derive the degree bins and the static PageRank plan from the tuning.
int apply_tuning(tg_partition *p, const Tuning &t) {
  GpuPart &gp = p->gpu;
  p->tune = t;
  ++p->tune_gen;
  if (gp.mapped_edges) {
    // the per-XCD class layouts copy the edges into device memory: with the
    // edges kept on the host the kernels read the CSR itself
    p->tune.pr_xcd = 0;
    p->tune.sssp_xcd = 0;
    p->tune.sssp_pull = 0;
  }
  p->tune.mapped_edges = gp.mapped_edges ? 1 : 0;  // fixed at build
  gp.out_bins = bins_of(gp.h_deg, t);
  gp.in_bins = gp.in_alias ? gp.out_bins : bins_of_unsorted(gp.h_in_deg, t);
  gp.max_out_hubs = gp.out_bins.bstart[1] - gp.out_bins.bstart[0];
  return TG_OK;
}

// A 32-bit copy of CSR offsets when every offset fits (m < 2^31): half the
// offset bytes of a bottom-up BFS step, which reads them for every
// unvisited vertex.  Left null otherwise.
// The first four in-neighbours of every vertex, four int32 per vertex (-1
// past the row): a bottom-up BFS step reads them with one 16-byte load per
// vertex, consecutive vertices side by side, and usually finds a parent
// among them (rows are sorted by id, i.e. by decreasing degree).
int upload_head(DevArena &A, int32_t **d, const std::vector<int64_t> &off, const std::vector<int32_t> &col,
                int64_t n) {
  std::vector<int32_t> head((size_t)std::max<int64_t>(n, 1) * 4, -1);
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v)
    for (int64_t j = 0; j < 4 && off[v] + j < off[v + 1]; ++j) head[(size_t)v * 4 + j] = col[off[v] + j];
  return upload(A, d, head.data(), head.size());
}

int upload_off32(DevArena &A, int32_t **d, const std::vector<int64_t> &off, int64_t m) {
  if (m >= (int64_t)INT32_MAX) return TG_OK;
  std::vector<int32_t> o32(off.size());
  for (size_t i = 0; i < off.size(); ++i) o32[i] = (int32_t)off[i];
  return upload(A, d, o32.data(), o32.size());
}

// Build and upload the GPU partition over the vertex subset `verts` (global
// ids).  Edges to vertices outside the subset are boundary edges: they are
// returned through `boundary` (per local source, the global destinations and
// weights) instead of being stored in the local CSR.
int build_gpu_part(tg_partition *p, const std::vector<int32_t> &verts, BoundaryEdges *boundary) {
  const tg_graph &G = *p->g;
  GpuPart &gp = p->gpu;
  const Tuning &t = p->tune;
  const int64_t V = G.n;
  // order the subset by decreasing local out-degree (counting sort, stable)
  std::vector<int32_t> order(verts);
  std::vector<int32_t> l_of_g((size_t)V, -1);
  for (size_t i = 0; i < verts.size(); ++i) l_of_g[verts[i]] = 0;  // membership
  std::vector<int64_t> ldeg((size_t)V, 0);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < (int64_t)verts.size(); ++i) {
    const int32_t u = verts[i];
    int64_t d = 0;
    for (int64_t e = G.off[u]; e < G.off[u + 1]; ++e) d += (l_of_g[G.col[e]] >= 0) ? 1 : 0;
    ldeg[u] = d;
  }
  sort_desc_by_key(ldeg, order);
  const int64_t n = (int64_t)order.size();
  for (int64_t i = 0; i < n; ++i) l_of_g[order[i]] = (int32_t)i;
  std::vector<int64_t> off((size_t)n + 1, 0);
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + ldeg[order[i]];
  const int64_t m = off[n];
  std::vector<int32_t> col((size_t)m);
  std::vector<int32_t> w(G.has_w ? (size_t)m : 0);
  if (boundary) {
    boundary->src_off.assign((size_t)n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
      const int32_t u = order[i];
      boundary->src_off[i + 1] = boundary->src_off[i] + (G.off[u + 1] - G.off[u]) - ldeg[u];
    }
    boundary->dst.resize((size_t)boundary->src_off[n]);
    boundary->w.resize(G.has_w ? (size_t)boundary->src_off[n] : 0);
  }
  int fail = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : fail)
  for (int64_t i = 0; i < n; ++i) {
    const int32_t u = order[i];
    std::vector<int64_t> tmp;
    tmp.reserve((size_t)(off[i + 1] - off[i]));
    int64_t bk = boundary ? boundary->src_off[i] : 0;
    for (int64_t e = G.off[u]; e < G.off[u + 1]; ++e) {
      const int32_t l = l_of_g[G.col[e]];
      const uint32_t wt = G.has_w ? (uint32_t)G.w[e] : 0u;
      if (l >= 0) {
        tmp.push_back(((int64_t)l << 32) | wt);
      } else if (boundary) {
        boundary->dst[bk] = G.col[e];
        if (G.has_w) boundary->w[bk] = G.w[e];
        ++bk;
      }
    }
    std::sort(tmp.begin(), tmp.end());
    if ((int64_t)tmp.size() != off[i + 1] - off[i]) fail |= 1;
    for (size_t k = 0; k < tmp.size(); ++k) {
      col[off[i] + k] = (int32_t)(tmp[k] >> 32);
      if (G.has_w) w[off[i] + k] = (int32_t)(uint32_t)(tmp[k] & 0xFFFFFFFFu);
    }
  }
  if (fail) return set_error(TG_EINVAL, "partition: inconsistent local degree count");

  gp.n = n;
  gp.m = m;
  gp.n_global = V;
  std::vector<int64_t> deg_in_order((size_t)n);
  for (int64_t i = 0; i < n; ++i) deg_in_order[i] = off[i + 1] - off[i];
  gp.n_dangling = 0;
  DevArena &A = p->arena;
  TG_TRY(upload(A, &gp.out.off, off.data(), (size_t)n + 1));
  // edge arrays: device memory, or mapped host memory read over the host link
  gp.mapped_edges = p->tune.mapped_edges != 0;
  auto edges = [&](int32_t **d, const std::vector<int32_t> &h) -> int {
    if (!gp.mapped_edges) return upload(A, d, h.data(), (size_t)m);
    return p->mapped.upload(reinterpret_cast<void **>(d), h.data(), (size_t)m * sizeof(int32_t));
  };
  TG_TRY(edges(&gp.out.col, col));
  if (G.has_w) TG_TRY(edges(&gp.out.w, w));
  gp.max_w = 0;
  if (G.has_w)
    for (int64_t e = 0; e < m; ++e) gp.max_w = std::max(gp.max_w, w[e]);
  if (G.has_w && n <= (int64_t)1 << 24) {
    // the relaxation's edge stream in one word per edge, if every weight fits in 8 bits
    bool small = true;
    for (int64_t e = 0; e < m && small; ++e) small = w[e] >= 0 && w[e] < 256;
    if (small) {
      // each row by weight (the word's top byte), so that the edges lighter
      // than a bound are a prefix of the row (the light/heavy split)
      std::vector<int32_t> cw((size_t)m);
#pragma omp parallel for schedule(dynamic, 1024)
      for (int64_t v = 0; v < n; ++v) {
        uint32_t *row = reinterpret_cast<uint32_t *>(cw.data()) + off[v];
        const int64_t len = off[v + 1] - off[v];
        for (int64_t k = 0; k < len; ++k) row[k] = (uint32_t)col[off[v] + k] | ((uint32_t)w[off[v] + k] << 24);
        std::sort(row, row + len);
      }
      TG_TRY(edges(reinterpret_cast<int32_t **>(&gp.out.cw), cw));
    }
  }
  gp.out.n = n;
  gp.out.m = m;
  gp.h_out_off = off;

  // in-edges (transpose) unless the whole graph is symmetric and local
  const bool alias = G.symmetric && !boundary;
  std::vector<int64_t> in_deg_in_order;
  if (alias) {
    gp.in = gp.out;
    gp.in_alias = true;
    in_deg_in_order = deg_in_order;
    for (int64_t i = 0; i < n; ++i) gp.n_dangling += (deg_in_order[i] == 0);
    gp.n_isolated = gp.n_dangling;
    TG_TRY(upload_off32(A, &gp.in_off32, off, m));
    TG_TRY(upload_head(A, &gp.in_head, off, col, n));
  } else {
    std::vector<int64_t> ioff;
    std::vector<int32_t> icol;
    transpose_csr(n, off, col, ioff, icol);
    TG_TRY(upload(A, &gp.in.off, ioff.data(), (size_t)n + 1));
    TG_TRY(edges(&gp.in.col, icol));
    TG_TRY(upload_off32(A, &gp.in_off32, ioff, m));
    TG_TRY(upload_head(A, &gp.in_head, ioff, icol, n));
    gp.in.n = n;
    gp.in.m = m;
    gp.in_alias = false;
    in_deg_in_order.resize((size_t)n);  // (by local id: only binned for reporting)
    for (int64_t i = 0; i < n; ++i) in_deg_in_order[i] = ioff[i + 1] - ioff[i];
    // dangling = local out-degree 0 AND no boundary out-edges
    for (int64_t i = 0; i < n; ++i) {
      const int64_t bdeg = boundary ? boundary->src_off[i + 1] - boundary->src_off[i] : 0;
      gp.n_dangling += (deg_in_order[i] == 0 && bdeg == 0);
    }
    gp.n_isolated = 0;
  }
  gp.h_deg = std::move(deg_in_order);
  gp.h_in_deg = std::move(in_deg_in_order);
  TG_TRY(apply_tuning(p, t));

  // id maps
  p->h_g_of_l = order;
  p->h_l_of_g = l_of_g;
  TG_TRY(upload(A, &gp.g_of_l, order.data(), (size_t)std::max<int64_t>(n, 1)));
  TG_TRY(upload(A, &gp.l_of_g, l_of_g.data(), (size_t)std::max<int64_t>(V, 1)));
  return TG_OK;
}

}  // namespace tg

namespace {

// The autotuner's cache: a JSON object whose keys are
// "<arch>:V2^<round(log2 V)>:deg<round(E / V)>:<sym|dir>" and whose values
// hold a "config" object of tuning keys.  Rounding is to nearest, ties to
// even.  The file is TG_TUNING_CACHE if set, else tuning_cache.json beside
// this library.
std::string tuning_cache_path() {
  const char *env = getenv("TG_TUNING_CACHE");
  if (env && *env) return env;
  Dl_info info;
  if (dladdr((void *)&tuning_cache_path, &info) && info.dli_fname) {
    std::string lib = info.dli_fname;
    const size_t slash = lib.rfind('/');
    return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/tuning_cache.json";
  }
  return "tuning_cache.json";
}

std::string graph_signature(const tg_graph &g, int device) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
  }
  const double v = (double)std::max<int64_t>(g.n, 1);
  char buf[160];
  snprintf(buf, sizeof(buf), "%s:V2^%.0f:deg%.0f:%s", arch.c_str(), nearbyint(log2(v)),
           nearbyint((double)g.m / v), g.symmetric ? "sym" : "dir");
  return buf;
}

// The "config" object of `key` in the cache text, or "" if absent.
std::string cached_config(const std::string &text, const std::string &key) {
  const size_t k = text.find("\"" + key + "\"");
  if (k == std::string::npos) return "";
  const size_t c = text.find("\"config\"", k);
  if (c == std::string::npos) return "";
  const size_t open = text.find('{', c);
  if (open == std::string::npos) return "";
  int depth = 0;
  for (size_t i = open; i < text.size(); ++i) {
    if (text[i] == '{') ++depth;
    else if (text[i] == '}' && --depth == 0) return text.substr(open, i - open + 1);
  }
  return "";
}

// tuning_json == NULL: the cached entry for this device and graph signature,
// else the built-in values.  `source` names what was used.
int resolve_tuning(const tg_graph &g, int device, const char *tuning_json, Tuning *t, std::string *source) {
  if (tuning_json) {
    *source = "caller";
    return parse_tuning(tuning_json, t);
  }
  const std::string key = graph_signature(g, device);
  std::string text;
  if (FILE *f = fopen(tuning_cache_path().c_str(), "rb")) {
    char buf[65536];
    size_t k;
    while ((k = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, k);
    fclose(f);
  }
  const std::string cfg = cached_config(text, key);
  if (!cfg.empty() && parse_tuning(cfg.c_str(), t) == TG_OK) {
    *source = "cache " + key;
    return TG_OK;
  }
  *source = "built-in";
  return parse_tuning(nullptr, t);
}

}  // namespace

extern "C" int partition_by_degree(const tg_graph *g, int strategy, double alpha, uint64_t seed,
                                   const char *tuning_json, tg_partition **out) {
  clear_error();
  if (!out) return set_error(TG_EINVAL, "partition_by_degree: out is NULL");
  *out = nullptr;
  if (!g) return set_error(TG_EINVAL, "partition_by_degree: graph is NULL");
  if (strategy != TG_PART_HIGH && strategy != TG_PART_LOW && strategy != TG_PART_RAND)
    return set_error(TG_EINVAL, "unknown partitioning strategy %d", strategy);
  if (!(alpha >= 0.0 && alpha < 1.0)) return set_error(TG_EINVAL, "cpu_edge_share %g outside [0, 1)", alpha);
  tg_partition *p = new (std::nothrow) tg_partition();
  if (!p) return set_error(TG_ENOMEM, "partition_by_degree: out of host memory");
  p->g = g;
  p->strategy = strategy;
  p->alpha = alpha;
  int rc = (hipGetDevice(&p->device) == hipSuccess) ? TG_OK : set_error(TG_EDEVICE, "no HIP device");
  if (rc == TG_OK) rc = resolve_tuning(*g, p->device, tuning_json, &p->tune, &p->tuning_source);
  if (rc == TG_OK) {
    try {
      if (alpha == 0.0) {
        std::vector<int32_t> all((size_t)g->n);
        for (int64_t v = 0; v < g->n; ++v) all[v] = (int32_t)v;
        rc = build_gpu_part(p, all, nullptr);
      } else {
        rc = build_hybrid(p, seed);
      }
    } catch (const std::bad_alloc &) {
      rc = set_error(TG_ENOMEM, "partition_by_degree: out of host memory");
    }
  }
  // uploads went through the null stream, which is not ordered before work
  // on non-blocking streams: let them land
  if (rc == TG_OK && hipDeviceSynchronize() != hipSuccess)
    rc = set_error(TG_EDEVICE, "partition_by_degree: hipDeviceSynchronize failed");
  if (rc != TG_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return TG_OK;
}

extern "C" int partition_retune(tg_partition *p, const char *tuning_json) {
  clear_error();
  if (!p) return set_error(TG_EINVAL, "partition_retune: partition is NULL");
  Tuning t;
  TG_TRY(parse_tuning(tuning_json, &t));
  if (hipSetDevice(p->device) != hipSuccess) return set_error(TG_EDEVICE, "partition_retune: hipSetDevice failed");
  TG_HIP(hipDeviceSynchronize());
  p->tuning_source = tuning_json ? "caller" : "built-in";
  return apply_tuning(p, t);
}

extern "C" void partition_free(tg_partition *p) {
  if (!p) return;
  TG_QUIET(hipSetDevice(p->device));
  hybrid_free(p);
  delete p->slots[0];
  delete p->slots[1];
  bcb_free(p);
  pr_slices_free(p->gpu);
  pr_rows_free(p->gpu);
  sssp_slices_free(p->gpu);
  sssp_pull_free(p->gpu);
  for (hipStream_t st : p->lane_stream)
    if (st) TG_QUIET(hipStreamDestroy(st));
  for (hipStream_t st : p->graph_stream)
    if (st) TG_QUIET(hipStreamDestroy(st));
  delete p;
}

extern "C" const char *tg_last_error(void) { return g_err.c_str(); }

extern "C" void tg_set_timing(int on) { set_timing(on != 0); }

static int emit(const std::string &s, char *buf, size_t cap) {
  if (buf && cap) {
    size_t k = std::min(cap - 1, s.size());
    memcpy(buf, s.data(), k);
    buf[k] = 0;
  }
  return (int)s.size();
}

extern "C" int tg_last_stats(char *json, size_t cap) {
  std::string s = g_stats.empty() ? std::string("{}") : g_stats + "}";
  return emit(s, json, cap);
}

extern "C" int partition_info(const tg_partition *p, char *json, size_t cap) {
  clear_error();
  if (!p) return set_error(TG_EINVAL, "partition_info: partition is NULL");
  const GpuPart &g = p->gpu;
  char buf[4096];
  std::string s = "{";
  snprintf(buf, sizeof(buf),
           "\"V\":%lld,\"E\":%lld,\"strategy\":%d,\"cpu_edge_share\":%.6f,\"gpu_vertices\":%lld,"
           "\"gpu_edges\":%lld,\"gpu_device_bytes\":%zu,\"symmetric\":%s,\"dangling\":%lld,"
           "\"packed_edges\":%s,",
           (long long)p->g->n, (long long)p->g->m, p->strategy, p->alpha, (long long)g.n, (long long)g.m,
           p->arena.bytes, p->g->symmetric ? "true" : "false", (long long)g.n_dangling,
           g.out.cw ? "true" : "false");
  s += buf;
  s += "\"out_bins\":[";
  for (int b = 0; b <= NBIN; ++b) {
    snprintf(buf, sizeof(buf), "%s%lld", b ? "," : "", (long long)g.out_bins.bstart[b]);
    s += buf;
  }
  s += "],\"in_bins\":[";
  for (int b = 0; b <= NBIN; ++b) {
    snprintf(buf, sizeof(buf), "%s%lld", b ? "," : "", (long long)g.in_bins.bstart[b]);
    s += buf;
  }
  snprintf(buf, sizeof(buf),
           "],\"tuning\":{\"hub_min_deg\":%lld,\"block_min_deg\":%lld,\"wave_min_deg\":%lld,"
           "\"g16_min_deg\":%lld,\"g4_min_deg\":%lld,\"hub_chunk\":%lld,\"pr_lds_verts\":%lld,"
           "\"pr_grid\":%lld,\"bfs_lds_words\":%lld,\"bfs_grid\":%lld,\"bfs_lds_min_vblocks\":%lld,"
           "\"sssp_delta\":%lld,\"sssp_lds_verts\":%lld,\"sssp_grid\":%lld,\"pr_xcd\":%lld,\"pr_rows\":%lld,"
           "\"bfs_do\":%lld,\"bfs_alpha\":%lld,\"bfs_beta\":%lld,\"sssp_xcd\":%lld,\"bfs_lanes\":%lld,"
           "\"bfs_td_grid\":%lld,\"bfs_bu_grid\":%lld,\"sssp_pull\":%lld,\"sssp_lanes\":%lld,\"bfs_graph\":%lld,\"mapped_edges\":%lld,\"sssp_packed\":%lld,\"sssp_ring\":%lld,\"sssp_split\":%lld,\"sssp_hpull\":%lld}",
           (long long)p->tune.min_deg[0], (long long)p->tune.min_deg[1], (long long)p->tune.min_deg[2],
           (long long)p->tune.min_deg[3], (long long)p->tune.min_deg[4], (long long)p->tune.hub_chunk,
           (long long)p->tune.pr_lds_verts, (long long)p->tune.pr_grid, (long long)p->tune.bfs_lds_words,
           (long long)p->tune.bfs_grid, (long long)p->tune.bfs_lds_min_vblocks, (long long)p->tune.sssp_delta,
           (long long)p->tune.sssp_lds_verts, (long long)p->tune.sssp_grid, (long long)p->tune.pr_xcd,
           (long long)p->tune.pr_rows, (long long)p->tune.bfs_do, (long long)p->tune.bfs_alpha,
           (long long)p->tune.bfs_beta, (long long)p->tune.sssp_xcd, (long long)p->tune.bfs_lanes,
           (long long)p->tune.bfs_td_grid, (long long)p->tune.bfs_bu_grid, (long long)p->tune.sssp_pull,
           (long long)p->tune.sssp_lanes, (long long)p->tune.bfs_graph, (long long)p->tune.mapped_edges,
           (long long)p->tune.sssp_packed, (long long)p->tune.sssp_ring, (long long)p->tune.sssp_split, (long long)p->tune.sssp_hpull);
  s += buf;
  s += ",\"tuning_source\":\"" + p->tuning_source + "\"";
  s += hybrid_info_json(p);
  s += "}";
  return emit(s, json, cap);
}

// ---------------------------------------------------------- algorithms
namespace {

int check_call(const tg_partition *p, const void *out, const char *name) {
  if (!p) return set_error(TG_EINVAL, "%s: partition is NULL", name);
  if (!out && p->g->n > 0) return set_error(TG_EINVAL, "%s: output buffer is NULL", name);
  if (hipSetDevice(p->device) != hipSuccess) return set_error(TG_EDEVICE, "%s: hipSetDevice failed", name);
  return TG_OK;
}

int check_roots(const tg_partition *p, const int32_t *roots, int32_t nr, const char *name) {
  if (nr < 0) return set_error(TG_EINVAL, "%s: negative root count", name);
  if (nr > 0 && !roots) return set_error(TG_EINVAL, "%s: roots is NULL", name);
  for (int32_t i = 0; i < nr; ++i)
    if (roots[i] < 0 || roots[i] >= p->g->n)
      return set_error(TG_EINVAL, "%s: root %d out of range [0, %lld)", name, roots[i], (long long)p->g->n);
  return TG_OK;
}

}  // namespace

extern "C" int bfs(const tg_partition *pc, const int32_t *roots, int32_t num_roots, int32_t *levels,
                   int32_t *parents, void *stream) {
  clear_error();
  TG_TRY(check_call(pc, levels, "bfs"));
  TG_TRY(check_roots(pc, roots, num_roots, "bfs"));
  tg_partition *p = const_cast<tg_partition *>(pc);
  hipStream_t s = (hipStream_t)stream;
  stats_reset("bfs");
  ktimer_reset();
  if (p->alpha > 0.0) return hybrid_bfs(p, roots, num_roots, levels, parents, s);
  std::vector<int32_t> local((size_t)num_roots);
  for (int32_t r = 0; r < num_roots; ++r) local[r] = p->h_l_of_g[roots[r]];
  int64_t supersteps = 0;
  TG_TRY(gpu_bfs_roots(p, local.data(), num_roots, levels, parents, s, &supersteps));
  // counters of every lane (the other lanes' work is ordered before s)
  const int nl = bfs_lane_count(p->tune, num_roots);
  Workspace *lanes[MAX_BFS_LANES] = {&p->ws};
  for (int l = 1; l < nl; ++l) lanes[l] = p->lane_ws[l - 1].get();
  for (int l = 0; l < nl; ++l)
    for (int k = 0; k < 6; ++k) TG_TRY(stat_fetch(*lanes[l], k, s));
  TG_HIP(hipStreamSynchronize(s));
  double sums[6] = {0, 0, 0, 0, 0, 0};
  for (int l = 0; l < nl; ++l)
    for (int k = 0; k < 6; ++k) sums[k] += (double)stat_sum(*lanes[l], k);
  stats_add("roots", num_roots);
  stats_add("supersteps", (double)supersteps);
  stats_add("edges_scanned", sums[0]);
  stats_add("vertices_expanded", sums[1]);
  stats_add("bottom_up_edges_checked", sums[2]);
  stats_add("bottom_up_steps", sums[3]);
  stats_add("bottom_up_vertices_examined", sums[5]);
  stats_add("lanes", nl);
  ktimer_emit();
  return TG_OK;
}

extern "C" int sssp(const tg_partition *pc, const int32_t *roots, int32_t num_roots, int32_t *dist,
                    void *stream) {
  clear_error();
  TG_TRY(check_call(pc, dist, "sssp"));
  TG_TRY(check_roots(pc, roots, num_roots, "sssp"));
  if (!pc->g->has_w) return set_error(TG_EUNSUPPORTED, "sssp: the graph was loaded without weights");
  tg_partition *p = const_cast<tg_partition *>(pc);
  hipStream_t s = (hipStream_t)stream;
  stats_reset("sssp");
  ktimer_reset();
  if (p->alpha > 0.0) return hybrid_sssp(p, roots, num_roots, dist, s);
  int64_t rounds_total = 0, pulls_total = 0;
  std::vector<int32_t> local((size_t)num_roots);
  for (int32_t r = 0; r < num_roots; ++r) local[r] = p->h_l_of_g[roots[r]];
  TG_TRY(gpu_sssp_roots(p, local.data(), num_roots, dist, s, &rounds_total, &pulls_total));
  TG_HIP(hipStreamSynchronize(s));
  stats_add("roots", num_roots);
  stats_add("supersteps", (double)rounds_total);
  stats_add("pull_supersteps", (double)pulls_total);
  ktimer_emit();
  return TG_OK;
}

extern "C" int cc(const tg_partition *pc, int32_t *labels, void *stream) {
  clear_error();
  TG_TRY(check_call(pc, labels, "cc"));
  if (pc->alpha > 0.0) return set_error(TG_EUNSUPPORTED, "cc: hybrid partitions are not supported");
  tg_partition *p = const_cast<tg_partition *>(pc);
  hipStream_t s = (hipStream_t)stream;
  stats_reset("cc");
  ktimer_reset();
  TG_TRY(p->ws.ensure(p->gpu, 0));
  TG_TRY(stat_zero_all(p->ws, s));
  int64_t rounds = 0;
  TG_TRY(gpu_cc(p, s, &rounds));
  if (p->gpu.n > 0) TG_TRY(collect_i32(p->gpu, p->ws.state, labels, s));
  TG_TRY(stat_fetch(p->ws, 0, s));
  TG_HIP(hipStreamSynchronize(s));
  stats_add("supersteps", (double)rounds);
  stats_add("edges_pushed", (double)stat_sum(p->ws, 0));
  ktimer_emit();
  return TG_OK;
}

extern "C" int pagerank(const tg_partition *pc, float damping, int32_t iterations, int32_t dangling_mode,
                        float *rank, void *stream) {
  clear_error();
  TG_TRY(check_call(pc, rank, "pagerank"));
  if (!(damping >= 0.0f && damping <= 1.0f)) return set_error(TG_EINVAL, "pagerank: damping %g outside [0, 1]", damping);
  if (iterations < 0) return set_error(TG_EINVAL, "pagerank: iterations < 0");
  if (dangling_mode != TG_PR_DANGLING_UNIFORM && dangling_mode != TG_PR_DANGLING_DROP)
    return set_error(TG_EINVAL, "pagerank: unknown dangling mode %d", dangling_mode);
  tg_partition *p = const_cast<tg_partition *>(pc);
  hipStream_t s = (hipStream_t)stream;
  stats_reset("pagerank");
  ktimer_reset();
  if (p->g->n == 0) return TG_OK;
  if (p->alpha > 0.0) return hybrid_pagerank(p, damping, iterations, dangling_mode, rank, s);
  TG_TRY(gpu_pagerank(p, (double)damping, iterations, dangling_mode, rank, s));
  TG_HIP(hipStreamSynchronize(s));
  stats_add("supersteps", iterations);
  ktimer_emit();
  return TG_OK;
}

extern "C" int bc(const tg_partition *pc, const int32_t *sources, int32_t num_sources, float *scores,
                  void *stream) {
  clear_error();
  TG_TRY(check_call(pc, scores, "bc"));
  TG_TRY(check_roots(pc, sources, num_sources, "bc"));
  tg_partition *p = const_cast<tg_partition *>(pc);
  hipStream_t s = (hipStream_t)stream;
  stats_reset("bc");
  ktimer_reset();
  if (p->alpha > 0.0) return hybrid_bc(p, sources, num_sources, scores, s);
  TG_TRY(p->ws.ensure(p->gpu, 0));
  TG_TRY(fill_f64(p->ws.bc_acc, p->gpu.n, 0.0, s));
  TG_HIP(hipMemsetAsync(p->ws.counters, 0, 64 * sizeof(uint32_t), s));
  for (int32_t i = 0; i < num_sources; ++i) TG_TRY(gpu_bc_source(p, p->h_l_of_g[sources[i]], s));
  TG_TRY(collect_f64_to_f32(p->gpu, p->ws.bc_acc, scores, s));
  TG_HIP(hipMemcpyAsync(p->ws.h_flags, p->ws.counters, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  if (p->ws.h_flags[2]) return set_error(TG_ERANGE, "bc: a shortest-path count reached 2^53");
  stats_add("sources", num_sources);
  ktimer_emit();
  return TG_OK;
}

extern "C" int bfs_batched(const tg_partition *pc, const int32_t *roots, int32_t num_roots, int32_t *levels,
                           void *stream) {
  clear_error();
  TG_TRY(check_call(pc, levels, "bfs_batched"));
  TG_TRY(check_roots(pc, roots, num_roots, "bfs_batched"));
  if (pc->alpha > 0.0) return set_error(TG_EUNSUPPORTED, "bfs_batched: hybrid partitions run bfs() only");
  tg_partition *p = const_cast<tg_partition *>(pc);
  hipStream_t s = (hipStream_t)stream;
  stats_reset("bfs_batched");
  ktimer_reset();
  int64_t steps = 0;
  TG_TRY(slots_run_batch(p, kSlotBfs, roots, num_roots, levels, s, &steps));
  TG_HIP(hipStreamSynchronize(s));
  stats_add("roots", num_roots);
  stats_add("supersteps", (double)steps);
  ktimer_emit();
  return TG_OK;
}

extern "C" int sssp_batched(const tg_partition *pc, const int32_t *roots, int32_t num_roots, int32_t *dist,
                            void *stream) {
  clear_error();
  TG_TRY(check_call(pc, dist, "sssp_batched"));
  TG_TRY(check_roots(pc, roots, num_roots, "sssp_batched"));
  if (!pc->g->has_w) return set_error(TG_EUNSUPPORTED, "sssp_batched: the graph was loaded without weights");
  if (pc->alpha > 0.0) return set_error(TG_EUNSUPPORTED, "sssp_batched: hybrid partitions run sssp() only");
  tg_partition *p = const_cast<tg_partition *>(pc);
  hipStream_t s = (hipStream_t)stream;
  stats_reset("sssp_batched");
  ktimer_reset();
  int64_t steps = 0;
  TG_TRY(slots_run_batch(p, kSlotSssp, roots, num_roots, dist, s, &steps));
  TG_HIP(hipStreamSynchronize(s));
  stats_add("roots", num_roots);
  stats_add("supersteps", (double)steps);
  ktimer_emit();
  return TG_OK;
}

extern "C" int bc_batched(const tg_partition *pc, const int32_t *sources, int32_t num_sources, float *scores,
                          void *stream) {
  clear_error();
  TG_TRY(check_call(pc, scores, "bc_batched"));
  TG_TRY(check_roots(pc, sources, num_sources, "bc_batched"));
  tg_partition *p = const_cast<tg_partition *>(pc);
  hipStream_t s = (hipStream_t)stream;
  stats_reset("bc_batched");
  ktimer_reset();
  if (p->alpha > 0.0) return set_error(TG_EUNSUPPORTED, "bc_batched: hybrid partitions are not supported");
  TG_TRY(p->ws.ensure(p->gpu, 0));
  TG_TRY(fill_f64(p->ws.bc_acc, p->gpu.n, 0.0, s));
  TG_TRY(gpu_bc_batched(p, sources, num_sources, s));
  TG_TRY(collect_f64_to_f32(p->gpu, p->ws.bc_acc, scores, s));
  TG_HIP(hipStreamSynchronize(s));
  stats_add("sources", num_sources);
  ktimer_emit();
  return TG_OK;
}

// Many graphs (section 5's workloads of uneven size): each graph's batched BC
// runs on a stream of its own, at most kMultiStreams graphs at a time, the
// largest first, so that small graphs fill the device together.  Each worker
// host thread drives one stream; the caller's stream is ordered before the
// first and after the last of them.
extern "C" int bc_multi(const tg_partition *const *parts, int32_t num_graphs, const int32_t *const *sources,
                        const int32_t *num_sources, float *const *scores, void *stream) {
  clear_error();
  constexpr int kMultiStreams = 8;
  if (num_graphs < 0) return set_error(TG_EINVAL, "bc_multi: negative graph count");
  if (num_graphs == 0) return TG_OK;
  if (!parts || !sources || !num_sources || !scores) return set_error(TG_EINVAL, "bc_multi: NULL array");
  for (int32_t i = 0; i < num_graphs; ++i) {
    TG_TRY(check_call(parts[i], scores[i], "bc_multi"));
    TG_TRY(check_roots(parts[i], sources[i], num_sources[i], "bc_multi"));
    if (parts[i]->alpha > 0.0) return set_error(TG_EUNSUPPORTED, "bc_multi: graph %d is a hybrid partition", i);
    if (parts[i]->device != parts[0]->device) return set_error(TG_EINVAL, "bc_multi: graphs on different devices");
    for (int32_t j = 0; j < i; ++j)
      if (parts[j] == parts[i]) return set_error(TG_EINVAL, "bc_multi: graph %d repeats graph %d", i, j);
  }
  hipStream_t s = (hipStream_t)stream;
  stats_reset("bc_multi");
  const int nstreams = std::min<int>(kMultiStreams, num_graphs);
  std::vector<hipStream_t> ws((size_t)nstreams, nullptr);
  hipEvent_t start = nullptr;
  TG_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
  TG_HIP(hipEventRecord(start, s));
  int rc = TG_OK;
  for (int k = 0; k < nstreams && rc == TG_OK; ++k) {
    if (hipStreamCreateWithFlags(&ws[k], hipStreamNonBlocking) != hipSuccess ||
        hipStreamWaitEvent(ws[k], start, 0) != hipSuccess)
      rc = set_error(TG_EDEVICE, "bc_multi: stream set-up failed");
  }
  if (rc == TG_OK) {
    std::vector<int32_t> order((size_t)num_graphs);
    for (int32_t i = 0; i < num_graphs; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return parts[a]->gpu.m + parts[a]->gpu.n > parts[b]->gpu.m + parts[b]->gpu.n;
    });
    std::atomic<int32_t> next{0};
    std::vector<int> wrc((size_t)nstreams, TG_OK);
    std::vector<std::string> werr((size_t)nstreams);
    auto work = [&](int k) {
      if (hipSetDevice(parts[0]->device) != hipSuccess) {
        wrc[k] = set_error(TG_EDEVICE, "bc_multi: hipSetDevice failed");
        werr[k] = tg_last_error();
        return;
      }
      for (;;) {
        const int32_t q = next.fetch_add(1);
        if (q >= num_graphs) break;
        const int32_t i = order[q];
        tg_partition *p = const_cast<tg_partition *>(parts[i]);
        auto one = [&]() -> int {
          TG_TRY(p->ws.ensure(p->gpu, 0));
          TG_TRY(fill_f64(p->ws.bc_acc, p->gpu.n, 0.0, ws[k]));
          TG_TRY(gpu_bc_batched(p, sources[i], num_sources[i], ws[k]));
          TG_TRY(collect_f64_to_f32(p->gpu, p->ws.bc_acc, scores[i], ws[k]));
          TG_HIP(hipStreamSynchronize(ws[k]));
          return TG_OK;
        };
        const int r = one();
        if (r != TG_OK) {
          wrc[k] = r;
          werr[k] = std::string("graph ") + std::to_string(i) + ": " + tg_last_error();
          next.store(num_graphs);  // stop handing out graphs
          return;
        }
      }
    };
    std::vector<std::thread> th;
    for (int k = 1; k < nstreams; ++k) th.emplace_back(work, k);
    work(0);
    for (auto &t : th) t.join();
    for (int k = 0; k < nstreams && rc == TG_OK; ++k)
      if (wrc[k] != TG_OK) rc = set_error(wrc[k], "bc_multi: %s", werr[k].c_str());
  }
  // the caller's stream waits for every worker stream
  for (int k = 0; k < nstreams; ++k) {
    if (!ws[k]) continue;
    hipEvent_t done = nullptr;
    if (hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess) {
      TG_QUIET(hipEventRecord(done, ws[k]));
      TG_QUIET(hipStreamWaitEvent(s, done, 0));
      TG_QUIET(hipEventDestroy(done));
    }
  }
  TG_QUIET(hipStreamSynchronize(s));
  for (int k = 0; k < nstreams; ++k)
    if (ws[k]) TG_QUIET(hipStreamDestroy(ws[k]));
  TG_QUIET(hipEventDestroy(start));
  if (rc != TG_OK) return rc;
  int64_t total = 0;
  for (int32_t i = 0; i < num_graphs; ++i) total += num_sources[i];
  stats_add("graphs", num_graphs);
  stats_add("sources", (double)total);
  stats_add("streams", nstreams);
  return TG_OK;
}

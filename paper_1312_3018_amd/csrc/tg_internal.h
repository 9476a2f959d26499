// Host-side internals of libtg: graph and partition objects, device
// workspace, error reporting and the launchers each kernel file provides.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/tg.h"
#include "kcommon.h"

using tgk::BinBounds;
using tgk::NBIN;
using tgk::Plan;

// ------------------------------------------------------------------ errors
namespace tg {
// per-kernel event timing (ktimer.cpp); no-ops unless TG_TIMING is set
bool timing_enabled();
void set_timing(bool on);
int ktimer_start(hipStream_t s);
void ktimer_stop(int start, hipStream_t s, const char *name);
void ktimer_flush();  // after a stream sync: fold pending event pairs into totals
void ktimer_reset();
void ktimer_emit();   // add totals to the call's stats
// Per kernel name: summed duration and launches, and each launch's interval
// from the call's reference event.
struct KTimes {
  std::map<std::string, std::pair<double, long long>> acc;
  std::map<std::string, std::vector<std::pair<float, float>>> iv;
};
// Totals gathered on another thread (a lane of a multi-search call) move to
// the calling thread: the lane measures from the caller's reference event
// (ktimer_ensure_ref there: records it on s if the call has none yet; null
// with timing off; ktimer_set_ref in the lane), exports after its last
// launch, and the caller imports.
KTimes ktimer_export();
void ktimer_import(const KTimes &k);
hipEvent_t ktimer_ensure_ref(hipStream_t s);
void ktimer_set_ref(hipEvent_t ref);
int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
void stats_reset(const char *algo);
void stats_add(const char *key, double value);
}  // namespace tg

#define TG_HIP(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return tg::set_error(TG_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// A runtime call whose failure is not an error of the current call (frees,
// timing queries): report it on stderr when TG_DEBUG is set.
namespace tg {
void debug_hip(hipError_t e, const char *what);
}
#define TG_QUIET(expr) tg::debug_hip((expr), #expr)

#define TG_TRY(expr)          \
  do {                        \
    int rc_ = (expr);         \
    if (rc_ != TG_OK) return rc_; \
  } while (0)

namespace tg {

// Degree thresholds of the bins (minimum degree of bins HUB..G4; G1 starts
// at degree 1) and the edges per HUB chunk.
struct Tuning {
  int64_t min_deg[tgk::BIN_G1];  // HUB, BLOCK, WAVE, G16, G4
  int64_t hub_chunk;
  int64_t pr_lds_verts;          // PageRank: hot contributions staged in LDS per workgroup (at most)
  int64_t pr_grid;               // PageRank: workgroups per launch (at most)
  int64_t bfs_lds_words;         // BFS: visited-bitmap words staged in LDS per block
  int64_t bfs_grid;              // BFS: blocks per launch when staging
  int64_t bfs_lds_min_vblocks;   // BFS: stage only for frontiers at least this large
  int64_t sssp_delta;            // SSSP: near/far distance step (0 = plain frontier Bellman-Ford)
  int64_t sssp_lds_verts;        // SSSP: distances of vertices [0, n) snapshotted in LDS per block
  int64_t sssp_grid;             // SSSP: blocks per launch when snapshotting
  int64_t pr_xcd;                // PageRank: 1 = gather split by source class per XCD
  int64_t pr_rows;               // PageRank: edges per row block (one wave's block)
  int64_t bfs_do;                // BFS: 1 = switch to bottom-up steps on large frontiers
  int64_t bfs_alpha, bfs_beta;   // BFS: top-down -> bottom-up when m_f > m_u / alpha; back when n_f < n / beta
  int64_t sssp_xcd;              // SSSP: 1 = relaxation split by destination class per XCD
  int64_t bfs_lanes;             // BFS: searches in flight on their own streams (1 or 2)
  int64_t bfs_td_grid;           // BFS: blocks of a top-down launch (fixed: the frontier size is on the device)
  int64_t bfs_bu_grid;           // BFS: blocks of a bottom-up launch's one-thread-per-vertex part
  int64_t sssp_pull;             // SSSP: pull a superstep whose frontier has more than this % of the edges (0: never)
  int64_t sssp_lanes;            // SSSP: searches in flight on their own streams (1..4)
  int64_t sssp_packed;           // SSSP: relax from the packed id|weight words when the partition has them
  int64_t sssp_ring;             // SSSP near/far: a ring of bucket bitmaps (1) or one far pile rescanned per step (0)
  int64_t sssp_split;            // SSSP ring: edges lighter than the step relax per pass, heavier ones once per bucket
  int64_t sssp_hpull;            // SSSP split, symmetric graphs: a bucket's heavy pass pulls when the unsettled
                                 // vertices' degree sum times this percent is below the members' (0: always push)
  int64_t bfs_graph;             // BFS: 1 = chunks of supersteps replayed as captured HIP graphs
  int64_t mapped_edges;          // partition build: 1 = edge arrays in mapped host memory
};
Tuning default_tuning();
int parse_tuning(const char *json, Tuning *t);

// Bin of a vertex with degree d.
inline int bin_of_degree(int64_t d, const Tuning &t) {
  if (d == 0) return tgk::BIN_ZERO;
  for (int b = 0; b < tgk::BIN_G1; ++b)
    if (d >= t.min_deg[b]) return b;
  return tgk::BIN_G1;
}

// ------------------------------------------------------------ device memory
struct DevArena {
  std::vector<void *> ptrs;
  size_t bytes = 0;
  int alloc(void **p, size_t n);  // zero-size -> 256 bytes
  void release();
  void release_one(void *p);       // free one allocation early
  ~DevArena() { release(); }
};

template <typename T>
int dalloc(DevArena &a, T **p, size_t count) {
  return a.alloc(reinterpret_cast<void **>(p), count * sizeof(T));
}

// Pinned host memory mapped into the device's address space (kernels read it
// over the host link), freed with the owner.
struct HostMappedArena {
  std::vector<void *> ptrs;
  size_t bytes = 0;
  // *dev: the device address of a new copy of src[0, count)
  int upload(void **dev, const void *src, size_t bytes);
  ~HostMappedArena();
};

// ------------------------------------------------------------ graph object
}  // namespace tg

struct tg_graph {
  int64_t n = 0, m = 0;
  bool symmetric = false;
  bool has_w = false;
  std::vector<int64_t> off;
  std::vector<int32_t> col;
  std::vector<int32_t> w;
};

namespace tg {

// A CSR in device memory with a static plan over all of its vertices.
struct DevCSR {
  int64_t n = 0, m = 0;
  int64_t *off = nullptr;
  int32_t *col = nullptr;
  int32_t *w = nullptr;
  // id and weight in one word, id | w << 24, where every id fits in 24 bits
  // and every weight in 8 (out-edges of a weighted partition only); each
  // row sorted by weight
  uint32_t *cw = nullptr;
};

struct PrSlices;
struct PrRows;
struct SsspSlices;
struct SsspPull;

// Per-XCD edge classes (class_csr.hip): class = 128-byte line of the 4-byte
// state of the vertex an edge points at, mod 8.
__host__ __device__ inline int line_class(int32_t u) { return (u >> 5) & 7; }
struct ClassBase {
  int64_t base[8];  // first edge of class k in scol / sw
};
struct ClassCsr {
  DevArena arena;
  int32_t *soff = nullptr;  // [8][n+1] row offsets relative to base[k]
  int32_t *scol = nullptr;  // [m + 64] targets, class by class (padded)
  int32_t *sw = nullptr;    // [m + 64] weights in the same order, or null
  ClassBase cb{};
  int64_t n = 0, m = 0;
};
// Build C from a CSR (off, col, optional w).  hsoff gets the host copy of
// soff and hcnt the class row lengths [8][n].  Waits on s.
int build_class_csr(const int64_t *off, const int32_t *col, const int32_t *w, int64_t n, int64_t m, ClassCsr &C,
                    std::vector<int32_t> &hsoff, std::vector<int32_t> &hcnt, hipStream_t s);

// Row blocks of a CSR for the PageRank gather (pr_rows.hip).
struct RowBlk {
  int64_t e0;  // first edge, relative to the CSR's own first edge
  int32_t r0;  // first row
  int32_t lr;  // -1: whole rows [r0, next block's r0); else this block is a chunk of long row `lr`
};
struct RowBlocksHost {
  std::vector<RowBlk> rb;       // blocks, then a sentinel {E, nrows, -1}
  std::vector<int32_t> lr_b0;   // long row -> index of its first chunk block (first_block-based)
  std::vector<int32_t> lr_nch;  // long row -> number of chunks
  std::vector<int64_t> lr_pos;  // long row -> where its result goes (pos_base + row)
};
// Pack rows [0, nrows) (offsets off64 or off32) into blocks of at most nnz
// edges and nnz - 1 rows; longer rows become chunks of nnz edges.
void build_row_blocks(int64_t nrows, const int64_t *off64, const int32_t *off32, int32_t nnz, int64_t first_block,
                      int64_t pos_base, RowBlocksHost &out);
struct RowsDev {
  DevArena arena;
  RowBlk *rb = nullptr;
  int32_t *lr_b0 = nullptr, *lr_nch = nullptr;
  int64_t *lr_pos = nullptr;
  double *chunk_part = nullptr;  // per block: chunk partial sums
  double *long_part = nullptr;   // per long-row block: dangling partials (LONG_GRID)
  int64_t nb_total = 0, nlr = 0;
};
constexpr int LONG_GRID = 1024;  // blocks of the long-row launch, at most
int rows_upload(RowsDev &D, const RowBlocksHost &h);
int long_grid(int64_t nlr);
// One block: *dsum_out = sum(pa[0..na)) + sum(pb[0..nb)) + iso_count * ((1-d)/N + d D/N)
int pr_dsum_launch(const double *pa, int32_t na, const double *pb, int32_t nb, double iso_count, double base,
                   double d, double inv_n, int32_t drop, const double *dsum_in, double *dsum_out, hipStream_t s);
// Kernel arguments.  Class mode: class k's blocks are rb[rb_base[k] ..
// rb_base[k] + nb[k]] (sentinel included), its rows' offsets are
// off + k * off_stride (int32, relative) and its edges col + ebase[k]; rows
// write partial sums into ps[k * n + v].  Single mode: class 0 only, and rows
// are finished as in the degree-bin gather.
struct RowsArgs {
  const RowBlk *rb;
  int64_t rb_base[8];
  int64_t nb[8];
  const void *off;
  int64_t off_stride;
  int64_t ebase[8];
  const int32_t *col;
  const int32_t *lr_b0, *lr_nch;
  const int64_t *lr_pos;
  double *chunk_part;
  double *long_part;
  int32_t nlr;
  int32_t nnz;
  int32_t lds_verts;
  const float *c_in;
  int64_t n;
  float *ps;
  double base, d, inv_n, iso_count;
  int32_t drop, last;
  int32_t od_rows;  // single mode: out-degree of a row = its length (symmetric whole graph)
  const double *dsum_in;
  double *dsum_out;
  double *partials;
  const int64_t *out_off;
  const int32_t *od32;      // single mode, od_rows == 0: out-degree of each row
  float *c_out;
  const int32_t *g_of_l;
  float *rank_out;
  const double *ghost;
  const int32_t *extra_deg;
};
size_t rows_lds_bytes(int32_t lds_verts, int32_t nnz, bool stage_od);
int rows_lds_limit();  // LDS bytes a workgroup may use on the current device
int rows_launch(const RowsArgs &A, bool classes, bool off32, int grid, hipStream_t s);

// The GPU partition: local ids 0..n-1 in decreasing out-degree order.
struct GpuPart {
  int64_t n = 0, m = 0;          // local vertices, local edges
  int64_t n_global = 0;          // vertices of the whole graph
  DevCSR out;                    // out-edges (local ids); weights if any
  DevCSR in;                     // in-edges (aliases `out` when symmetric)
  bool in_alias = true;
  int32_t *g_of_l = nullptr;     // local -> global id
  int32_t *l_of_g = nullptr;     // global -> local id or -1 (size V)
  BinBounds out_bins{};          // out-degree bins over local ids
  BinBounds in_bins{};           // in-degree bins as positions in decreasing in-degree order (symmetric whole graph: out_bins)
  int64_t n_dangling = 0;        // vertices with out-degree 0
  int32_t max_w = 0;             // largest edge weight (weighted partitions)
  // SSSP light/heavy split at split_delta (packed rows only): per vertex the
  // number of out-edges lighter than it and the rest, and degree bins for the
  // light parts
  int32_t *lcnt = nullptr, *hcnt = nullptr;
  int64_t split_delta = 0;
  BinBounds light_bins{};
  int64_t n_isolated = 0;        // out-degree 0 and in-degree 0 (ZERO bin of in_bins when symmetric)
  int64_t max_out_hubs = 0;      // vertices in the HUB bin (out-degree)
  int32_t *in_off32 = nullptr;   // in-edge offsets as int32 when m < 2^31 (the bottom-up BFS step), else null
  int32_t *in_head = nullptr;    // 4 per vertex: its first four in-neighbours, -1 past the row (bottom-up BFS)
  bool mapped_edges = false;     // edge arrays (col, w; in-edge col) in mapped host memory (fixed at build)
  std::vector<int64_t> h_out_off;  // host copy of the local out offsets
  std::vector<int64_t> h_deg;      // out-degree of each local id (non-increasing)
  std::vector<int64_t> h_in_deg;   // in-degree of each local id
  PrSlices *slices = nullptr;      // PageRank in-edges split by source class (lazy)
  PrRows *rows = nullptr;          // PageRank row blocks of the in-edges (lazy)
  SsspSlices *sslices = nullptr;   // SSSP out-edges split by destination class (lazy)
  SsspPull *spull = nullptr;       // SSSP in-edges by source class, row blocks (lazy; pull supersteps)
};

// Per-partition scratch, grown on demand.
struct Workspace {
  DevArena arena;
  int64_t cap_n = -1;
  int64_t nwords = 0;            // bitmap words, padded to a multiple of 1024
  uint32_t *bits_a = nullptr, *bits_b = nullptr, *bits_c = nullptr;
  int32_t *queue = nullptr;      // n entries (BC: all levels back to back)
  int32_t *state = nullptr;      // levels / distances (n)
  int32_t *settled = nullptr;    // SSSP: distance each vertex last relaxed with (n)
  float *cbuf[2] = {nullptr, nullptr};
  double *sigma = nullptr;       // BC path counts (n)
  float *delta = nullptr;        // BC dependencies (n)
  double *bc_acc = nullptr;      // BC scores accumulated over sources (n)
  double *partials = nullptr;    // per-block partial sums
  double *hub_partials = nullptr;  // per-hub-chunk partial sums
  double *hub_dangling = nullptr;
  double *scalars = nullptr;     // small fp64 cells (dangling sums, ...)
  uint32_t *counters = nullptr;  // small counters and flags (zeroed)
  // per-call counters, STAT_COUNTERS of them, each spread over STAT_SLOTS
  // slots (stat_counter / stat_add): 0 edges scanned or relaxations, 1
  // vertices expanded or activations, 2 bottom-up edges checked, 3
  // bottom-up steps, 4 the BFS frontier's out-degree sum, 5 and 6 the
  // near/far SSSP vertices left beyond the threshold and their least
  // distance (BFS: 5 = vertices a bottom-up step examined)
  unsigned long long *work = nullptr;
  unsigned long long *h_work = nullptr;  // small pinned scratch
  unsigned long long *h_stat = nullptr;  // pinned mirror of `work`
  uint32_t *bcount = nullptr;    // per-block counts for compaction
  Plan *plan = nullptr;          // device frontier plan
  int64_t *hubpref = nullptr;    // frontier hub chunk prefix
  Plan *h_plan = nullptr;        // pinned host copy of the plan
  uint32_t *h_flags = nullptr;   // pinned host flags
  int32_t *fd = nullptr;         // SSSP pull steps: frontier distances (n), allocated on first use
  uint32_t *pull_part = nullptr; // SSSP pull steps: least candidate per chunk block, allocated on first use
  uint32_t *buckets = nullptr;   // SSSP near/far: a ring of bucket bitmaps (nwords each), allocated on first use
  int32_t buckets_k = 0;         // bitmaps in the ring
  int64_t pull_part_cap = 0;
  tgk::BfsCtl *ctl = nullptr;    // device-resident BFS control block
  tgk::BfsCtl *h_ctl = nullptr;  // pinned host copy of it (read once per chunk of supersteps)
  int64_t hub_chunks_cap = 0;
  int64_t hubs_cap = 0;
  int64_t partials_cap = 0;
  // captured chunks of device-resident BFS supersteps (k supersteps each),
  // valid for this workspace's buffers (gen) and one tuning of the partition
  struct GraphChunk {
    int k;
    uint64_t tune_gen, gen;
    hipGraphExec_t exec;
  };
  std::vector<GraphChunk> graphs;
  uint64_t gen = 0;  // bumped whenever the buffers are reallocated
  void drop_graphs();
  int ensure(const GpuPart &g, int64_t hub_chunks_needed);
  // Point the buffers a device-resident BFS uses into caller-owned device
  // memory [base, base + bytes) instead of allocating them; the other
  // buffers stay null.  TG_ENOMEM (with the size needed) if it does not fit.
  int bind_bfs(const GpuPart &g, void *base, size_t bytes);
  ~Workspace();
};

// Spread counters (see `work`): zero counter k (or all), copy it to h_stat
// (asynchronously on s), and sum its slots on the host after a wait.
int stat_zero(Workspace &ws, int k, hipStream_t s);
int stat_zero_all(Workspace &ws, hipStream_t s);
int stat_fetch(Workspace &ws, int k, hipStream_t s);
unsigned long long stat_sum(const Workspace &ws, int k);

struct HybridState;
struct SlotEngine;
struct BcBatchState;
constexpr int MAX_LANES = 8;  // searches in flight of one multi-root call
constexpr int MAX_BFS_LANES = 4;  // BFS searches in flight (within MAX_LANES)
// BFS searches in flight for nr roots under tuning t.
inline int bfs_lane_count(const Tuning &t, int64_t nr) {
  int64_t n = t.bfs_lanes < nr ? t.bfs_lanes : nr;
  if (n > MAX_BFS_LANES) n = MAX_BFS_LANES;
  return n < 1 ? 1 : (int)n;
}

}  // namespace tg

struct tg_partition {
  const tg_graph *g = nullptr;
  int strategy = TG_PART_HIGH;
  double alpha = 0.0;
  int device = 0;
  tg::Tuning tune{};
  uint64_t tune_gen = 0;  // bumped by every (re)tuning: captured launches depend on it
  std::string tuning_source = "built-in";  // "caller", "built-in" or "cache <key>"
  tg::DevArena arena;
  tg::HostMappedArena mapped;     // edge arrays kept in host memory (mapped_edges)
  tg::GpuPart gpu;
  tg::Workspace ws;
  // lanes 1.. of the multi-search drivers (BFS, SSSP): a workspace and a
  // stream (default priority) each, created on first use
  std::unique_ptr<tg::Workspace> lane_ws[tg::MAX_LANES - 1];
  hipStream_t lane_stream[tg::MAX_LANES - 1] = {};
  hipStream_t graph_stream[tg::MAX_LANES] = {};  // lanes of a BFS replaying captured chunks (capture needs an own stream)
  std::vector<int32_t> h_l_of_g;  // global -> GPU-local id (or -1)
  std::vector<int32_t> h_g_of_l;  // GPU-local -> global id
  tg::HybridState *hy = nullptr;  // host partition + boundary buffers (cpu_edge_share > 0)
  tg::SlotEngine *slots[2] = {nullptr, nullptr};  // batched BFS / SSSP engines (lazy)
  tg::BcBatchState *bcb = nullptr;                 // batched BC scratch (lazy)
};

namespace tg {

// --------------------------------------------------------- kernel launchers
// frontier.hip
int frontier_init_bitmaps(Workspace &ws, hipStream_t s);
// Compact a bitmap into a sorted queue + plan.  mode 0 (BFS): new = bits & ~prev,
// prev |= new.  mode 1 (active set): new = bits, bits cleared.  mode 2: as 1,
// and prev := the bits taken (membership of the current frontier).  If `level` is
// non-null, level[v] = level_value for every new vertex.
int frontier_compact(const GpuPart &g, Workspace &ws, int mode, uint32_t *bits, uint32_t *prev,
                     int32_t *queue, int32_t *level, int32_t level_value, hipStream_t s);
// Turn the compaction result (in ws.plan) into virtual-block offsets and the
// hub chunk prefix, then copy the plan to ws.h_plan and wait for it.
int frontier_plan(const GpuPart &g, Workspace &ws, const int32_t *queue, const Tuning &t,
                  hipStream_t s, bool sync);
// SSSP compaction of the active bitmap: a vertex is taken if dist < settled
// (it really got lower since it last relaxed; settled := dist when taken) and,
// with `near`, dist < thresh; stale bits are dropped; with `near` the others
// stay active and spread counters 5 and 6 get their count and least
// distance.
// With `degsum`, the taken frontier's out-degree sum is added to it; with
// `members`, the taken bits are also ORed into that bitmap; with `lcnt`,
// taken vertices with no light edge (lcnt[v] == 0) are left out of the
// queue (they are still taken, and still ORed into `members`).
int frontier_compact_sssp(const GpuPart &g, Workspace &ws, uint32_t *bits, int32_t *queue, const int32_t *dist,
                          int32_t *settled, int32_t thresh, bool near, const BinBounds &bb, hipStream_t s,
                          unsigned long long *degsum = nullptr, uint32_t *members = nullptr,
                          const int32_t *lcnt = nullptr);
// The end of an SSSP bucket (light/heavy split): with `pull` false, the
// bucket's members (bitmap `members`, left as it is) go to the queue and
// their out-degree sum is added to `degsum`; with `pull` true, the vertices
// with out-edges in neither `members` nor `done` (those whose distance is
// not yet final and that have edges to pull over) go to the queue.  Either
// queue is sorted by id and binned by out_bins.
int frontier_compact_bucket_end(const GpuPart &g, Workspace &ws, uint32_t *members, uint32_t *done, bool pull,
                                int32_t *queue, unsigned long long *degsum, hipStream_t s);
// done |= members, members := 0 (ws.nwords words each).
int bitmap_merge_clear(Workspace &ws, uint32_t *done, uint32_t *members, hipStream_t s);
// Plan over the queue with bins `bb` (queue positions set by a compaction
// with the same bins) and hub chunks sized by len[v] edges.
int frontier_plan_bins(const GpuPart &g, Workspace &ws, const int32_t *queue, const BinBounds &bb,
                       const int32_t *len, const Tuning &t, hipStream_t s, bool sync);
// As frontier_plan, with hub chunks sized by the degrees in `off`; with
// include_zero, frontier vertices of out-degree 0 get virtual blocks too
// (a pull over in-edges must visit them).
int frontier_plan_off(const GpuPart &g, Workspace &ws, const int32_t *queue, const int64_t *off,
                      const Tuning &t, hipStream_t s, bool sync, bool include_zero = false);
// Device-resident BFS (ws.ctl): start a search from local vertex `root`
// (control block, degree-sum slots, the root's visited bit; the bitmaps must
// be clear); the compaction of a superstep (visited ws.bits_a, previous
// ws.bits_b, frontier bitmap ws.bits_c, levels ws.state, level and degree
// counting from the control block); and the plan + direction decision.
int bfs_dev_start(const GpuPart &g, Workspace &ws, int32_t root, hipStream_t s);
int frontier_compact_bfs_dev(const GpuPart &g, Workspace &ws, const Tuning &t, hipStream_t s);
int frontier_plan_bfs_dev(const GpuPart &g, Workspace &ws, const Tuning &t, hipStream_t s);
// Before the compaction of superstep L of a search fed from outside the
// partition: reactivate the control block if its own frontier ran empty,
// and set its level to L.  (`root` < 0 in bfs_dev_start: no local root.)
int bfs_dev_resume(Workspace &ws, int32_t L, hipStream_t s);
// bfs.hip: one device-resident superstep's expansion (no plan, no compaction)
int bfs_dev_step(const GpuPart &g, Workspace &ws, const Tuning &t, hipStream_t s, bool timed);
int launch_grid(int64_t vblocks);
// bfs.hip: expansion of the frontier in `queue` (plan in ws.plan) into ws.bits_a
int bfs_expand_launch(const GpuPart &g, Workspace &ws, const int32_t *queue, int64_t vblocks,
                      const Tuning &t, hipStream_t s);
int set_bit(uint32_t *bits, int32_t v, hipStream_t s);

void sssp_slices_free(GpuPart &g);
// sssp.hip: relaxation of the frontier in `queue` (dist in ws.state, next
// active set in ws.bits_a, or with bucket_k > 0 in bitmap
// (d / bucket_delta) mod bucket_k of the ring ws.buckets; overflow marks in
// ws.bits_c).  range 1 / 2: only the light / heavy part of each row (the
// packed rows, split at p->gpu.split_delta)
int sssp_relax_launch(const GpuPart &g, Workspace &ws, const int32_t *queue, int64_t vblocks, const Tuning &t,
                      hipStream_t s, int32_t bucket_delta = 0, int32_t bucket_k = 0, int range = 0);
int sssp_overflow_check(const GpuPart &g, Workspace &ws, hipStream_t s);
// sssp_pull.hip: one superstep in the pull direction for the frontier whose
// members are the set bits of `taken` (distances in ws.state, next active set
// in ws.bits_a, overflow marks in ws.bits_c); only where supported.
bool sssp_pull_supported(const GpuPart &g);
int sssp_pull_prepare(tg_partition *p, hipStream_t s);  // builds the pull layout once
int sssp_pull_launch(tg_partition *p, Workspace &ws, const uint32_t *taken, hipStream_t s);
void sssp_pull_free(GpuPart &g);

// collect.hip
int collect_levels(const GpuPart &g, const uint32_t *visited, const int32_t *level, int32_t *out,
                   hipStream_t s);
int collect_i32(const GpuPart &g, const int32_t *state, int32_t *out, hipStream_t s);
int collect_f64_to_f32(const GpuPart &g, const double *state, float *out, hipStream_t s);
int fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
int fill_f64(double *p, int64_t n, double v, hipStream_t s);
int fill_f32(float *p, int64_t n, float v, hipStream_t s);
int bfs_parents(const GpuPart &g, const uint32_t *visited, const int32_t *level, int32_t root_local,
                int32_t *out, hipStream_t s);

// api.cpp: derive bins and plans of p->gpu from a tuning
int apply_tuning(tg_partition *p, const Tuning &t);

// pagerank.hip
int pr_init_contrib(const GpuPart &g, float *c, double N, hipStream_t s, const int32_t *extra_deg = nullptr);
int gpu_pagerank_setup(tg_partition *p, double damping, int mode, hipStream_t s, const int32_t *extra_deg,
                       double d0);
int gpu_pagerank_step(tg_partition *p, double damping, int mode, int32_t k, bool last, float *rank_out,
                      hipStream_t s, const double *ghost, const int32_t *extra_deg);
// pr_sliced.hip: the same step through the per-XCD source classes
int gpu_pagerank_sliced_step(tg_partition *p, double damping, int mode, int32_t k, bool last, float *rank_out,
                             hipStream_t s);
void pr_slices_free(GpuPart &g);
// pr_rows.hip: the step over row blocks of the in-edges
int gpu_pagerank_rows_step(tg_partition *p, double damping, int mode, int32_t k, bool last, float *rank_out,
                           hipStream_t s, const double *ghost, const int32_t *extra_deg);
void pr_rows_free(GpuPart &g);
int pr_write_initial(const GpuPart &g, float *rank_out, double N, hipStream_t s);

// algorithms (GPU partition only)
// Lane i of a multi-search call: its workspace (lane 0: p->ws) and stream
// (lane 0: the caller's s), created on first use.
int lane_workspace(tg_partition *p, int i, Workspace **out);
int lane_stream(tg_partition *p, int i, hipStream_t s, hipStream_t *out);
int graph_stream(tg_partition *p, int i, hipStream_t *out);
// BFS from each local root; levels (and parents, if non-null) of root r go
// to row r of the outputs (original ids, V per row).  *supersteps gets the
// superstep count summed over the roots.
int gpu_bfs_roots(tg_partition *p, const int32_t *roots_local, int32_t nr, int32_t *levels, int32_t *parents,
                  hipStream_t s, int64_t *supersteps);
// The same searches on one workspace the caller bound (Workspace::bind_bfs),
// one root after another on s, with no allocation of any kind: the control
// block is read back into *host_ctl.  Roots are original ids.
int gpu_bfs_roots_bound(tg_partition *p, Workspace &ws, const int32_t *roots, int32_t nr, int32_t *levels,
                        hipStream_t s, tgk::BfsCtl *host_ctl);
// Device bytes Workspace::bind_bfs needs for partition g.
size_t bfs_scratch_bytes(const GpuPart &g);
// SSSP from local root on workspace ws (distances left in ws.state).
int gpu_sssp(tg_partition *p, Workspace &ws, int32_t root_local, hipStream_t s, int64_t *rounds_out,
             int64_t *pulls_out = nullptr);
// Per-partition layouts the SSSP schedules read (light counts and bins of
// the split, pull and per-XCD layouts when enabled); built once, before
// several searches share the partition.
int sssp_prepare(tg_partition *p, hipStream_t s);
// SSSP from each local root, row r of dist (original ids, V per row), with
// up to tune.sssp_lanes searches in flight (a host thread, workspace and
// stream each); *rounds and *pulls get the superstep counts summed over the
// roots.  On error the first failing search's status is returned.
int gpu_sssp_roots(tg_partition *p, const int32_t *roots_local, int32_t nr, int32_t *dist, hipStream_t s,
                   int64_t *rounds, int64_t *pulls);
int gpu_pagerank(tg_partition *p, double damping, int32_t iters, int mode, float *rank_out,
                 hipStream_t s);
int gpu_bc_source(tg_partition *p, int32_t src_local, hipStream_t s);
// cc.hip: component labels (original ids) into ws.state
int gpu_cc(tg_partition *p, hipStream_t s, int64_t *rounds_out);
// bcb.hip: adds the dependencies of `sources` (original ids) into ws.bc_acc
int gpu_bc_batched(tg_partition *p, const int32_t *sources, int32_t ns, hipStream_t s);
void bcb_free(tg_partition *p);

}  // namespace tg

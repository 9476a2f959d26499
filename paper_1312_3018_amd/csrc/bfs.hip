// BFS superstep (section 6.3.2, Figure 11): every frontier vertex at level L
// marks its unvisited neighbours in the visited bitmap.  The new frontier is
// the set of bits that turned on during the superstep; the compaction kernel
// turns it into the next (sorted, degree-binned) queue and writes level L+1.
// A superstep ends when the new frontier is empty (the termination vote of
// section 4.1).
//
// Direction optimisation (the bottom-up step the paper's BFS leaves for
// later work): when the frontier's edges outnumber the unexplored edges by a
// factor (m_f > m_u / alpha), a superstep instead lets every unvisited vertex
// look through its in-neighbours for one in the frontier bitmap and stop at
// the first; it returns to top-down steps once the frontier is small again
// (n_f < n / beta).  Both directions produce the same levels.
#include <algorithm>

#include "tg_internal.h"

using namespace tgk;

namespace {

__global__ void k_set_bit(uint32_t *bits, int32_t v) {
  if (threadIdx.x == 0) atomicOr(bits + (v >> 5), 1u << (v & 31));
}

// Test-then-set on the visited bitmap.  A plain load filters out neighbours
// already visited before this superstep (stale reads only cost a redundant
// atomic); the atomic OR is the arbiter.  No return value is needed: the
// compaction derives the new frontier from the bitmap.  The bitmap words of
// the hottest vertices (lowest local ids) are tested against a per-block LDS
// snapshot taken at launch: a bit set there was set before, so the test
// never reports "visited" wrongly.
__device__ __forceinline__ const uint32_t *word_ptr(const uint32_t *visited, const uint32_t *lds_bits,
                                                    int32_t hot_words, int32_t nb) {
  const int32_t wi = nb >> 5;
  // a generic pointer: one load instruction serves both the LDS and the
  // global case, so the loads of several neighbours stay in flight together
  return wi < hot_words ? lds_bits + wi : visited + wi;
}

__device__ __forceinline__ void mark(uint32_t *visited, uint32_t *lds_bits, int32_t hot_words, int32_t nb,
                                     uint32_t word) {
  const uint32_t bit = 1u << (nb & 31);
  if ((word & bit) == 0) {
    const int32_t wi = nb >> 5;
    atomicOr(visited + wi, bit);
    if (wi < hot_words) atomicOr(lds_bits + wi, bit);
  }
}

// Top-down expansion of the frontier in `queue` (plan P, already in LDS):
// every frontier vertex marks its out-neighbours in `visited`.  Virtual
// blocks blk, blk + nblk, ...
__device__ __forceinline__ void expand_body(const Plan &P, const int32_t *__restrict__ queue,
                                            const int64_t *__restrict__ hubpref, const int64_t *__restrict__ off,
                                            const int32_t *__restrict__ col, uint32_t *visited, uint32_t *lds_bits,
                                            int32_t hot_words, int64_t hub_chunk, int64_t blk, int64_t nblk,
                                            unsigned long long &n_edges, unsigned long long &n_verts) {
  const int64_t total = P.vb[NBIN];
  for (int64_t vb = blk; vb < total; vb += nblk) {
    const Assign a = assign_work(vb, P, queue, nullptr, hubpref, off, hub_chunk);
    if (!a.ok) continue;
    if (a.lane == 0) {
      n_edges += (unsigned long long)(a.e_end - a.e_begin);
      n_verts += (a.bin != BIN_HUB || a.e_begin == off[a.v]) ? 1 : 0;
    }
    const int64_t st = a.stride;
    int64_t e = a.e_begin + a.lane;
    // four independent edge loads in flight per lane
    for (; e + 3 * st < a.e_end; e += 4 * st) {
      const int32_t n0 = stream_load(col + e), n1 = stream_load(col + e + st);
      const int32_t n2 = stream_load(col + e + 2 * st), n3 = stream_load(col + e + 3 * st);
      const uint32_t w0 = *word_ptr(visited, lds_bits, hot_words, n0);
      const uint32_t w1 = *word_ptr(visited, lds_bits, hot_words, n1);
      const uint32_t w2 = *word_ptr(visited, lds_bits, hot_words, n2);
      const uint32_t w3 = *word_ptr(visited, lds_bits, hot_words, n3);
      mark(visited, lds_bits, hot_words, n0, w0);
      mark(visited, lds_bits, hot_words, n1, w1);
      mark(visited, lds_bits, hot_words, n2, w2);
      mark(visited, lds_bits, hot_words, n3, w3);
    }
    for (; e < a.e_end; e += st) {
      const int32_t n0 = stream_load(col + e);
      mark(visited, lds_bits, hot_words, n0, *word_ptr(visited, lds_bits, hot_words, n0));
    }
  }
}

__global__ __launch_bounds__(BLOCK) void k_bfs_expand(const Plan *__restrict__ Pp,
                                                      const int32_t *__restrict__ queue,
                                                      const int64_t *__restrict__ hubpref,
                                                      const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ col,
                                                      uint32_t *visited, int64_t hub_chunk,
                                                      unsigned long long *work, int32_t hot_words) {
  extern __shared__ uint32_t lds_bits[];
  for (int32_t i = threadIdx.x; i < hot_words; i += BLOCK) lds_bits[i] = visited[i];
  const Plan &P = load_plan(Pp);  // (its barrier also publishes lds_bits)
  unsigned long long n_edges = 0, n_verts = 0;
  expand_body(P, queue, hubpref, off, col, visited, lds_bits, hot_words, hub_chunk, blockIdx.x, gridDim.x, n_edges,
              n_verts);
  n_edges = block_sum(n_edges);
  n_verts = block_sum(n_verts);
  if (threadIdx.x == 0 && n_edges + n_verts > 0) {
    stat_add(stat_counter(work, 0), n_edges);
    stat_add(stat_counter(work, 1), n_verts);
  }
}

// Out-degree of a vertex that joins the next frontier: from the in-edge
// offsets already loaded when in- and out-edges are the same (`ooff` null),
// else from the out-edge offsets.
__device__ __forceinline__ unsigned long long joined_degree(const int64_t *ooff, int64_t v, int64_t e0, int64_t e1) {
  return (unsigned long long)(ooff ? ooff[v + 1] - ooff[v] : e1 - e0);
}

// A vertex that joins in a bottom-up step writes its level (by local id:
// the lanes of a wave hold consecutive vertices, so the stores coalesce).
struct LevelOut {
  int32_t *level;
  int32_t value;
  __device__ __forceinline__ void put(int32_t v) const { level[v] = value; }
};

// Bottom-up step, one thread per vertex in [v0, v1): an unvisited vertex
// looks at its in-neighbours four at a time and joins the next frontier at
// the first one found in `fbits` (the level-L set).  The first four come
// from `head` (one 16-byte load per vertex, consecutive vertices side by
// side), the rest from the in-edge rows.  The out-degrees of the
// vertices that join are summed into `joined` (the direction switch's m_f).
// Waves cover whole bitmap words (lanes 0-31 one word, 32-63 the next), so
// the joins of a word are set with one atomic instead of one per lane.
// Blocks [blk0, blk0 + nblk) of the grid share the range.
template <typename OffT>
__device__ __forceinline__ void bottom_up_threads(const OffT *__restrict__ ioff, const int32_t *__restrict__ icol,
                                                  const int4 *__restrict__ head,
                                                  const uint32_t *__restrict__ fbits, uint32_t *visited, int64_t v0,
                                                  int64_t v1, const int64_t *__restrict__ ooff, int64_t blk,
                                                  int64_t nblk, const LevelOut &lo, unsigned long long &checked,
                                                  unsigned long long &joined, unsigned long long &examined) {
  const int lane = threadIdx.x & 63;
  const int64_t start = v0 & ~(int64_t)31;
  for (int64_t vb = start + blk * BLOCK; vb < v1; vb += nblk * BLOCK) {
    const int64_t v = vb + threadIdx.x;
    bool joins = false;
    if (v >= v0 && v < v1 && !(visited[v >> 5] & (1u << (v & 31)))) {
      ++examined;
      const int64_t e0 = (int64_t)ioff[v], e1 = (int64_t)ioff[v + 1];
      bool hhit = false;
      if (head) {
        const int4 h = head[v];
        const int32_t hu[4] = {h.x, h.y, h.z, h.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) hhit |= hu[k] >= 0 && ((fbits[hu[k] >> 5] >> (hu[k] & 31)) & 1u);
        checked += (unsigned long long)(e1 - e0 < 4 ? e1 - e0 : 4);
        if (hhit) {
          joins = true;
          joined += joined_degree(ooff, v, e0, e1);
          lo.put((int32_t)v);
        }
      }
      for (int64_t e = e0 + (head ? 4 : 0); !hhit && e < e1; e += 4) {
        int32_t u[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) u[k] = icol[e + k < e1 ? e + k : e1 - 1];
        bool hit = false;
#pragma unroll
        for (int k = 0; k < 4; ++k) hit |= (e + k < e1) && ((fbits[u[k] >> 5] >> (u[k] & 31)) & 1u);
        checked += (unsigned long long)(e1 - e < 4 ? e1 - e : 4);
        if (hit) {
          joins = true;
          joined += joined_degree(ooff, v, e0, e1);
          lo.put((int32_t)v);
          break;
        }
      }
    }
    const uint64_t m = __ballot(joins);
    if (lane == 0 && (uint32_t)m) atomicOr(visited + (v >> 5), (uint32_t)m);
    if (lane == 32 && (uint32_t)(m >> 32)) atomicOr(visited + (v >> 5), (uint32_t)(m >> 32));
  }
}

// The same with one wave per vertex in [v0, v1) (high in-degree): the wave
// checks 64 in-neighbours per round and stops at the first round with a hit.
template <typename OffT>
__device__ __forceinline__ void bottom_up_waves(const OffT *__restrict__ ioff, const int32_t *__restrict__ icol,
                                                const uint32_t *__restrict__ fbits, uint32_t *visited, int64_t v0,
                                                int64_t v1, const int64_t *__restrict__ ooff, int64_t blk,
                                                int64_t nblk, const LevelOut &lo, unsigned long long &checked,
                                                unsigned long long &joined, unsigned long long &examined) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (nblk * BLOCK) >> 6;
  for (int64_t v = v0 + ((blk * BLOCK + threadIdx.x) >> 6); v < v1; v += nw) {
    const uint32_t bit = 1u << (v & 31);
    if (visited[v >> 5] & bit) continue;
    if (lane == 0) ++examined;
    const int64_t e0 = (int64_t)ioff[v], e1 = (int64_t)ioff[v + 1];
    for (int64_t e = e0; e < e1; e += 64) {
      const bool live = e + lane < e1;
      const int32_t u = live ? icol[e + lane] : 0;
      const bool hit = live && ((fbits[u >> 5] >> (u & 31)) & 1u);
      if (lane == 0) checked += (unsigned long long)(e1 - e < 64 ? e1 - e : 64);
      if (__ballot(hit)) {
        if (lane == 0) {
          atomicOr(visited + (v >> 5), bit);
          joined += joined_degree(ooff, v, e0, e1);
          lo.put((int32_t)v);
        }
        break;
      }
    }
  }
}

// One device-resident superstep's expansion, in the direction the control
// block holds.  Top-down: every block walks the frontier queue's virtual
// blocks.  Bottom-up: blocks [0, wave_blocks) give a wave to each vertex of
// [0, wave_end), the others a thread to each vertex of [wave_end, n_end),
// and each vertex that joins writes its level.
template <typename OffT>
__global__ __launch_bounds__(BLOCK) void k_bfs_step(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                    const int64_t *__restrict__ hubpref,
                                                    const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                    uint32_t *visited, int64_t hub_chunk, unsigned long long *work,
                                                    const OffT *__restrict__ ioff, const int32_t *__restrict__ icol,
                                                    const int4 *__restrict__ head,
                                                    const uint32_t *__restrict__ fbits, int64_t wave_end,
                                                    int64_t n_end, int64_t wave_blocks,
                                                    const int64_t *__restrict__ ooff, unsigned long long *degsum,
                                                    int32_t *level, const BfsCtl *__restrict__ ctl) {
  if (!ctl->active) return;
  if (!ctl->bottom_up) {
    const Plan &P = load_plan(Pp);
    unsigned long long n_edges = 0, n_verts = 0;
    expand_body(P, queue, hubpref, off, col, visited, nullptr, 0, hub_chunk, blockIdx.x, gridDim.x, n_edges,
                n_verts);
    n_edges = block_sum(n_edges);
    n_verts = block_sum(n_verts);
    if (threadIdx.x == 0 && n_edges + n_verts > 0) {
      stat_add(stat_counter(work, 0), n_edges);
      stat_add(stat_counter(work, 1), n_verts);
    }
    return;
  }
  const LevelOut lo{level, ctl->L + 1};
  unsigned long long checked = 0, joined = 0, examined = 0;
  if ((int64_t)blockIdx.x < wave_blocks)
    bottom_up_waves(ioff, icol, fbits, visited, 0, wave_end, ooff, blockIdx.x, wave_blocks, lo, checked, joined,
                    examined);
  else
    bottom_up_threads(ioff, icol, head, fbits, visited, wave_end, n_end, ooff, blockIdx.x - wave_blocks,
                      gridDim.x - wave_blocks, lo, checked, joined, examined);
  checked = block_sum(checked);
  joined = block_sum(joined);
  examined = block_sum(examined);
  if (threadIdx.x == 0 && checked) stat_add(stat_counter(work, 2), checked);
  if (threadIdx.x == 0 && examined) stat_add(stat_counter(work, 5), examined);
  if (threadIdx.x == 0 && joined) stat_add(degsum, joined);
}

}  // namespace

namespace tg {

int set_bit(uint32_t *bits, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_bit, dim3(1), dim3(64), 0, s, bits, v);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int bfs_expand_launch(const GpuPart &g, Workspace &ws, const int32_t *queue, int64_t vblocks,
                      const Tuning &t, hipStream_t s) {
  if (vblocks <= 0) return TG_OK;
  // large frontiers: a bounded grid stages the hottest bitmap words in LDS
  // once per block; small frontiers skip the staging
  const bool stage = vblocks >= t.bfs_lds_min_vblocks;
  const int32_t hot_words = stage ? (int32_t)std::min<int64_t>(t.bfs_lds_words, (g.n + 31) / 32) : 0;
  const int grid = stage ? (int)std::min<int64_t>(launch_grid(vblocks), t.bfs_grid) : launch_grid(vblocks);
  const int tk = ktimer_start(s);
  hipLaunchKernelGGL(k_bfs_expand, dim3(grid), dim3(BLOCK), (size_t)hot_words * sizeof(uint32_t), s, ws.plan,
                     queue, ws.hubpref, g.out.off, g.out.col, ws.bits_a, t.hub_chunk, ws.work, hot_words);
  ktimer_stop(tk, s, "bfs_expand");
  TG_HIP(hipGetLastError());
  return TG_OK;
}

namespace {

}  // namespace

// The expansion of one device-resident superstep (k_bfs_step in the
// direction the control block holds), without the plan and the compaction.
int bfs_dev_step(const GpuPart &g, Workspace &ws, const Tuning &t, hipStream_t s, bool timed) {
  // vertices with in-edges: a symmetric whole graph ends them at its
  // degree-0 tail and has its in-degrees sorted, so its head (HUB and BLOCK
  // bins) gets a wave per vertex; most vertices find a parent among their
  // first few in-neighbours, so everything else takes a thread each
  const int64_t n_end = g.in_alias ? g.out_bins.bstart[BIN_ZERO] : g.n;
  const int64_t wave_end = g.in_alias ? g.out_bins.bstart[BIN_WAVE] : 0;
  const int64_t wave_blocks = (t.bfs_do && wave_end > 0) ? std::max<int64_t>(t.bfs_bu_grid / 2, 1) : 0;
  const int64_t thread_blocks = (t.bfs_do && n_end > wave_end) ? t.bfs_bu_grid : 0;
  // one launch for either direction: the top-down walk uses every block of
  // the grid (the frontier size lives on the device, so the grid is fixed)
  const unsigned grid = (unsigned)std::max<int64_t>(t.bfs_td_grid, wave_blocks + thread_blocks);
  // the joining vertices' out-degrees: in-edge rows are out-edge rows on a
  // symmetric whole graph
  const int64_t *ooff = g.in_alias ? nullptr : g.out.off;
  const int tk = timed ? ktimer_start(s) : -1;
  if (g.in_off32)
    hipLaunchKernelGGL(k_bfs_step<int32_t>, dim3(grid), dim3(BLOCK), 0, s, ws.plan, ws.queue, ws.hubpref, g.out.off,
                       g.out.col, ws.bits_a, t.hub_chunk, ws.work, g.in_off32, g.in.col,
                       reinterpret_cast<const int4 *>(g.in_head), ws.bits_c, wave_end, n_end,
                       wave_blocks, ooff, stat_counter(ws.work, 4), ws.state, ws.ctl);
  else
    hipLaunchKernelGGL(k_bfs_step<int64_t>, dim3(grid), dim3(BLOCK), 0, s, ws.plan, ws.queue, ws.hubpref, g.out.off,
                       g.out.col, ws.bits_a, t.hub_chunk, ws.work, g.in.off, g.in.col,
                       reinterpret_cast<const int4 *>(g.in_head), ws.bits_c, wave_end, n_end,
                       wave_blocks, ooff, stat_counter(ws.work, 4), ws.state, ws.ctl);
  ktimer_stop(tk, s, "bfs_step");
  TG_HIP(hipGetLastError());
  return TG_OK;
}

namespace {

// One device-resident superstep on workspace `ws`: plan and direction
// (k_plan_bfs), the top-down expansion and the bottom-up step (each exits at
// once unless the control block selects it), then the compaction of the new
// frontier.  Nothing here waits for the host.
int bfs_dev_superstep(const GpuPart &g, Workspace &ws, const Tuning &t, hipStream_t s, bool timed = true) {
  TG_TRY(frontier_plan_bfs_dev(g, ws, t, s));
  TG_TRY(bfs_dev_step(g, ws, t, s, timed));
  return frontier_compact_bfs_dev(g, ws, t, s);
}


// Enqueue k supersteps, then the read-back of the control block and `ev`.
// The k supersteps as one captured graph (captured on first use, replayed
// after): their launches take fixed pointers and read everything else from
// the device, so one capture serves every search on this workspace until
// the buffers or the tuning change.  No memory set or copy is captured.
int bfs_graph_chunk(const tg_partition *p, Workspace &ws, int k, hipStream_t s) {
  for (const Workspace::GraphChunk &c : ws.graphs)
    if (c.k == k && c.tune_gen == p->tune_gen && c.gen == ws.gen) {
      TG_HIP(hipGraphLaunch(c.exec, s));
      return TG_OK;
    }
  TG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int rc = TG_OK;
  for (int i = 0; i < k && rc == TG_OK; ++i) rc = bfs_dev_superstep(p->gpu, ws, p->tune, s, false);
  hipGraph_t gr = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &gr);
  if (rc == TG_OK && e != hipSuccess) rc = set_error(TG_EDEVICE, "bfs: capture failed: %s", hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  if (rc == TG_OK && hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) != hipSuccess)
    rc = set_error(TG_EDEVICE, "bfs: hipGraphInstantiate failed");
  if (gr) TG_QUIET(hipGraphDestroy(gr));
  if (rc != TG_OK) return rc;
  // a few chunk lengths recur (the learned first chunk, the follow-up chunk)
  if (ws.graphs.size() >= 6) {
    TG_QUIET(hipGraphExecDestroy(ws.graphs.front().exec));
    ws.graphs.erase(ws.graphs.begin());
  }
  ws.graphs.push_back({k, p->tune_gen, ws.gen, ex});
  TG_HIP(hipGraphLaunch(ex, s));
  return TG_OK;
}

// Enqueue k supersteps (eagerly, or replaying a captured chunk), then the
// read-back of the control block and `ev`.
int bfs_dev_chunk(const tg_partition *p, Workspace &ws, int k, hipStream_t s, hipEvent_t ev, bool graph) {
  if (graph) TG_TRY(bfs_graph_chunk(p, ws, k, s));
  else
    for (int i = 0; i < k; ++i) TG_TRY(bfs_dev_superstep(p->gpu, ws, p->tune, s));
  TG_HIP(hipMemcpyAsync(ws.h_ctl, ws.ctl, sizeof(BfsCtl), hipMemcpyDeviceToHost, s));
  TG_HIP(hipEventRecord(ev, s));
  return TG_OK;
}

struct BfsLane {
  Workspace *ws = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  int32_t r = -1;        // root index in flight (-1: idle)
  int64_t issued = 0;    // supersteps enqueued for it
};

}  // namespace

// Supersteps run on the device in chunks: a search starts with as many
// supersteps as the previous one needed (plus the one that finds the empty
// frontier), and the host reads the control block once per chunk, adding
// two more supersteps at a time if the search is still going.  With
// several lanes (up to four), as many searches run on streams with a
// workspace each, so one lane's read-back overlaps the others' kernels.
int gpu_bfs_roots(tg_partition *p, const int32_t *roots_local, int32_t nr, int32_t *levels, int32_t *parents,
                  hipStream_t s, int64_t *supersteps) {
  GpuPart &g = p->gpu;
  const Tuning &t = p->tune;
  const int nl = bfs_lane_count(t, nr);
  // captured chunks replay without per-kernel timing events; capture needs
  // streams of the library's own (the caller's may be the null stream)
  const bool graph = t.bfs_graph != 0 && !timing_enabled();
  BfsLane lane[MAX_BFS_LANES];
  lane[0].ws = &p->ws;
  lane[0].s = s;
  if (graph) TG_TRY(graph_stream(p, 0, &lane[0].s));
  for (int l = 1; l < nl; ++l) {
    TG_TRY(lane_workspace(p, l, &lane[l].ws));
    if (graph) TG_TRY(graph_stream(p, l, &lane[l].s));
    else TG_TRY(lane_stream(p, l, s, &lane[l].s));
  }
  const int64_t V = g.n_global;
  int rc = TG_OK;
  hipEvent_t join = nullptr;
  for (int l = 0; l < nl && rc == TG_OK; ++l) {
    rc = lane[l].ws->ensure(g, 0);
    if (rc == TG_OK && hipEventCreateWithFlags(&lane[l].ev, hipEventDisableTiming) != hipSuccess)
      rc = set_error(TG_EDEVICE, "bfs: hipEventCreate failed");
  }
  if (rc == TG_OK && hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess)
    rc = set_error(TG_EDEVICE, "bfs: hipEventCreate failed");
  // kernel timings (if on) are measured from a reference recorded on s
  // before either lane starts
  ktimer_ensure_ref(s);
  if (rc == TG_OK) {
    // lanes on streams other than s start after the caller's earlier work on s
    bool ok = hipEventRecord(join, s) == hipSuccess;
    for (int l = 0; l < nl && ok; ++l)
      if (lane[l].s != s) ok = hipStreamWaitEvent(lane[l].s, join, 0) == hipSuccess;
    if (!ok) rc = set_error(TG_EDEVICE, "bfs: stream ordering failed");
  }
  for (int l = 0; l < nl && rc == TG_OK; ++l) rc = stat_zero_all(*lane[l].ws, lane[l].s);
  int first_chunk = 4;  // supersteps of the next search's first chunk (learned)
  int32_t next = 0;
  int64_t total = 0;
  auto start = [&](BfsLane &L) -> int {
    Workspace &ws = *L.ws;
    L.r = next++;
    TG_HIP(hipMemsetAsync(ws.bits_a, 0, ws.nwords * sizeof(uint32_t), L.s));
    TG_HIP(hipMemsetAsync(ws.bits_b, 0, ws.nwords * sizeof(uint32_t), L.s));
    TG_TRY(bfs_dev_start(g, ws, roots_local[L.r], L.s));
    TG_TRY(frontier_compact_bfs_dev(g, ws, t, L.s));  // the root's frontier, level 0
    L.issued = first_chunk;
    return bfs_dev_chunk(p, ws, first_chunk, L.s, L.ev, graph);
  };
  for (int l = 0; l < nl && rc == TG_OK && next < nr; ++l) rc = start(lane[l]);
  // serve the lanes in turn until every search has ended
  for (int cur = 0; rc == TG_OK;) {
    BfsLane &L = lane[cur];
    cur = (cur + 1) % nl;
    if (L.r < 0) {
      bool busy = false;
      for (int l = 0; l < nl; ++l) busy |= lane[l].r >= 0;
      if (!busy) break;
      continue;
    }
    if (hipEventSynchronize(L.ev) != hipSuccess) {
      rc = set_error(TG_EDEVICE, "bfs: hipEventSynchronize failed");
      break;
    }
    const BfsCtl c = *L.ws->h_ctl;
    if (c.active) {
      if (L.issued > g.n + 2) {
        rc = set_error(TG_EDEVICE, "bfs: more supersteps than vertices");
        break;
      }
      L.issued += 2;
      rc = bfs_dev_chunk(p, *L.ws, 2, L.s, L.ev, graph);
      continue;
    }
    // this search has ended: collect it and start the next one on the lane
    total += c.steps + 1;
    first_chunk = std::max(c.steps + 1, 1);
    rc = collect_levels(g, L.ws->bits_a, L.ws->state, levels + (int64_t)L.r * V, L.s);
    if (rc == TG_OK && parents)
      rc = bfs_parents(g, L.ws->bits_a, L.ws->state, roots_local[L.r], parents + (int64_t)L.r * V, L.s);
    L.r = -1;
    if (rc == TG_OK && next < nr) rc = start(L);
  }
  for (int l = 0; l < nl && rc == TG_OK; ++l) {
    // the caller's stream waits for the lanes on other streams
    if (lane[l].s == s) continue;
    if (hipEventRecord(lane[l].ev, lane[l].s) != hipSuccess || hipStreamWaitEvent(s, lane[l].ev, 0) != hipSuccess)
      rc = set_error(TG_EDEVICE, "bfs: stream ordering failed");
  }
  if (rc != TG_OK) {
    // leave no work of this call running on the lanes' streams
    for (int l = 0; l < nl; ++l) TG_QUIET(hipStreamSynchronize(lane[l].s));
    TG_QUIET(hipStreamSynchronize(s));
  }
  for (int l = 0; l < nl; ++l)
    if (lane[l].ev) TG_QUIET(hipEventDestroy(lane[l].ev));
  if (join) TG_QUIET(hipEventDestroy(join));
  if (supersteps) *supersteps = total;
  return rc;
}

int gpu_bfs_roots_bound(tg_partition *p, Workspace &ws, const int32_t *roots, int32_t nr, int32_t *levels,
                        hipStream_t s, BfsCtl *host_ctl) {
  GpuPart &g = p->gpu;
  const Tuning &t = p->tune;
  const int64_t V = g.n_global;
  TG_TRY(stat_zero_all(ws, s));
  int chunk = 4;  // supersteps of a search's first chunk (learned from the previous search)
  for (int32_t r = 0; r < nr; ++r) {
    TG_HIP(hipMemsetAsync(ws.bits_a, 0, ws.nwords * sizeof(uint32_t), s));
    TG_HIP(hipMemsetAsync(ws.bits_b, 0, ws.nwords * sizeof(uint32_t), s));
    TG_TRY(bfs_dev_start(g, ws, p->h_l_of_g[roots[r]], s));
    TG_TRY(frontier_compact_bfs_dev(g, ws, t, s));  // the root's frontier, level 0
    int64_t issued = 0;
    for (int k = chunk;; k = 2) {
      for (int i = 0; i < k; ++i) TG_TRY(bfs_dev_superstep(g, ws, t, s, false));
      issued += k;
      TG_HIP(hipMemcpyAsync(host_ctl, ws.ctl, sizeof(BfsCtl), hipMemcpyDeviceToHost, s));
      TG_HIP(hipStreamSynchronize(s));
      if (!host_ctl->active) break;
      if (issued > g.n + 2) return set_error(TG_EDEVICE, "bfs: more supersteps than vertices");
    }
    chunk = std::max(host_ctl->steps + 1, 1);
    TG_TRY(collect_levels(g, ws.bits_a, ws.state, levels + (int64_t)r * V, s));
  }
  TG_HIP(hipStreamSynchronize(s));
  return TG_OK;
}

}  // namespace tg

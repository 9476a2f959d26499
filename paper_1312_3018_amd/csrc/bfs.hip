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

__global__ void k_count_step(unsigned long long *c) {
  if (threadIdx.x == 0) *c += 1ull;
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
  const int64_t total = P.vb[NBIN];
  unsigned long long n_edges = 0, n_verts = 0;
  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
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

// Bottom-up step, one thread per vertex in [v0, v1): an unvisited vertex
// looks at its in-neighbours four at a time and joins the next frontier at
// the first one found in `fbits` (the level-L set).  The out-degrees of the
// vertices that join are summed into `degsum` (the direction switch's m_f).
// Waves cover whole bitmap words (lanes 0-31 one word, 32-63 the next), so
// the joins of a word are set with one atomic instead of one per lane.
__global__ __launch_bounds__(BLOCK) void k_bfs_bottom_up_thread(const int64_t *__restrict__ ioff,
                                                                const int32_t *__restrict__ icol,
                                                                const uint32_t *__restrict__ fbits, uint32_t *visited,
                                                                int64_t v0, int64_t v1, unsigned long long *work,
                                                                const int64_t *__restrict__ ooff,
                                                                unsigned long long *degsum) {
  unsigned long long checked = 0, joined = 0;
  const int lane = threadIdx.x & 63;
  const int64_t start = v0 & ~(int64_t)31;
  for (int64_t vb = start + (int64_t)blockIdx.x * BLOCK; vb < v1; vb += (int64_t)gridDim.x * BLOCK) {
    const int64_t v = vb + threadIdx.x;
    bool joins = false;
    if (v >= v0 && v < v1 && !(visited[v >> 5] & (1u << (v & 31)))) {
      const int64_t e0 = ioff[v], e1 = ioff[v + 1];
      for (int64_t e = e0; e < e1; e += 4) {
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
          break;
        }
      }
    }
    const uint64_t m = __ballot(joins);
    if (lane == 0 && (uint32_t)m) atomicOr(visited + (v >> 5), (uint32_t)m);
    if (lane == 32 && (uint32_t)(m >> 32)) atomicOr(visited + (v >> 5), (uint32_t)(m >> 32));
  }
  checked = block_sum(checked);
  joined = block_sum(joined);
  if (threadIdx.x == 0 && checked) stat_add(work, checked);
  if (threadIdx.x == 0 && joined) stat_add(degsum, joined);
}

// The same with one wave per vertex in [v0, v1) (high in-degree): the wave
// checks 64 in-neighbours per round and stops at the first round with a hit.
__global__ __launch_bounds__(BLOCK) void k_bfs_bottom_up_wave(const int64_t *__restrict__ ioff,
                                                              const int32_t *__restrict__ icol,
                                                              const uint32_t *__restrict__ fbits, uint32_t *visited,
                                                              int64_t v0, int64_t v1, unsigned long long *work,
                                                              const int64_t *__restrict__ ooff,
                                                              unsigned long long *degsum) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * BLOCK) >> 6;
  unsigned long long checked = 0, joined = 0;
  for (int64_t v = v0 + (((int64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6); v < v1; v += nw) {
    const uint32_t bit = 1u << (v & 31);
    if (visited[v >> 5] & bit) continue;
    const int64_t e0 = ioff[v], e1 = ioff[v + 1];
    for (int64_t e = e0; e < e1; e += 64) {
      const bool live = e + lane < e1;
      const int32_t u = live ? icol[e + lane] : 0;
      const bool hit = live && ((fbits[u >> 5] >> (u & 31)) & 1u);
      if (lane == 0) checked += (unsigned long long)(e1 - e < 64 ? e1 - e : 64);
      if (__ballot(hit)) {
        if (lane == 0) {
          atomicOr(visited + (v >> 5), bit);
          joined += joined_degree(ooff, v, e0, e1);
        }
        break;
      }
    }
  }
  checked = block_sum(checked);
  joined = block_sum(joined);
  if (threadIdx.x == 0 && checked) stat_add(work, checked);
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

// One bottom-up step over the in-edges: vertices [0, wave_end) one wave each,
// [wave_end, n_end) one thread each.
static int bfs_bottom_up_launch(const GpuPart &g, Workspace &ws, const uint32_t *fbits, int64_t wave_end,
                                int64_t n_end, unsigned long long *degsum, hipStream_t s) {
  // the joining vertices' out-degrees: in-edge rows are out-edge rows on a
  // symmetric whole graph
  const int64_t *ooff = g.in_alias ? nullptr : g.out.off;
  const int tk = ktimer_start(s);
  if (wave_end > 0) {
    const int grid = (int)std::min<int64_t>((wave_end * 64 + BLOCK - 1) / BLOCK, 8192);
    hipLaunchKernelGGL(k_bfs_bottom_up_wave, dim3(grid), dim3(BLOCK), 0, s, g.in.off, g.in.col, fbits, ws.bits_a,
                       (int64_t)0, wave_end, stat_counter(ws.work, 2), ooff, degsum);
  }
  if (n_end > wave_end) {
    const int grid = (int)std::min<int64_t>((n_end - wave_end + BLOCK - 1) / BLOCK, 16384);
    hipLaunchKernelGGL(k_bfs_bottom_up_thread, dim3(grid), dim3(BLOCK), 0, s, g.in.off, g.in.col, fbits, ws.bits_a,
                       wave_end, n_end, stat_counter(ws.work, 2), ooff, degsum);
  }
  ktimer_stop(tk, s, "bfs_bottom_up");
  TG_HIP(hipGetLastError());
  return TG_OK;
}

// BFS from local vertex `root` over the GPU partition.  Leaves the visited
// bitmap in ws.bits_a and levels in ws.state (valid where visited).
int gpu_bfs(tg_partition *p, int32_t root, hipStream_t s, int64_t *levels_out) {
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  const Tuning &t = p->tune;
  TG_TRY(ws.ensure(g, 0));
  uint32_t *visited = ws.bits_a, *prev = ws.bits_b, *fbits = ws.bits_c;
  TG_HIP(hipMemsetAsync(visited, 0, ws.nwords * sizeof(uint32_t), s));
  TG_HIP(hipMemsetAsync(prev, 0, ws.nwords * sizeof(uint32_t), s));
  TG_TRY(set_bit(visited, root, s));
  unsigned long long *degsum = stat_counter(ws.work, 4);
  TG_TRY(frontier_compact_bfs(g, ws, visited, prev, fbits, ws.queue, ws.state, 0, degsum, true, s));
  // vertices with in-edges: a symmetric whole graph ends them at its
  // degree-0 tail and has its in-degrees sorted, so its head (HUB and BLOCK
  // bins) gets a wave per vertex; most vertices find a parent among their
  // first few in-neighbours, so everything else takes a thread each
  const int64_t n_end = g.in_alias ? g.out_bins.bstart[BIN_ZERO] : g.n;
  const int64_t wave_end = g.in_alias ? g.out_bins.bstart[BIN_WAVE] : 0;
  int64_t m_u = g.m;  // edges of vertices not yet in a frontier
  bool bottom_up = false;
  int32_t L = 0;
  for (;; ++L) {
    if (L > g.n) return set_error(TG_EDEVICE, "bfs: more supersteps than vertices");
    TG_TRY(frontier_plan(g, ws, ws.queue, t, s, false));
    TG_HIP(hipMemcpyAsync(ws.h_plan, ws.plan, sizeof(Plan), hipMemcpyDeviceToHost, s));
    TG_TRY(stat_fetch(ws, 4, s));
    TG_HIP(hipStreamSynchronize(s));
    ktimer_flush();
    const int64_t n_f = ws.h_plan->count;
    if (n_f == 0) break;
    const int64_t m_f = (int64_t)stat_sum(ws, 4);
    m_u -= m_f;
    if (t.bfs_do) {
      // Beamer's switch: bottom-up while the frontier is heavy, back once it is small
      if (!bottom_up && m_f > m_u / t.bfs_alpha) bottom_up = true;
      else if (bottom_up && n_f < g.n / t.bfs_beta) bottom_up = false;
    }
    if (bottom_up) {
      // the bottom-up kernels sum the new frontier's out-degrees themselves
      TG_TRY(stat_zero(ws, 4, s));
      TG_TRY(bfs_bottom_up_launch(g, ws, fbits, wave_end, n_end, degsum, s));
      hipLaunchKernelGGL(k_count_step, dim3(1), dim3(64), 0, s, stat_counter(ws.work, 3));
      TG_HIP(hipGetLastError());
    } else {
      TG_TRY(bfs_expand_launch(g, ws, ws.queue, ws.h_plan->vb[NBIN], t, s));
    }
    TG_TRY(frontier_compact_bfs(g, ws, visited, prev, fbits, ws.queue, ws.state, L + 1, degsum, !bottom_up, s));
  }
  if (levels_out) *levels_out = L;
  return TG_OK;
}

}  // namespace tg

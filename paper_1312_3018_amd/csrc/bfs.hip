// BFS superstep (section 6.3.2, Figure 11): every frontier vertex at level L
// marks its unvisited neighbours in the visited bitmap.  The new frontier is
// the set of bits that turned on during the superstep; the compaction kernel
// turns it into the next (sorted, degree-binned) queue and writes level L+1.
// A superstep ends when the new frontier is empty (the termination vote of
// section 4.1).
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
    atomicAdd(work, n_edges);
    atomicAdd(work + 1, n_verts);
  }
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

// BFS from local vertex `root` over the GPU partition.  Leaves the visited
// bitmap in ws.bits_a and levels in ws.state (valid where visited).
int gpu_bfs(tg_partition *p, int32_t root, hipStream_t s, int64_t *levels_out) {
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  TG_TRY(ws.ensure(g, 0));
  uint32_t *visited = ws.bits_a, *prev = ws.bits_b;
  TG_HIP(hipMemsetAsync(visited, 0, ws.nwords * sizeof(uint32_t), s));
  TG_HIP(hipMemsetAsync(prev, 0, ws.nwords * sizeof(uint32_t), s));
  TG_TRY(set_bit(visited, root, s));
  TG_TRY(frontier_compact(g, ws, 0, visited, prev, ws.queue, ws.state, 0, s));
  int32_t L = 0;
  for (;; ++L) {
    if (L > g.n) return set_error(TG_EDEVICE, "bfs: more supersteps than vertices");
    TG_TRY(frontier_plan(g, ws, ws.queue, p->tune, s, true));
    if (ws.h_plan->count == 0) break;
    TG_TRY(bfs_expand_launch(g, ws, ws.queue, ws.h_plan->vb[NBIN], p->tune, s));
    TG_TRY(frontier_compact(g, ws, 0, visited, prev, ws.queue, ws.state, L + 1, s));
  }
  if (levels_out) *levels_out = L;
  return TG_OK;
}

}  // namespace tg

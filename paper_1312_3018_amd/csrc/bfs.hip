// BFS superstep (section 6.3.2, Figure 11): every frontier vertex at level L
// marks its unvisited neighbours in the visited bitmap.  The new frontier is
// the set of bits that turned on during the superstep; the compaction kernel
// turns it into the next (sorted, degree-binned) queue and writes level L+1.
// A superstep ends when the new frontier is empty (the termination vote of
// section 4.1).
#include "tg_internal.h"

using namespace tgk;

namespace {

__global__ void k_set_bit(uint32_t *bits, int32_t v) {
  if (threadIdx.x == 0) atomicOr(bits + (v >> 5), 1u << (v & 31));
}

// Test-then-set on the visited bitmap.  A plain load filters out neighbours
// already visited before this superstep (stale reads only cost a redundant
// atomic); the atomic OR is the arbiter.  No return value is needed: the
// compaction derives the new frontier from the bitmap.
__device__ __forceinline__ void visit(uint32_t *visited, int32_t nb) {
  const uint32_t bit = 1u << (nb & 31);
  uint32_t *wp = visited + (nb >> 5);
  if ((*wp & bit) == 0) atomicOr(wp, bit);
}

__global__ __launch_bounds__(BLOCK) void k_bfs_expand(const Plan *__restrict__ Pp,
                                                      const int32_t *__restrict__ queue,
                                                      const int64_t *__restrict__ hubpref,
                                                      const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ col,
                                                      uint32_t *visited, int64_t hub_chunk,
                                                      unsigned long long *work) {
  const Plan P = *Pp;
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
      const int32_t n0 = col[e], n1 = col[e + st], n2 = col[e + 2 * st], n3 = col[e + 3 * st];
      visit(visited, n0);
      visit(visited, n1);
      visit(visited, n2);
      visit(visited, n3);
    }
    for (; e < a.e_end; e += st) visit(visited, col[e]);
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
  const int tk = ktimer_start(s);
  hipLaunchKernelGGL(k_bfs_expand, dim3(launch_grid(vblocks)), dim3(BLOCK), 0, s, ws.plan, queue,
                     ws.hubpref, g.out.off, g.out.col, ws.bits_a, t.hub_chunk, ws.work);
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

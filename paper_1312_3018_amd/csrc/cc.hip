// Connected components by minimum-label propagation (the fifth algorithm of
// section 9.4, run on the undirected graph; labels are reduced by minimum,
// section 3.4).  Every vertex starts with its own original id as its label;
// each superstep, every vertex whose label dropped since it last pushed sends
// it to its neighbours with an atomic minimum and marks those it may lower;
// the run ends when no label drops.  The fixed point gives each vertex the
// smallest original id of its component.  A directed graph gives its weak
// components: labels travel along out-edges and in-edges.
//
// The frontier machinery is SSSP's (frontier.hip): the active bitmap, the
// compaction's `settled` filter (a marked vertex is taken only if its label is
// below the one it last pushed), the degree-binned plan.
#include <algorithm>

#include "tg_internal.h"

using namespace tgk;

namespace {

__global__ __launch_bounds__(BLOCK) void k_cc_init(const int32_t *__restrict__ g_of_l, int64_t n,
                                                   int32_t *__restrict__ label) {
  const int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v < n) label[v] = g_of_l[v];
}

// every local vertex active
__global__ __launch_bounds__(BLOCK) void k_cc_all_active(uint32_t *__restrict__ bits, int64_t n, int64_t nwords) {
  const int64_t w = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (w >= nwords) return;
  const int64_t lo = w * 32;
  uint32_t m = 0;
  if (lo + 32 <= n) m = 0xFFFFFFFFu;
  else if (lo < n) m = (1u << (n - lo)) - 1u;
  bits[w] = m;
}

__device__ __forceinline__ void push(int32_t *label, uint32_t *active, int32_t lu, int32_t nb, int32_t cur) {
  if (lu < cur) {
    atomicMin(label + nb, lu);  // no return value: nothing waits on it
    atomicOr(active + (nb >> 5), 1u << (nb & 31));
  }
}

// One superstep over the edges in `off`/`col` of the frontier in `queue`.
__global__ __launch_bounds__(BLOCK) void k_cc_push(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                   const int64_t *__restrict__ hubpref,
                                                   const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                   int32_t *label, uint32_t *active, int64_t hub_chunk,
                                                   unsigned long long *work) {
  const Plan &P = load_plan(Pp);
  const int64_t total = P.vb[NBIN];
  unsigned long long n_edges = 0;
  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const Assign a = assign_work(vb, P, queue, nullptr, hubpref, off, hub_chunk);
    if (!a.ok) continue;
    if (a.lane == 0) n_edges += (unsigned long long)(a.e_end - a.e_begin);
    const int32_t lu = label[a.v];
    const int64_t st = a.stride;
    int64_t e = a.e_begin + a.lane;
    for (; e + 3 * st < a.e_end; e += 4 * st) {
      int32_t nb[4], cur[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) nb[q] = stream_load(col + e + q * st);
#pragma unroll
      for (int q = 0; q < 4; ++q) cur[q] = label[nb[q]];
#pragma unroll
      for (int q = 0; q < 4; ++q) push(label, active, lu, nb[q], cur[q]);
    }
    for (; e < a.e_end; e += st) {
      const int32_t n0 = stream_load(col + e);
      push(label, active, lu, n0, label[n0]);
    }
  }
  n_edges = block_sum(n_edges);
  if (threadIdx.x == 0 && n_edges > 0) stat_add(work, n_edges);
}

}  // namespace

namespace tg {

static int cc_push_launch(const GpuPart &g, Workspace &ws, const int64_t *off, const int32_t *col, int64_t vblocks,
                          const Tuning &t, hipStream_t s) {
  if (vblocks <= 0) return TG_OK;
  const int tk = ktimer_start(s);
  hipLaunchKernelGGL(k_cc_push, dim3(launch_grid(vblocks)), dim3(BLOCK), 0, s, ws.plan, ws.queue, ws.hubpref, off, col,
                     ws.state, ws.bits_a, t.hub_chunk, ws.work);
  ktimer_stop(tk, s, "cc_push");
  TG_HIP(hipGetLastError());
  return TG_OK;
}

// Labels (original ids) of the GPU partition's vertices in ws.state.
int gpu_cc(tg_partition *p, hipStream_t s, int64_t *rounds_out) {
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  const Tuning &t = p->tune;
  TG_TRY(ws.ensure(g, 0));
  if (g.n == 0) return TG_OK;
  const unsigned nb = (unsigned)((g.n + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(k_cc_init, dim3(nb), dim3(BLOCK), 0, s, g.g_of_l, g.n, ws.state);
  hipLaunchKernelGGL(k_cc_all_active, dim3((unsigned)((ws.nwords + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s,
                     ws.bits_a, g.n, ws.nwords);
  TG_TRY(fill_i32(ws.settled, g.n, TG_INF, s));
  TG_HIP(hipGetLastError());
  int64_t rounds = 0;
  for (;; ++rounds) {
    // labels only drop, and a component settles within its diameter
    if (rounds > g.n + 1) return set_error(TG_EDEVICE, "cc: no convergence after %lld rounds", (long long)rounds);
    TG_TRY(frontier_compact_sssp(g, ws, ws.bits_a, ws.queue, ws.state, ws.settled, TG_INF, false, g.out_bins, s));
    TG_TRY(frontier_plan(g, ws, ws.queue, t, s, true));
    if (ws.h_plan->count == 0) break;
    TG_TRY(cc_push_launch(g, ws, g.out.off, g.out.col, ws.h_plan->vb[NBIN], t, s));
    if (!g.in_alias) {
      // the other direction: the same frontier over its in-edges (hub chunks
      // by in-degree; vertices without out-edges push too)
      TG_TRY(frontier_plan_off(g, ws, ws.queue, g.in.off, t, s, true, true));
      TG_TRY(cc_push_launch(g, ws, g.in.off, g.in.col, ws.h_plan->vb[NBIN], t, s));
    }
  }
  if (rounds_out) *rounds_out = rounds;
  return TG_OK;
}

}  // namespace tg

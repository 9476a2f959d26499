// Brandes betweenness centrality built from the BFS superstep (section 7.2,
// Figure 18), one source at a time.
//
// Forward cycle: the BFS superstep discovers level L+1; then each new vertex
// w pulls sigma(w) = sum of sigma(u) over in-neighbours u at level L.  The
// pull form needs no atomics and is exact: sigma is an integer held in fp64.
// Backward cycle: levels from the deepest up to 1 (the source receives
// nothing); each vertex v at level L computes
//   delta(v) = sum over out-neighbours w at level L+1 of sigma(v)/sigma(w) * (1 + delta(w))
// (Brandes' recurrence) and adds it to its score.  The ratio is taken in
// fp64; delta is kept in fp32.
#include "gather.h"
#include "tg_internal.h"

using namespace tgk;

namespace {

__global__ void k_set_f64(double *p, int64_t i, double v) {
  if (threadIdx.x == 0) p[i] = v;
}

struct SigmaPull : SumF64 {
  const int32_t *col;
  const int32_t *level;
  const double *sigma_r;
  double *sigma_w;
  uint32_t *flags;
  int32_t parent_level;
  __device__ double vstate(int32_t) const { return 0.0; }
  __device__ double term(double, int64_t e) const {
    const int32_t u = col[e];
    return level[u] == parent_level ? sigma_r[u] : 0.0;
  }
  __device__ void finish(int32_t v, double s) const {
    sigma_w[v] = s;
    if (s >= 9007199254740992.0) flags[2] = 1u;  // 2^53: fp64 counts stop being exact
  }
};

struct DeltaAccum : SumF64 {
  const int32_t *col;
  const int32_t *level;
  const double *sigma;
  float *delta;
  double *score;
  int32_t child_level;
  __device__ double vstate(int32_t v) const { return sigma[v]; }
  __device__ double term(double sv, int64_t e) const {
    const int32_t w = col[e];
    if (level[w] != child_level) return 0.0;
    const float ratio = (float)(sv / sigma[w]);
    return (double)(ratio * (1.0f + delta[w]));
  }
  __device__ void finish(int32_t v, double s) const {
    const float d = (float)s;
    delta[v] = d;
    score[v] += (double)d;
  }
};

}  // namespace

namespace tg {

int gpu_bc_source(tg_partition *p, int32_t src, hipStream_t s) {
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  const Tuning &t = p->tune;
  uint32_t *visited = ws.bits_a, *prev = ws.bits_b;
  int32_t *level = ws.state;
  TG_HIP(hipMemsetAsync(visited, 0, ws.nwords * sizeof(uint32_t), s));
  TG_HIP(hipMemsetAsync(prev, 0, ws.nwords * sizeof(uint32_t), s));
  TG_TRY(fill_i32(level, g.n, TG_INF, s));
  TG_TRY(fill_f64(ws.sigma, g.n, 0.0, s));
  TG_TRY(fill_f32(ws.delta, g.n, 0.0f, s));
  hipLaunchKernelGGL(k_set_f64, dim3(1), dim3(64), 0, s, ws.sigma, (int64_t)src, 1.0);
  TG_TRY(set_bit(visited, src, s));
  TG_TRY(frontier_compact(g, ws, 0, visited, prev, ws.queue, level, 0, s));
  TG_TRY(frontier_plan_off(g, ws, ws.queue, g.out.off, t, s, true));

  std::vector<Plan> plans;
  std::vector<int64_t> segoff;
  int64_t off = 0;
  int32_t L = 0;
  for (;;) {
    if (L > g.n) return set_error(TG_EDEVICE, "bc: more supersteps than vertices");
    const Plan cur = *ws.h_plan;
    plans.push_back(cur);
    segoff.push_back(off);
    TG_TRY(bfs_expand_launch(g, ws, ws.queue + off, cur.vb[NBIN], t, s));
    const int64_t noff = off + cur.count;
    TG_TRY(frontier_compact(g, ws, 0, visited, prev, ws.queue + noff, level, L + 1, s));
    TG_TRY(frontier_plan_off(g, ws, ws.queue + noff, g.out.off, t, s, true));
    if (ws.h_plan->count == 0) break;
    int64_t vbs = ws.h_plan->vb[NBIN];
    if (!g.in_alias) {
      // the pull runs over in-edges: hub chunks follow the in-degree, and
      // vertices without out-edges still pull
      TG_TRY(frontier_plan_off(g, ws, ws.queue + noff, g.in.off, t, s, true, true));
      vbs = ws.h_plan->vb[NBIN];
    }
    SigmaPull op{{}, g.in.col, level, ws.sigma, ws.sigma, ws.counters, L};
    hipLaunchKernelGGL(k_gather<SigmaPull>, dim3(launch_grid(vbs)), dim3(BLOCK), 0, s, ws.plan,
                       ws.queue + noff, ws.hubpref, g.in.off, t.hub_chunk, ws.hub_partials, op);
    hipLaunchKernelGGL(k_gather_hubs<SigmaPull>, dim3(64), dim3(BLOCK), 0, s, ws.plan, ws.queue + noff, ws.hubpref,
                       ws.hub_partials, op);
    TG_HIP(hipGetLastError());
    if (!g.in_alias) {
      // restore the out-degree plan for the next expansion
      TG_TRY(frontier_plan_off(g, ws, ws.queue + noff, g.out.off, t, s, true));
    }
    off = noff;
    ++L;
  }
  // backward: F_L (deepest) keeps delta = 0; accumulate levels L-1 .. 1
  for (int32_t lv = L - 1; lv >= 1; --lv) {
    TG_HIP(hipMemcpyAsync(ws.plan, &plans[lv], sizeof(Plan), hipMemcpyHostToDevice, s));
    TG_TRY(frontier_plan_off(g, ws, ws.queue + segoff[lv], g.out.off, t, s, false));
    DeltaAccum op{{}, g.out.col, level, ws.sigma, ws.delta, ws.bc_acc, lv + 1};
    hipLaunchKernelGGL(k_gather<DeltaAccum>, dim3(launch_grid(plans[lv].vb[NBIN])), dim3(BLOCK), 0, s,
                       ws.plan, ws.queue + segoff[lv], ws.hubpref, g.out.off, t.hub_chunk, ws.hub_partials, op);
    hipLaunchKernelGGL(k_gather_hubs<DeltaAccum>, dim3(64), dim3(BLOCK), 0, s, ws.plan, ws.queue + segoff[lv],
                       ws.hubpref, ws.hub_partials, op);
    TG_HIP(hipGetLastError());
  }
  return TG_OK;
}

}  // namespace tg

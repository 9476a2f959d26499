// PageRank pull gather (section 7.1, Figure 14).  One launch per iteration:
// every vertex v pulls c(u) = r(u)/outdeg(u) over its in-edges, and
//   r'(v) = (1 - d)/N + d * (sum c(u) + D/N),
// where D is the rank held by out-degree-0 vertices (uniform mode) or 0 (drop
// mode).  The same pass writes c'(v) for the next iteration and a per-block
// partial of the new dangling mass; the last block to finish combines the
// partials in block order, so the result is deterministic for a fixed grid.
// Pull needs no atomics on vertex state (the reason Figure 14 pulls).
//
// Hub vertices are split into chunks of `hub_chunk` in-edges, one block per
// chunk; the last chunk block of a hub to finish sums the chunk partials in
// chunk order and finalises that vertex.
#include <algorithm>

#include "tg_internal.h"

using namespace tgk;

namespace {

struct PRParams {
  double base;         // (1 - d) / N
  double d;            // damping
  double inv_n;        // 1 / N
  double iso_count;    // isolated vertices not walked this launch (their r is `add`)
  int64_t hub_chunk;
  int32_t drop;        // 1: dangling mass discarded
  int32_t last;        // 1: write ranks instead of contributions
  int32_t nh;          // hub vertices
  int32_t lds_verts;   // contributions of vertices [0, lds_verts) are staged in LDS
};

template <bool ORDER>
__global__ __launch_bounds__(BLOCK) void k_pr_gather(
    const Plan *__restrict__ Pp, const int32_t *__restrict__ order, const int64_t *__restrict__ hubpref,
    const int64_t *__restrict__ in_off, const int32_t *__restrict__ in_col,
    const int64_t *__restrict__ out_off, const float *__restrict__ c_in, float *__restrict__ c_out,
    PRParams prm, const double *__restrict__ dsum_in, double *__restrict__ dsum_out,
    double *__restrict__ partials, double *hub_partials, double *__restrict__ hub_dangling,
    uint32_t *hub_counters, uint32_t *done_counter, const int32_t *__restrict__ g_of_l,
    float *__restrict__ rank_out, const double *__restrict__ ghost, const int32_t *__restrict__ extra_deg) {
  __shared__ int s_last;
  // The hottest gather targets (lowest local ids: highest out-degree) are
  // staged in LDS once per block; c_in is read-only during the launch.
  extern __shared__ float lds_c[];
  for (int32_t i = threadIdx.x; i < prm.lds_verts; i += BLOCK) lds_c[i] = c_in[i];
  const Plan &P = load_plan(Pp);  // (its barrier also publishes lds_c)
  const double D = prm.drop ? 0.0 : *dsum_in;
  const double add = prm.base + prm.d * D * prm.inv_n;
  double dang = 0.0;
  const int64_t total = P.vb[NBIN];

  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const Assign a = assign_work(vb, P, nullptr, ORDER ? order : nullptr, hubpref, in_off, prm.hub_chunk);
    double s = 0.0;
    if (a.ok) {
      const int64_t st = a.stride;
      int64_t e = a.e_begin + a.lane;
      double s1 = 0.0;
      const int32_t H = prm.lds_verts;
      for (; e + st < a.e_end; e += 2 * st) {
        const int32_t u0 = stream_load(in_col + e), u1 = stream_load(in_col + e + st);
        // generic pointers: one load instruction for the LDS or global case
        const float *p0 = u0 < H ? lds_c + u0 : c_in + u0;
        const float *p1 = u1 < H ? lds_c + u1 : c_in + u1;
        s += (double)*p0;
        s1 += (double)*p1;
      }
      if (e < a.e_end) {
        const int32_t u = stream_load(in_col + e);
        const float *p0 = u < H ? lds_c + u : c_in + u;
        s += (double)*p0;
      }
      s += s1;
    }
    if (a.bin == BIN_HUB) {
      s = block_sum(s);
      const int32_t hi = a.qi - P.pos[0];
      if (threadIdx.x == 0) {
        hub_partials[a.chunk] = s;
        __threadfence();
        const uint32_t nchunks = (uint32_t)(hubpref[hi + 1] - hubpref[hi]);
        const uint32_t prev = atomicAdd(hub_counters + hi, 1u);
        s_last = (prev == nchunks - 1) ? 1 : 0;
      }
      __syncthreads();
      if (s_last && threadIdx.x == 0) {
        __threadfence();
        double tot = 0.0;
        for (int64_t k = hubpref[hi]; k < hubpref[hi + 1]; ++k)
          tot += __hip_atomic_load(hub_partials + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t v = a.v;
        const double r = add + prm.d * (tot + (ghost ? ghost[v] : 0.0));
        const int64_t od = out_off[v + 1] - out_off[v] + (extra_deg ? extra_deg[v] : 0);
        if (prm.last) rank_out[g_of_l[v]] = (float)r;
        else if (od > 0) c_out[v] = (float)(r / (double)od);
        hub_dangling[hi] = (od == 0) ? r : 0.0;
        hub_counters[hi] = 0u;
      }
      __syncthreads();
      continue;
    }
    if (a.bin == BIN_BLOCK) s = block_sum(s);
    else s = group_sum(s, a.stride);
    if (a.ok && a.lane == 0) {
      const int32_t v = a.v;
      const double r = add + prm.d * (s + (ghost ? ghost[v] : 0.0));
      const int64_t od = out_off[v + 1] - out_off[v] + (extra_deg ? extra_deg[v] : 0);
      if (prm.last) rank_out[g_of_l[v]] = (float)r;
      else if (od > 0) __builtin_nontemporal_store((float)(r / (double)od), c_out + v);
      if (od == 0) dang += r;
    }
  }

  // dangling mass of this launch: per-block partials, combined by the last block
  dang = block_sum(dang);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = dang;
    __threadfence();
    const uint32_t prev = atomicAdd(done_counter, 1u);
    s_last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  double acc = 0.0;
  for (uint32_t i = threadIdx.x; i < gridDim.x; i += BLOCK)
    acc += __hip_atomic_load(partials + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int32_t i = threadIdx.x; i < prm.nh; i += BLOCK)
    acc += __hip_atomic_load(hub_dangling + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  acc = block_sum(acc);
  if (threadIdx.x == 0) {
    *dsum_out = acc + prm.iso_count * add;
    *done_counter = 0u;
  }
}

__global__ __launch_bounds__(BLOCK) void k_pr_init(const int64_t *__restrict__ out_off, int64_t n,
                                                   double inv_n, float *__restrict__ c,
                                                   const int32_t *__restrict__ extra_deg) {
  const int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v >= n) return;
  const int64_t od = out_off[v + 1] - out_off[v] + (extra_deg ? extra_deg[v] : 0);
  c[v] = od > 0 ? (float)(inv_n / (double)od) : 0.0f;
}

__global__ __launch_bounds__(BLOCK) void k_pr_uniform(const int32_t *__restrict__ g_of_l, int64_t n,
                                                      float value, float *__restrict__ rank_out) {
  const int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v < n) rank_out[g_of_l[v]] = value;
}

}  // namespace

namespace tg {

int pr_init_contrib(const GpuPart &g, float *c, double N, hipStream_t s, const int32_t *extra_deg) {
  hipLaunchKernelGGL(k_pr_init, dim3((unsigned)((g.n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, g.out.off,
                     g.n, 1.0 / N, c, extra_deg);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int pr_write_initial(const GpuPart &g, float *rank_out, double N, hipStream_t s) {
  hipLaunchKernelGGL(k_pr_uniform, dim3((unsigned)((g.n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, g.g_of_l,
                     g.n, (float)(1.0 / N), rank_out);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int gpu_pagerank_setup(tg_partition *p, double damping, int mode, hipStream_t s, const int32_t *extra_deg,
                       double d0) {
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  TG_TRY(ws.ensure(g, g.pr.work.vb[1]));
  const double N = (double)g.n_global;
  TG_HIP(hipMemcpyAsync(ws.scalars, &d0, sizeof(double), hipMemcpyHostToDevice, s));
  TG_HIP(hipMemsetAsync(ws.counters, 0, 4 * sizeof(uint32_t), s));
  TG_HIP(hipMemsetAsync(ws.hub_counters, 0, (g.pr.nh + 1) * sizeof(uint32_t), s));
  TG_TRY(pr_init_contrib(g, ws.cbuf[0], N, s, extra_deg));
  (void)damping;
  (void)mode;
  return TG_OK;
}

// One pull iteration k (contributions cbuf[k&1] -> cbuf[(k+1)&1], dangling
// sum scalars[k&1] -> scalars[(k+1)&1]); `last` writes ranks instead.
int gpu_pagerank_step(tg_partition *p, double damping, int mode, int32_t k, bool last, float *rank_out,
                      hipStream_t s, const double *ghost, const int32_t *extra_deg) {
  if (p->tune.pr_rows) return gpu_pagerank_rows_step(p, damping, mode, k, last, rank_out, s, ghost, extra_deg);
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  const double N = (double)g.n_global;
  double *dsum = ws.scalars;
  const bool ordered = g.pr_order != nullptr;
  PRParams prm;
  prm.base = (1.0 - damping) / N;
  prm.d = damping;
  prm.inv_n = 1.0 / N;
  prm.hub_chunk = p->tune.hub_chunk;
  prm.drop = (mode == TG_PR_DANGLING_DROP) ? 1 : 0;
  prm.nh = g.pr.nh;
  prm.lds_verts = (int32_t)std::min<int64_t>(p->tune.pr_lds_verts, g.n);
  const size_t lds_bytes = (size_t)prm.lds_verts * sizeof(float);
  // Isolated vertices (no in- or out-edges) only need walking when their
  // rank is written; otherwise their share of the dangling mass is added
  // analytically.  Directed graphs walk every vertex (in-degree-0 vertices
  // may still have out-edges whose contribution must be refreshed).
  const bool walk_all = ordered || last;
  const Plan *plan = walk_all ? g.pr.d_all : g.pr.d_work;
  const int64_t vbs = walk_all ? g.pr.all.vb[NBIN] : g.pr.work.vb[NBIN];
  prm.last = last ? 1 : 0;
  prm.iso_count = walk_all ? 0.0 : (double)g.n_isolated;
  // one pass of blocks over the chip: each block stages lds_c once
  const int grid = (int)std::min<int64_t>(launch_grid(vbs), p->tune.pr_grid);
  const int tk = ktimer_start(s);
  const float *cin = ws.cbuf[k & 1];
  float *cout = ws.cbuf[(k + 1) & 1];
  if (ordered)
    hipLaunchKernelGGL(k_pr_gather<true>, dim3(grid), dim3(BLOCK), lds_bytes, s, plan, g.pr_order, g.pr.hubpref,
                       g.in.off, g.in.col, g.out.off, cin, cout, prm, dsum + (k & 1), dsum + ((k + 1) & 1),
                       ws.partials, ws.hub_partials, ws.hub_dangling, ws.hub_counters, ws.counters, g.g_of_l,
                       rank_out, ghost, extra_deg);
  else
    hipLaunchKernelGGL(k_pr_gather<false>, dim3(grid), dim3(BLOCK), lds_bytes, s, plan, nullptr, g.pr.hubpref,
                       g.in.off, g.in.col, g.out.off, cin, cout, prm, dsum + (k & 1), dsum + ((k + 1) & 1),
                       ws.partials, ws.hub_partials, ws.hub_dangling, ws.hub_counters, ws.counters, g.g_of_l,
                       rank_out, ghost, extra_deg);
  ktimer_stop(tk, s, "pr_gather");
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int gpu_pagerank(tg_partition *p, double damping, int32_t iters, int mode, float *rank_out,
                 hipStream_t s) {
  GpuPart &g = p->gpu;
  if (g.n == 0) return TG_OK;
  const double N = (double)g.n_global;
  // r_0 = 1/N, so c_0(u) = 1/(N outdeg(u)) and D_0 = (#dangling)/N
  TG_TRY(gpu_pagerank_setup(p, damping, mode, s, nullptr, (double)g.n_dangling / N));
  if (iters == 0) return pr_write_initial(g, rank_out, N, s);
  for (int32_t k = 0; k < iters; ++k) {
    if (p->tune.pr_xcd)
      TG_TRY(gpu_pagerank_sliced_step(p, damping, mode, k, k == iters - 1, rank_out, s));
    else
      TG_TRY(gpu_pagerank_step(p, damping, mode, k, k == iters - 1, rank_out, s, nullptr, nullptr));
  }
  return TG_OK;
}

}  // namespace tg

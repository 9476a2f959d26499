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
};

template <bool ORDER>
__global__ __launch_bounds__(BLOCK) void k_pr_gather(
    const Plan *__restrict__ Pp, const int32_t *__restrict__ order, const int64_t *__restrict__ hubpref,
    const int64_t *__restrict__ in_off, const int32_t *__restrict__ in_col,
    const int64_t *__restrict__ out_off, const float *__restrict__ c_in, float *__restrict__ c_out,
    PRParams prm, const double *__restrict__ dsum_in, double *__restrict__ dsum_out,
    double *__restrict__ partials, double *hub_partials, double *__restrict__ hub_dangling,
    uint32_t *hub_counters, uint32_t *done_counter, const int32_t *__restrict__ g_of_l,
    float *__restrict__ rank_out) {
  __shared__ int s_last;
  const Plan P = *Pp;
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
      for (; e + st < a.e_end; e += 2 * st) {
        const int32_t u0 = in_col[e], u1 = in_col[e + st];
        s += (double)c_in[u0];
        s1 += (double)c_in[u1];
      }
      if (e < a.e_end) s += (double)c_in[in_col[e]];
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
        const double r = add + prm.d * tot;
        const int64_t od = out_off[v + 1] - out_off[v];
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
      const double r = add + prm.d * s;
      const int64_t od = out_off[v + 1] - out_off[v];
      if (prm.last) rank_out[g_of_l[v]] = (float)r;
      else if (od > 0) c_out[v] = (float)(r / (double)od);
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
                                                   double inv_n, float *__restrict__ c) {
  const int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v >= n) return;
  const int64_t od = out_off[v + 1] - out_off[v];
  c[v] = od > 0 ? (float)(inv_n / (double)od) : 0.0f;
}

__global__ __launch_bounds__(BLOCK) void k_pr_uniform(const int32_t *__restrict__ g_of_l, int64_t n,
                                                      float value, float *__restrict__ rank_out) {
  const int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v < n) rank_out[g_of_l[v]] = value;
}

}  // namespace

namespace tg {

int pr_init_contrib(const GpuPart &g, float *c, double N, hipStream_t s) {
  hipLaunchKernelGGL(k_pr_init, dim3((unsigned)((g.n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, g.out.off,
                     g.n, 1.0 / N, c);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int pr_write_initial(const GpuPart &g, float *rank_out, double N, hipStream_t s) {
  hipLaunchKernelGGL(k_pr_uniform, dim3((unsigned)((g.n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, g.g_of_l,
                     g.n, (float)(1.0 / N), rank_out);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int gpu_pagerank(tg_partition *p, double damping, int32_t iters, int mode, float *rank_out,
                 hipStream_t s) {
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  const int64_t n = g.n;
  if (n == 0) return TG_OK;
  const int64_t chunks = g.pr.work.vb[1];
  TG_TRY(ws.ensure(g, chunks));
  const double N = (double)g.n_global;
  // r_0 = 1/N, so c_0(u) = 1/(N outdeg(u)) and D_0 = (#dangling)/N
  double *dsum = ws.scalars;
  const double d0 = (double)g.n_dangling / N;
  TG_HIP(hipMemcpyAsync(dsum, &d0, sizeof(double), hipMemcpyHostToDevice, s));
  TG_HIP(hipMemsetAsync(ws.counters, 0, 4 * sizeof(uint32_t), s));
  TG_HIP(hipMemsetAsync(ws.hub_counters, 0, (g.pr.nh + 1) * sizeof(uint32_t), s));
  TG_TRY(pr_init_contrib(g, ws.cbuf[0], N, s));
  const bool ordered = g.pr_order != nullptr;
  PRParams prm;
  prm.base = (1.0 - damping) / N;
  prm.d = damping;
  prm.inv_n = 1.0 / N;
  prm.hub_chunk = p->tune.hub_chunk;
  prm.drop = (mode == TG_PR_DANGLING_DROP) ? 1 : 0;
  prm.nh = g.pr.nh;
  if (iters == 0) return pr_write_initial(g, rank_out, N, s);
  for (int32_t k = 0; k < iters; ++k) {
    const bool last = (k == iters - 1);
    // Isolated vertices (no in- or out-edges) only need walking when their
    // rank is written; otherwise their share of the dangling mass is added
    // analytically.  Directed graphs walk every vertex (in-degree-0 vertices
    // may still have out-edges whose contribution must be refreshed).
    const bool walk_all = ordered || last;
    const Plan *plan = walk_all ? g.pr.d_all : g.pr.d_work;
    const int64_t vbs = walk_all ? g.pr.all.vb[NBIN] : g.pr.work.vb[NBIN];
    prm.last = last ? 1 : 0;
    prm.iso_count = walk_all ? 0.0 : (double)g.n_isolated;
    const int grid = launch_grid(vbs);
    const int tk = ktimer_start(s);
    const float *cin = ws.cbuf[k & 1];
    float *cout = ws.cbuf[(k + 1) & 1];
    if (ordered)
      hipLaunchKernelGGL(k_pr_gather<true>, dim3(grid), dim3(BLOCK), 0, s, plan, g.pr_order, g.pr.hubpref,
                         g.in.off, g.in.col, g.out.off, cin, cout, prm, dsum + (k & 1),
                         dsum + ((k + 1) & 1), ws.partials, ws.hub_partials, ws.hub_dangling,
                         ws.hub_counters, ws.counters, g.g_of_l, rank_out);
    else
      hipLaunchKernelGGL(k_pr_gather<false>, dim3(grid), dim3(BLOCK), 0, s, plan, nullptr, g.pr.hubpref,
                         g.in.off, g.in.col, g.out.off, cin, cout, prm, dsum + (k & 1),
                         dsum + ((k + 1) & 1), ws.partials, ws.hub_partials, ws.hub_dangling,
                         ws.hub_counters, ws.counters, g.g_of_l, rank_out);
    ktimer_stop(tk, s, "pr_gather");
    TG_HIP(hipGetLastError());
  }
  return TG_OK;
}

}  // namespace tg

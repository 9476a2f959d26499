// PageRank (section 7.1, Figure 14): set-up and the iteration driver.  Each
// iteration every vertex v pulls c(u) = r(u)/outdeg(u) over its in-edges and
//   r'(v) = (1 - d)/N + d * (sum c(u) + D/N),
// where D is the rank held by out-degree-0 vertices (uniform mode) or 0 (drop
// mode).  Pull needs no atomics on vertex state (the reason Figure 14 pulls).
// The gather itself is in pr_rows.hip (whole CSR) and pr_sliced.hip (per-XCD
// source classes).
#include <algorithm>

#include "tg_internal.h"

using namespace tgk;

namespace {

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
  TG_TRY(ws.ensure(g, 0));
  const double N = (double)g.n_global;
  TG_HIP(hipMemcpyAsync(ws.scalars, &d0, sizeof(double), hipMemcpyHostToDevice, s));
  TG_TRY(pr_init_contrib(g, ws.cbuf[0], N, s, extra_deg));
  (void)damping;
  (void)mode;
  return TG_OK;
}

// One pull iteration k (contributions cbuf[k&1] -> cbuf[(k+1)&1], dangling
// sum scalars[k&1] -> scalars[(k+1)&1]); `last` writes ranks instead.  The
// gather runs over row blocks of the in-edges (pr_rows.hip).
int gpu_pagerank_step(tg_partition *p, double damping, int mode, int32_t k, bool last, float *rank_out,
                      hipStream_t s, const double *ghost, const int32_t *extra_deg) {
  return gpu_pagerank_rows_step(p, damping, mode, k, last, rank_out, s, ghost, extra_deg);
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

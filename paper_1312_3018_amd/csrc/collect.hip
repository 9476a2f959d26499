// Collect (Appendix 1, the collect callback): move per-vertex state from the
// partition's local id space to the caller's buffer in original id order,
// plus small fill kernels and the BFS parent pass.
#include "tg_internal.h"

using namespace tgk;

namespace {

inline int blocks_for(int64_t n) { return (int)((n + BLOCK - 1) / BLOCK); }

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_fill(T *__restrict__ p, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) p[i] = v;
}

// out[g] = level of local vertex l_of_g[g] if visited, else INF.  Global ids
// that belong to another partition (l < 0) are left untouched.
__global__ __launch_bounds__(BLOCK) void k_collect_levels(const int32_t *__restrict__ l_of_g, int64_t V,
                                                          const uint32_t *__restrict__ visited,
                                                          const int32_t *__restrict__ level,
                                                          int32_t *__restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (gid >= V) return;
  const int32_t l = l_of_g[gid];
  if (l < 0) return;
  const bool seen = (visited[l >> 5] >> (l & 31)) & 1u;
  out[gid] = seen ? level[l] : TG_INF;
}

__global__ __launch_bounds__(BLOCK) void k_collect_i32(const int32_t *__restrict__ l_of_g, int64_t V,
                                                       const int32_t *__restrict__ st,
                                                       int32_t *__restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (gid >= V) return;
  const int32_t l = l_of_g[gid];
  if (l >= 0) out[gid] = st[l];
}

__global__ __launch_bounds__(BLOCK) void k_collect_f64_f32(const int32_t *__restrict__ l_of_g, int64_t V,
                                                           const double *__restrict__ st,
                                                           float *__restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (gid >= V) return;
  const int32_t l = l_of_g[gid];
  if (l >= 0) out[gid] = (float)st[l];
}

// parent[g] of local l: root -> root; unreached -> -1; otherwise the first
// in-neighbour (in local order) whose level is one less.  Deterministic.
__global__ __launch_bounds__(BLOCK) void k_parents(const int32_t *__restrict__ l_of_g, int64_t V,
                                                   const int32_t *__restrict__ g_of_l,
                                                   const int64_t *__restrict__ in_off,
                                                   const int32_t *__restrict__ in_col,
                                                   const uint32_t *__restrict__ visited,
                                                   const int32_t *__restrict__ level, int32_t root,
                                                   int32_t *__restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (gid >= V) return;
  const int32_t l = l_of_g[gid];
  if (l < 0) return;
  if (l == root) { out[gid] = (int32_t)gid; return; }
  if (!((visited[l >> 5] >> (l & 31)) & 1u)) { out[gid] = -1; return; }
  const int32_t want = level[l] - 1;
  int32_t best = -1;
  for (int64_t e = in_off[l]; e < in_off[l + 1]; ++e) {
    const int32_t u = in_col[e];
    if (((visited[u >> 5] >> (u & 31)) & 1u) && level[u] == want) { best = u; break; }
  }
  out[gid] = best < 0 ? -1 : g_of_l[best];
}

}  // namespace

namespace tg {

int fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return TG_OK;
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(blocks_for(n)), dim3(BLOCK), 0, s, p, n, v);
  TG_HIP(hipGetLastError());
  return TG_OK;
}
int fill_f64(double *p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return TG_OK;
  hipLaunchKernelGGL(k_fill<double>, dim3(blocks_for(n)), dim3(BLOCK), 0, s, p, n, v);
  TG_HIP(hipGetLastError());
  return TG_OK;
}
int fill_f32(float *p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return TG_OK;
  hipLaunchKernelGGL(k_fill<float>, dim3(blocks_for(n)), dim3(BLOCK), 0, s, p, n, v);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int collect_levels(const GpuPart &g, const uint32_t *visited, const int32_t *level, int32_t *out,
                   hipStream_t s) {
  const int64_t V = (int64_t)g.n_global;
  if (V <= 0) return TG_OK;
  hipLaunchKernelGGL(k_collect_levels, dim3(blocks_for(V)), dim3(BLOCK), 0, s, g.l_of_g, V, visited,
                     level, out);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int collect_i32(const GpuPart &g, const int32_t *state, int32_t *out, hipStream_t s) {
  const int64_t V = (int64_t)g.n_global;
  if (V <= 0) return TG_OK;
  hipLaunchKernelGGL(k_collect_i32, dim3(blocks_for(V)), dim3(BLOCK), 0, s, g.l_of_g, V, state, out);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int collect_f64_to_f32(const GpuPart &g, const double *state, float *out, hipStream_t s) {
  const int64_t V = (int64_t)g.n_global;
  if (V <= 0) return TG_OK;
  hipLaunchKernelGGL(k_collect_f64_f32, dim3(blocks_for(V)), dim3(BLOCK), 0, s, g.l_of_g, V, state,
                     out);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int bfs_parents(const GpuPart &g, const uint32_t *visited, const int32_t *level, int32_t root_local,
                int32_t *out, hipStream_t s) {
  const int64_t V = (int64_t)g.n_global;
  if (V <= 0) return TG_OK;
  hipLaunchKernelGGL(k_parents, dim3(blocks_for(V)), dim3(BLOCK), 0, s, g.l_of_g, V, g.g_of_l,
                     g.in.off, g.in.col, visited, level, root_local, out);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

}  // namespace tg

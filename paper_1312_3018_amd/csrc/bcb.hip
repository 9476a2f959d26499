// Batched Brandes betweenness (section 7.2, Figure 18) for up to 64 sources
// per chain of supersteps.  Vertex state is laid out [vertex][source] so that
// one 64-lane wavefront holds a vertex's row with lane = source: a vertex's
// sigma row is one coalesced 512-byte read.
//
// Forward: a multi-source BFS superstep (one bit per source in the frontier,
// visited and next masks) discovers level L+1 for every source at once; then
// each newly reached vertex w pulls, for every source s whose frontier
// reached it, sigma[w][s] = sum of sigma[u][s] over in-neighbours u that were
// on s's frontier at level L (the level-L masks are kept until the pull is
// done).  Backward: for L from the deepest level down to 1, every vertex v
// with some source at level L computes, per such source,
//   delta[v][s] = sum over out-neighbours w with level[w][s] == L+1 of
//                 sigma[v][s] / sigma[w][s] * (1 + delta[w][s])
// and adds the row sum to its score.  Hubs (the HUB bin) are split into
// chunks of hub_chunk edges, one 256-thread block per chunk leaving a row of
// per-source partial sums, and one wavefront per hub adds its chunks in
// order; vertices of the BLOCK bin get a block each, whose four wavefronts
// split the edge list and combine in LDS; all others a wavefront each, which
// walks the edge list four edges at a time with no barrier.
#include <string.h>

#include <algorithm>
#include <vector>

#include "tg_internal.h"

using namespace tgk;

namespace tg {
namespace {

using u64 = unsigned long long;
constexpr int S = 64;  // sources per chain

inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>((n + BLOCK - 1) / BLOCK, 1); }

__global__ __launch_bounds__(BLOCK) void k_bb_expand(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                     const int64_t *__restrict__ hubpref,
                                                     const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                     const u64 *front, const u64 *visited, u64 *next,
                                                     uint32_t *touched, int64_t hub_chunk) {
  const Plan &P = load_plan(Pp);
  const int64_t total = P.vb[NBIN];
  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const Assign a = assign_work(vb, P, queue, nullptr, hubpref, off, hub_chunk);
    if (!a.ok) continue;
    const u64 m = front[a.v];
    if (m == 0) continue;
    for (int64_t e = a.e_begin + a.lane; e < a.e_end; e += a.stride) {
      const int32_t nb = stream_load(col + e);
      const u64 x = m & ~visited[nb];
      if (x && atomicOr(next + nb, x) == 0) atomicOr(touched + (nb >> 5), 1u << (nb & 31));
    }
  }
}

// Settle level L+1: new bits, visited, the new frontier masks and levels.
__global__ __launch_bounds__(BLOCK) void k_bb_finalize(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                       u64 *visited, u64 *front_new, u64 *next, int32_t *lev,
                                                       int32_t level) {
  const int32_t count = Pp->count;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < count; i += (int64_t)gridDim.x * BLOCK) {
    const int32_t v = queue[i];
    const u64 nb = next[v] & ~visited[v];
    next[v] = 0;
    visited[v] |= nb;
    front_new[v] = nb;
    u64 bits = nb;
    while (bits) {
      const int s = __ffsll((long long)bits) - 1;
      bits &= bits - 1;
      lev[(int64_t)v * S + s] = level;
    }
  }
}

// Combine the four wavefronts' per-lane partials of one block.
__device__ __forceinline__ double block_lane_sum(double x, double *red) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  red[w * 64 + lane] = x;
  __syncthreads();
  return red[lane] + red[64 + lane] + red[128 + lane] + red[192 + lane];
}

// sigma pull for the vertices that were reached at level L+1.
__global__ __launch_bounds__(BLOCK) void k_bb_sigma(const int32_t *__restrict__ queue, int32_t lo, int32_t hi,
                                                    const int64_t *__restrict__ ioff, const int32_t *__restrict__ icol,
                                                    const u64 *__restrict__ front_old, const u64 *__restrict__ front_new,
                                                    double *sigma, uint32_t *flags) {
  __shared__ double red[BLOCK];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t i = lo + (int64_t)blockIdx.x; i < hi; i += gridDim.x) {
    const int32_t v = queue[i];
    const u64 m = front_new[v];  // block-uniform
    if (m == 0) continue;
    double acc = 0.0;
    for (int64_t e = ioff[v] + w; e < ioff[v + 1]; e += 4) {
      const int32_t u = icol[e];
      const u64 mu = front_old[u] & m;
      if ((mu >> lane) & 1ull) acc += sigma[(int64_t)u * S + lane];
    }
    acc = block_lane_sum(acc, red);
    if (w == 0 && ((m >> lane) & 1ull)) {
      sigma[(int64_t)v * S + lane] = acc;
      if (acc >= 9007199254740992.0) flags[2] = 1u;  // 2^53
    }
  }
}

// Dependencies of the vertices with some source at level L.
__global__ __launch_bounds__(BLOCK) void k_bb_delta(const int32_t *__restrict__ queue, int32_t lo, int32_t hi,
                                                    const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                    const int32_t *__restrict__ lev, const double *__restrict__ sigma,
                                                    float *delta, double *score, int32_t level) {
  __shared__ double red[BLOCK];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t i = lo + (int64_t)blockIdx.x; i < hi; i += gridDim.x) {
    const int32_t v = queue[i];
    const bool mine = lev[(int64_t)v * S + lane] == level;
    const double sv = mine ? sigma[(int64_t)v * S + lane] : 0.0;
    double acc = 0.0;
    if (mine)
      for (int64_t e = off[v] + w; e < off[v + 1]; e += 4) {
        const int32_t x = col[e];
        const int64_t r = (int64_t)x * S + lane;
        if (lev[r] == level + 1) {
          const float ratio = (float)(sv / sigma[r]);
          acc += (double)(ratio * (1.0f + delta[r]));
        }
      }
    acc = block_lane_sum(acc, red);
    if (w == 0) {
      const float d = (float)acc;
      if (mine) delta[(int64_t)v * S + lane] = d;
      double row = mine ? (double)d : 0.0;
      for (int o = 32; o > 0; o >>= 1) row += __shfl_xor(row, o, 64);
      if (lane == 0) score[v] += row;
    }
  }
}

// Hub chunks: virtual block j of the plan's HUB segment covers edges
// [e0, e1) of one hub; its four wavefronts split them and the per-source
// partial sum goes to part[j][source].  The sigma pass pulls over in-edges,
// the delta pass over out-edges.
__global__ __launch_bounds__(BLOCK) void k_bb_sigma_hubs(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                         const int64_t *__restrict__ hubpref,
                                                         const int64_t *__restrict__ ioff,
                                                         const int32_t *__restrict__ icol,
                                                         const u64 *__restrict__ front_old,
                                                         const u64 *__restrict__ front_new,
                                                         const double *__restrict__ sigma, int64_t hub_chunk,
                                                         double *part) {
  __shared__ double red[BLOCK];
  const Plan &P = load_plan(Pp);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t vb = blockIdx.x; vb < P.vb[1]; vb += gridDim.x) {
    const Assign a = assign_work(vb, P, queue, nullptr, hubpref, ioff, hub_chunk);  // HUB: block-uniform
    const u64 m = front_new[a.v];
    double acc = 0.0;
    if (m != 0)
      for (int64_t e = a.e_begin + w; e < a.e_end; e += 4) {
        const int32_t u = icol[e];
        if (((front_old[u] & m) >> lane) & 1ull) acc += sigma[(int64_t)u * S + lane];
      }
    acc = block_lane_sum(acc, red);
    if (w == 0) part[a.chunk * S + lane] = acc;
  }
}

__global__ __launch_bounds__(BLOCK) void k_bb_delta_hubs(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                         const int64_t *__restrict__ hubpref,
                                                         const int64_t *__restrict__ off,
                                                         const int32_t *__restrict__ col,
                                                         const int32_t *__restrict__ lev,
                                                         const double *__restrict__ sigma,
                                                         const float *__restrict__ delta, int32_t level,
                                                         int64_t hub_chunk, double *part) {
  __shared__ double red[BLOCK];
  const Plan &P = load_plan(Pp);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t vb = blockIdx.x; vb < P.vb[1]; vb += gridDim.x) {
    const Assign a = assign_work(vb, P, queue, nullptr, hubpref, off, hub_chunk);
    const int32_t v = a.v;
    const bool mine = lev[(int64_t)v * S + lane] == level;
    const double sv = mine ? sigma[(int64_t)v * S + lane] : 0.0;
    double acc = 0.0;
    if (mine)
      for (int64_t e = a.e_begin + w; e < a.e_end; e += 4) {
        const int64_t r = (int64_t)col[e] * S + lane;
        if (lev[r] == level + 1) {
          const float ratio = (float)(sv / sigma[r]);
          acc += (double)(ratio * (1.0f + delta[r]));
        }
      }
    acc = block_lane_sum(acc, red);
    if (w == 0) part[a.chunk * S + lane] = acc;
  }
}

// One wavefront per hub of the plan: its chunks' partial sums, added in
// chunk order, finish the hub like the block kernels do.
__global__ __launch_bounds__(BLOCK) void k_bb_hubs_finish(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                          const int64_t *__restrict__ hubpref,
                                                          const double *__restrict__ part, int mode,
                                                          const u64 *__restrict__ front_new, double *sigma,
                                                          uint32_t *flags, const int32_t *__restrict__ lev,
                                                          float *delta, double *score, int32_t level) {
  const int lane = threadIdx.x & 63;
  const int32_t p0 = Pp->pos[0], nh = Pp->pos[1] - p0;
  const int64_t nw = ((int64_t)gridDim.x * BLOCK) >> 6;
  for (int64_t i = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6; i < nh; i += nw) {
    const int32_t v = queue[p0 + i];
    double acc = 0.0;
    for (int64_t c = hubpref[i]; c < hubpref[i + 1]; ++c) acc += part[c * S + lane];
    if (mode == 0) {
      if ((front_new[v] >> lane) & 1ull) {
        sigma[(int64_t)v * S + lane] = acc;
        if (acc >= 9007199254740992.0) flags[2] = 1u;  // 2^53
      }
    } else {
      const bool mine = lev[(int64_t)v * S + lane] == level;
      const float d = (float)acc;
      if (mine) delta[(int64_t)v * S + lane] = d;
      double row = mine ? (double)d : 0.0;
      for (int o = 32; o > 0; o >>= 1) row += __shfl_xor(row, o, 64);
      if (lane == 0) score[v] += row;
    }
  }
}

// The same two passes with one wavefront per vertex (lane = source) for the
// vertices [lo, hi) of the queue, four edges in flight per step.
__global__ __launch_bounds__(BLOCK) void k_bb_sigma_wave(const int32_t *__restrict__ queue, int32_t lo, int32_t hi,
                                                         const int64_t *__restrict__ ioff,
                                                         const int32_t *__restrict__ icol,
                                                         const u64 *__restrict__ front_old,
                                                         const u64 *__restrict__ front_new, double *sigma,
                                                         uint32_t *flags) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * BLOCK) >> 6;
  for (int64_t i = lo + (((int64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6); i < hi; i += nw) {
    const int32_t v = queue[i];
    const u64 m = front_new[v];  // wave-uniform
    if (m == 0) continue;
    const int64_t e0 = ioff[v], e1 = ioff[v + 1];
    double acc = 0.0;
    int64_t e = e0;
    for (; e + 3 < e1; e += 4) {
      int32_t u[4];
      u64 mu[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) u[k] = icol[e + k];
#pragma unroll
      for (int k = 0; k < 4; ++k) mu[k] = front_old[u[k]] & m;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if ((mu[k] >> lane) & 1ull) acc += sigma[(int64_t)u[k] * S + lane];
    }
    for (; e < e1; ++e) {
      const int32_t u = icol[e];
      if (((front_old[u] & m) >> lane) & 1ull) acc += sigma[(int64_t)u * S + lane];
    }
    if ((m >> lane) & 1ull) {
      sigma[(int64_t)v * S + lane] = acc;
      if (acc >= 9007199254740992.0) flags[2] = 1u;  // 2^53
    }
  }
}

__global__ __launch_bounds__(BLOCK) void k_bb_delta_wave(const int32_t *__restrict__ queue, int32_t lo, int32_t hi,
                                                         const int64_t *__restrict__ off,
                                                         const int32_t *__restrict__ col,
                                                         const int32_t *__restrict__ lev,
                                                         const double *__restrict__ sigma, float *delta,
                                                         double *score, int32_t level) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * BLOCK) >> 6;
  for (int64_t i = lo + (((int64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6); i < hi; i += nw) {
    const int32_t v = queue[i];
    const bool mine = lev[(int64_t)v * S + lane] == level;
    if (!__ballot(mine)) continue;
    const double sv = mine ? sigma[(int64_t)v * S + lane] : 0.0;
    double acc = 0.0;
    if (mine) {
      const int64_t e0 = off[v], e1 = off[v + 1];
      int64_t e = e0;
      for (; e + 3 < e1; e += 4) {
        int32_t x[4], lx[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = col[e + k];
#pragma unroll
        for (int k = 0; k < 4; ++k) lx[k] = lev[(int64_t)x[k] * S + lane];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (lx[k] == level + 1) {
            const int64_t r = (int64_t)x[k] * S + lane;
            const float ratio = (float)(sv / sigma[r]);
            acc += (double)(ratio * (1.0f + delta[r]));
          }
      }
      for (; e < e1; ++e) {
        const int64_t r = (int64_t)col[e] * S + lane;
        if (lev[r] == level + 1) {
          const float ratio = (float)(sv / sigma[r]);
          acc += (double)(ratio * (1.0f + delta[r]));
        }
      }
    }
    const float d = (float)acc;
    if (mine) delta[(int64_t)v * S + lane] = d;
    double row = mine ? (double)d : 0.0;
    for (int o = 32; o > 0; o >>= 1) row += __shfl_xor(row, o, 64);
    if (lane == 0) score[v] += row;
  }
}

__global__ void k_bb_join(u64 *next, uint32_t *touched, double *sigma, int32_t root, int slot) {
  if (threadIdx.x != 0) return;
  atomicOr(next + root, 1ull << slot);
  atomicOr(touched + (root >> 5), 1u << (root & 31));
  sigma[(int64_t)root * S + slot] = 1.0;
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_bb_fill(T *p, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) p[i] = v;
}

// Queue positions: hubs in chunks (plan P, with its hub chunk prefix in
// ws.hubpref and on the device in ws.plan, sized for the edges walked),
// the BLOCK bin a block each, the rest a wavefront each.
int launch_sigma(const GpuPart &g, Workspace &ws, const Tuning &t, const Plan &P, const int32_t *queue,
                 const u64 *front_old, const u64 *front_new, double *sigma, uint32_t *flags, double *part,
                 hipStream_t s) {
  const int32_t hubs = P.pos[1], split = P.pos[BIN_WAVE], count = P.count;
  if (hubs > 0) {
    hipLaunchKernelGGL(k_bb_sigma_hubs, dim3((unsigned)launch_grid(P.vb[1])), dim3(BLOCK), 0, s, ws.plan, queue,
                       ws.hubpref, g.in.off, g.in.col, front_old, front_new, sigma, t.hub_chunk, part);
    hipLaunchKernelGGL(k_bb_hubs_finish, dim3((unsigned)std::max<int32_t>((hubs + 3) / 4, 1)), dim3(BLOCK), 0, s,
                       ws.plan, queue, ws.hubpref, part, 0, front_new, sigma, flags, nullptr, nullptr, nullptr, 0);
  }
  if (split > hubs)
    hipLaunchKernelGGL(k_bb_sigma, dim3((unsigned)std::min<int32_t>(split - hubs, 16384)), dim3(BLOCK), 0, s, queue,
                       hubs, split, g.in.off, g.in.col, front_old, front_new, sigma, flags);
  if (count > split)
    hipLaunchKernelGGL(k_bb_sigma_wave, dim3((unsigned)std::min<int64_t>((count - split + 3) / 4, 16384)),
                       dim3(BLOCK), 0, s, queue, split, count, g.in.off, g.in.col, front_old, front_new, sigma, flags);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int launch_delta(const GpuPart &g, Workspace &ws, const Tuning &t, const Plan &P, const int32_t *queue,
                 const int32_t *lev, const double *sigma, float *delta, double *score, int32_t level, double *part,
                 hipStream_t s) {
  const int32_t hubs = P.pos[1], split = P.pos[BIN_WAVE], count = P.count;
  if (hubs > 0) {
    hipLaunchKernelGGL(k_bb_delta_hubs, dim3((unsigned)launch_grid(P.vb[1])), dim3(BLOCK), 0, s, ws.plan, queue,
                       ws.hubpref, g.out.off, g.out.col, lev, sigma, delta, level, t.hub_chunk, part);
    hipLaunchKernelGGL(k_bb_hubs_finish, dim3((unsigned)std::max<int32_t>((hubs + 3) / 4, 1)), dim3(BLOCK), 0, s,
                       ws.plan, queue, ws.hubpref, part, 1, nullptr, nullptr, nullptr, lev, delta, score, level);
  }
  if (split > hubs)
    hipLaunchKernelGGL(k_bb_delta, dim3((unsigned)std::min<int32_t>(split - hubs, 16384)), dim3(BLOCK), 0, s, queue,
                       hubs, split, g.out.off, g.out.col, lev, sigma, delta, score, level);
  if (count > split)
    hipLaunchKernelGGL(k_bb_delta_wave, dim3((unsigned)std::min<int64_t>((count - split + 3) / 4, 16384)),
                       dim3(BLOCK), 0, s, queue, split, count, g.out.off, g.out.col, lev, sigma, delta, score, level);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

}  // namespace

// Scratch of the batched BC (lazy, per partition).
struct BcBatchState {
  DevArena arena;
  Workspace ws;
  int64_t n = -1;
  u64 *visited = nullptr, *front[2] = {nullptr, nullptr}, *next = nullptr;
  int32_t *lev = nullptr;
  double *sigma = nullptr;
  float *delta = nullptr;
  int32_t *queue_all = nullptr;  // level queues back to back
  double *hub_part = nullptr;     // per hub chunk, a partial sum per source
};

void bcb_free(tg_partition *p) {
  delete p->bcb;
  p->bcb = nullptr;
}

int gpu_bc_batched(tg_partition *p, const int32_t *sources, int32_t ns, hipStream_t s) {
  GpuPart &g = p->gpu;
  const Tuning &t = p->tune;
  if (!p->bcb) {
    p->bcb = new (std::nothrow) BcBatchState();
    if (!p->bcb) return set_error(TG_ENOMEM, "bc_batched: out of host memory");
  }
  BcBatchState &B = *p->bcb;
  const int64_t n = std::max<int64_t>(g.n, 1);
  if (B.n != g.n) {
    B.arena.release();
    TG_TRY(B.ws.ensure(g, 0));
    TG_TRY(dalloc(B.arena, &B.visited, (size_t)n));
    TG_TRY(dalloc(B.arena, &B.front[0], (size_t)n));
    TG_TRY(dalloc(B.arena, &B.front[1], (size_t)n));
    TG_TRY(dalloc(B.arena, &B.next, (size_t)n));
    TG_TRY(dalloc(B.arena, &B.lev, (size_t)n * S));
    TG_TRY(dalloc(B.arena, &B.sigma, (size_t)n * S));
    TG_TRY(dalloc(B.arena, &B.delta, (size_t)n * S));
    TG_TRY(dalloc(B.arena, &B.queue_all, (size_t)n * 64 + 1));
    // hub chunks of one level: at most (edges / 256 + hubs), hub_chunk >= 256
    TG_TRY(dalloc(B.arena, &B.hub_part, (size_t)(g.m / 256 + g.max_out_hubs + 1) * S));
    B.n = g.n;
  }
  Workspace &ws = B.ws;
  const unsigned fill_grid = 4096;
  for (int32_t c0 = 0; c0 < ns; c0 += S) {
    const int32_t cn = std::min<int32_t>(S, ns - c0);
    TG_HIP(hipMemsetAsync(B.visited, 0, (size_t)n * sizeof(u64), s));
    TG_HIP(hipMemsetAsync(B.front[0], 0, (size_t)n * sizeof(u64), s));
    TG_HIP(hipMemsetAsync(B.front[1], 0, (size_t)n * sizeof(u64), s));
    TG_HIP(hipMemsetAsync(B.next, 0, (size_t)n * sizeof(u64), s));
    TG_HIP(hipMemsetAsync(ws.bits_a, 0, ws.nwords * sizeof(uint32_t), s));
    hipLaunchKernelGGL(k_bb_fill<int32_t>, dim3(fill_grid), dim3(BLOCK), 0, s, B.lev, n * S, (int32_t)TG_INF);
    hipLaunchKernelGGL(k_bb_fill<double>, dim3(fill_grid), dim3(BLOCK), 0, s, B.sigma, n * S, 0.0);
    hipLaunchKernelGGL(k_bb_fill<float>, dim3(fill_grid), dim3(BLOCK), 0, s, B.delta, n * S, 0.0f);
    for (int32_t k = 0; k < cn; ++k)
      hipLaunchKernelGGL(k_bb_join, dim3(1), dim3(64), 0, s, B.next, ws.bits_a, B.sigma, p->h_l_of_g[sources[c0 + k]],
                         k);
    TG_HIP(hipGetLastError());
    // level 0: the sources
    std::vector<Plan> plans;
    std::vector<int64_t> segoff;
    int64_t off = 0;
    int cur = 0;
    TG_TRY(frontier_compact(g, ws, 1, ws.bits_a, nullptr, B.queue_all, nullptr, 0, s));
    TG_TRY(frontier_plan(g, ws, B.queue_all, t, s, false));
    hipLaunchKernelGGL(k_bb_finalize, dim3(nblk(std::min<int64_t>(n, 1 << 20))), dim3(BLOCK), 0, s, ws.plan,
                       B.queue_all, B.visited, B.front[cur], B.next, B.lev, 0);
    TG_HIP(hipMemcpyAsync(ws.h_plan, ws.plan, sizeof(Plan), hipMemcpyDeviceToHost, s));
    TG_HIP(hipStreamSynchronize(s));
    int32_t L = 0;
    for (;;) {
      if (L > g.n) return set_error(TG_EDEVICE, "bc_batched: more supersteps than vertices");
      const Plan P = *ws.h_plan;
      plans.push_back(P);
      segoff.push_back(off);
      const int64_t noff = off + P.count;
      if (noff + (int64_t)g.n > (int64_t)n * 64)
        return set_error(TG_EDEVICE, "bc_batched: level queues exceed their buffer");
      if (P.vb[NBIN] > 0)
        hipLaunchKernelGGL(k_bb_expand, dim3(launch_grid(P.vb[NBIN])), dim3(BLOCK), 0, s, ws.plan, B.queue_all + off,
                           ws.hubpref, g.out.off, g.out.col, B.front[cur], B.visited, B.next, ws.bits_a,
                           t.hub_chunk);
      TG_TRY(frontier_compact(g, ws, 1, ws.bits_a, nullptr, B.queue_all + noff, nullptr, 0, s));
      TG_TRY(frontier_plan(g, ws, B.queue_all + noff, t, s, false));
      hipLaunchKernelGGL(k_bb_finalize, dim3(nblk(std::min<int64_t>(n, 1 << 20))), dim3(BLOCK), 0, s, ws.plan,
                         B.queue_all + noff, B.visited, B.front[cur ^ 1], B.next, B.lev, L + 1);
      TG_HIP(hipMemcpyAsync(ws.h_plan, ws.plan, sizeof(Plan), hipMemcpyDeviceToHost, s));
      TG_HIP(hipStreamSynchronize(s));
      TG_HIP(hipGetLastError());
      if (ws.h_plan->count == 0) break;
      // the hub chunks of the sigma pull follow the in-edges
      if (!g.in_alias && ws.h_plan->pos[1] > 0) TG_TRY(frontier_plan_off(g, ws, B.queue_all + noff, g.in.off, t, s, false));
      const int tk = ktimer_start(s);
      TG_TRY(launch_sigma(g, ws, t, *ws.h_plan, B.queue_all + noff, B.front[cur], B.front[cur ^ 1], B.sigma,
                          ws.counters, B.hub_part, s));
      ktimer_stop(tk, s, "bcb_sigma");
      TG_HIP(hipMemsetAsync(B.front[cur], 0, (size_t)n * sizeof(u64), s));
      cur ^= 1;
      off = noff;
      ++L;
    }
    // backward: level L is the deepest reached; its dependencies stay 0
    for (int32_t lv = L - 1; lv >= 1; --lv) {
      if (plans[lv].pos[1] > 0) {
        // this level's plan back on the device, with the hub chunk prefix
        // of its queue over the out-edges
        TG_HIP(hipMemcpyAsync(ws.plan, &plans[lv], sizeof(Plan), hipMemcpyHostToDevice, s));
        TG_TRY(frontier_plan_off(g, ws, B.queue_all + segoff[lv], g.out.off, t, s, false));
      }
      const int tk = ktimer_start(s);
      TG_TRY(launch_delta(g, ws, t, plans[lv], B.queue_all + segoff[lv], B.lev, B.sigma, B.delta, p->ws.bc_acc, lv,
                          B.hub_part, s));
      ktimer_stop(tk, s, "bcb_delta");
      TG_HIP(hipGetLastError());
    }
    TG_HIP(hipMemcpyAsync(ws.h_flags, ws.counters, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    TG_HIP(hipStreamSynchronize(s));
    if (ws.h_flags[2]) return set_error(TG_ERANGE, "bc_batched: a shortest-path count reached 2^53");
  }
  return TG_OK;
}

}  // namespace tg

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
// and adds the row sum to its score.  One 256-thread block per vertex: its
// four wavefronts split the edge list and combine in LDS.
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
__global__ __launch_bounds__(BLOCK) void k_bb_sigma(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                    const int64_t *__restrict__ ioff, const int32_t *__restrict__ icol,
                                                    const u64 *__restrict__ front_old, const u64 *__restrict__ front_new,
                                                    double *sigma, uint32_t *flags) {
  __shared__ double red[BLOCK];
  const int32_t count = Pp->count;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
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
__global__ __launch_bounds__(BLOCK) void k_bb_delta(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                    const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                    const int32_t *__restrict__ lev, const double *__restrict__ sigma,
                                                    float *delta, double *score, int32_t level) {
  __shared__ double red[BLOCK];
  const int32_t count = Pp->count;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
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
      const int tk = ktimer_start(s);
      hipLaunchKernelGGL(k_bb_sigma, dim3((unsigned)std::min<int64_t>(ws.h_plan->count, 16384)), dim3(BLOCK), 0, s,
                         ws.plan, B.queue_all + noff, g.in.off, g.in.col, B.front[cur], B.front[cur ^ 1], B.sigma,
                         ws.counters);
      ktimer_stop(tk, s, "bcb_sigma");
      TG_HIP(hipMemsetAsync(B.front[cur], 0, (size_t)n * sizeof(u64), s));
      cur ^= 1;
      off = noff;
      ++L;
    }
    // backward: level L is the deepest reached; its dependencies stay 0
    for (int32_t lv = L - 1; lv >= 1; --lv) {
      TG_HIP(hipMemcpyAsync(ws.plan, &plans[lv], sizeof(Plan), hipMemcpyHostToDevice, s));
      const int tk = ktimer_start(s);
      hipLaunchKernelGGL(k_bb_delta, dim3((unsigned)std::min<int64_t>(std::max<int32_t>(plans[lv].count, 1), 16384)),
                         dim3(BLOCK), 0, s, ws.plan, B.queue_all + segoff[lv], g.out.off, g.out.col, B.lev, B.sigma,
                         B.delta, p->ws.bc_acc, lv);
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

// Multi-source supersteps: up to 64 independent BFS or SSSP queries ("slots")
// advance together over one GPU partition.  Each vertex carries one bit per
// slot (BFS: visited / frontier / next masks) or one distance per slot (SSSP),
// so a frontier vertex's edges are streamed once per superstep for every slot
// that has it on its frontier, instead of once per query.
//
// Slots are independent: a slot joins at any superstep boundary (its root
// enters the next frontier with level 0 at that superstep) and retires once
// its frontier is empty, which is what lets a server admit queries while
// others are running (continuous batching).  A superstep is:
//   expand(Q_t) -> clear(Q_t) -> compact(touched) = Q_{t+1} -> finalize(Q_{t+1})
// where "touched" marks vertices that received any slot bit this superstep.
#include <string.h>

#include <algorithm>

#include "slots.h"

using namespace tgk;

namespace tg {
namespace {

using u64 = unsigned long long;

inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>((n + BLOCK - 1) / BLOCK, 1); }

__device__ __forceinline__ void touch(uint32_t *touched, int32_t v) {
  atomicOr(touched + (v >> 5), 1u << (v & 31));
}

// BFS: new bits of a neighbour = frontier(v) & ~visited(n).
__global__ __launch_bounds__(BLOCK) void k_ms_bfs_expand(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                         const int64_t *__restrict__ hubpref,
                                                         const int64_t *__restrict__ off,
                                                         const int32_t *__restrict__ col, const u64 *frontier,
                                                         const u64 *visited, u64 *next, uint32_t *touched,
                                                         int64_t hub_chunk) {
  const Plan &P = load_plan(Pp);
  const int64_t total = P.vb[NBIN];
  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const Assign a = assign_work(vb, P, queue, nullptr, hubpref, off, hub_chunk);
    if (!a.ok) continue;
    const u64 m = frontier[a.v];
    if (m == 0) continue;
    for (int64_t e = a.e_begin + a.lane; e < a.e_end; e += a.stride) {
      const int32_t nb = stream_load(col + e);
      const u64 x = m & ~visited[nb];
      if (x) {
        const u64 old = atomicOr(next + nb, x);
        if (old == 0) touch(touched, nb);
      }
    }
  }
}

// SSSP: relax every slot on v's frontier mask; a lowered distance puts the
// slot on the neighbour's next mask.
__global__ __launch_bounds__(BLOCK) void k_ms_sssp_expand(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                          const int64_t *__restrict__ hubpref,
                                                          const int64_t *__restrict__ off,
                                                          const int32_t *__restrict__ col,
                                                          const int32_t *__restrict__ wgt, const u64 *frontier,
                                                          int32_t *dist, u64 *next, uint32_t *touched, u64 *ovf,
                                                          u64 *ovf_slots, int64_t hub_chunk) {
  const Plan &P = load_plan(Pp);
  const int64_t total = P.vb[NBIN];
  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const Assign a = assign_work(vb, P, queue, nullptr, hubpref, off, hub_chunk);
    if (!a.ok) continue;
    const u64 m = frontier[a.v];
    if (m == 0) continue;
    const int32_t *dv = dist + (int64_t)a.v * kSlots;
    for (int64_t e = a.e_begin + a.lane; e < a.e_end; e += a.stride) {
      const int32_t nb = stream_load(col + e);
      const int32_t w = stream_load(wgt + e);
      int32_t *dn = dist + (int64_t)nb * kSlots;
      u64 bits = m, gained = 0;
      while (bits) {
        const int s = __ffsll((long long)bits) - 1;
        bits &= bits - 1;
        const int64_t nd = (int64_t)dv[s] + (int64_t)w;
        if (nd >= (int64_t)TG_INF) {
          // the candidate does not fit: mark (vertex, slot); the slot's
          // verdict is taken when it retires (k_ms_ovf_check)
          if (dn[s] == TG_INF) {
            atomicOr(ovf + nb, 1ull << s);
            atomicOr(ovf_slots, 1ull << s);
          }
          continue;
        }
        if (nd < (int64_t)dn[s]) {
          const int32_t old = atomicMin(dn + s, (int32_t)nd);
          if (nd < (int64_t)old) gained |= 1ull << s;
        }
      }
      if (gained) {
        const u64 old = atomicOr(next + nb, gained);
        if (old == 0) touch(touched, nb);
      }
    }
  }
}

__global__ __launch_bounds__(BLOCK) void k_ms_clear(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                    u64 *frontier) {
  const int32_t count = Pp->count;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < count; i += (int64_t)gridDim.x * BLOCK)
    frontier[queue[i]] = 0;
}

// OR over the block, then one atomic per block into slot (block mod
// STAT_SLOTS) of `dst` (slots STAT_STRIDE words apart; the host ORs them).
__device__ __forceinline__ void block_or_into(u64 x, u64 *dst) {
  for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
  __shared__ u64 red[BLOCK / 64];
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 s = 0;
    for (int k = 0; k < BLOCK / 64; ++k) s |= red[k];
    if (s) atomicOr(dst + (size_t)(blockIdx.x & (STAT_SLOTS - 1)) * STAT_STRIDE, s);
  }
}

// BFS: settle the bits that arrived this superstep and write their levels.
__global__ __launch_bounds__(BLOCK) void k_ms_bfs_finalize(const Plan *__restrict__ Pp,
                                                           const int32_t *__restrict__ queue, u64 *visited,
                                                           u64 *frontier, u64 *next,
                                                           const int32_t *__restrict__ g_of_l, SlotTable tab,
                                                           int32_t step, u64 *alive) {
  const int32_t count = Pp->count;
  u64 any = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < count; i += (int64_t)gridDim.x * BLOCK) {
    const int32_t v = queue[i];
    const u64 nb = next[v] & ~visited[v];
    next[v] = 0;
    visited[v] |= nb;
    frontier[v] = nb;
    any |= nb;
    u64 bits = nb;
    const int32_t gv = g_of_l[v];
    while (bits) {
      const int s = __ffsll((long long)bits) - 1;
      bits &= bits - 1;
      tab.out[s][gv] = step - tab.join[s];
    }
  }
  block_or_into(any, alive);
}

// SSSP: the next frontier is whatever slot improved; distances stay in place.
__global__ __launch_bounds__(BLOCK) void k_ms_sssp_finalize(const Plan *__restrict__ Pp,
                                                            const int32_t *__restrict__ queue, u64 *frontier,
                                                            u64 *next, u64 *alive) {
  const int32_t count = Pp->count;
  u64 any = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < count; i += (int64_t)gridDim.x * BLOCK) {
    const int32_t v = queue[i];
    const u64 nb = next[v];
    next[v] = 0;
    frontier[v] = nb;
    any |= nb;
  }
  block_or_into(any, alive);
}

// A slot joins: its root gets the slot bit on the next frontier.
__global__ void k_ms_join(u64 *next, uint32_t *touched, int32_t *dist, int32_t root, int slot) {
  if (threadIdx.x != 0) return;
  atomicOr(next + root, 1ull << slot);
  touch(touched, root);
  if (dist) dist[(int64_t)root * kSlots + slot] = 0;
}

// Overflow verdict of retiring slots: bit s of *bad is set if some vertex
// received an overflowing candidate from slot s and stayed unreached (its
// true distance is finite but does not fit below INT32_MAX).  A vertex whose
// candidate overflowed but that was reached otherwise has its exact
// distance: path prefixes only grow, so an overflowing prefix never leads to
// a shorter path.
__global__ __launch_bounds__(BLOCK) void k_ms_ovf_check(const u64 *__restrict__ ovf, const int32_t *__restrict__ dist,
                                                        int64_t n, u64 mask, u64 *bad) {
  u64 found = 0;
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK) {
    u64 bits = ovf[v] & mask;
    while (bits) {
      const int s = __ffsll((long long)bits) - 1;
      bits &= bits - 1;
      if (dist[v * kSlots + s] == TG_INF) found |= 1ull << s;
    }
  }
  for (int o = 32; o > 0; o >>= 1) found |= __shfl_xor(found, o, 64);
  if ((threadIdx.x & 63) == 0 && found) atomicOr(bad, found);
}

// Retiring slots: drop their bits / reset their distances and overflow
// marks everywhere.
__global__ __launch_bounds__(BLOCK) void k_ms_release(u64 *visited, int32_t *dist, u64 *ovf, int64_t n, u64 mask) {
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK) {
    if (visited) visited[v] &= ~mask;
    if (ovf) ovf[v] &= ~mask;
    if (dist) {
      u64 bits = mask;
      while (bits) {
        const int s = __ffsll((long long)bits) - 1;
        bits &= bits - 1;
        dist[v * kSlots + s] = TG_INF;
      }
    }
  }
}

// SSSP result of one slot into its output (original ids).
__global__ __launch_bounds__(BLOCK) void k_ms_sssp_collect(const int32_t *__restrict__ dist, int64_t n, int slot,
                                                           const int32_t *__restrict__ g_of_l, int32_t *out) {
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK)
    out[g_of_l[v]] = dist[v * kSlots + slot];
}

__global__ void k_clear_bits64(u64 *word, u64 mask) {
  if (threadIdx.x == 0) atomicAnd(word, ~mask);
}

__global__ __launch_bounds__(BLOCK) void k_fill_i32_out(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) p[i] = v;
}

__global__ __launch_bounds__(BLOCK) void k_fill_i32_all(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) p[i] = v;
}

}  // namespace

SlotEngine::~SlotEngine() {
  if (h_alive) TG_QUIET(hipHostFree(h_alive));
  if (h_ovf) TG_QUIET(hipHostFree(h_ovf));
}

int SlotEngine::init(tg_partition *part, int kind_, hipStream_t stream) {
  p = part;
  kind = kind_;
  s = stream;
  const GpuPart &g = p->gpu;
  if (kind == kSlotSssp && !g.out.w) return set_error(TG_EUNSUPPORTED, "sssp: the graph was loaded without weights");
  arena.release();
  TG_TRY(ws.ensure(g, 0));
  const int64_t n = std::max<int64_t>(g.n, 1);
  TG_TRY(dalloc(arena, &frontier, (size_t)n));
  TG_TRY(dalloc(arena, &next, (size_t)n));
  TG_TRY(dalloc(arena, &alive, STAT_SPAN));
  TG_HIP(hipMemset(frontier, 0, (size_t)n * sizeof(u64)));
  TG_HIP(hipMemset(next, 0, (size_t)n * sizeof(u64)));
  if (kind == kSlotBfs) {
    TG_TRY(dalloc(arena, &visited, (size_t)n));
    TG_HIP(hipMemset(visited, 0, (size_t)n * sizeof(u64)));
  } else {
    TG_TRY(dalloc(arena, &ovf, (size_t)n));
    TG_TRY(dalloc(arena, &ovf_slots, 2));
    TG_HIP(hipMemset(ovf, 0, (size_t)n * sizeof(u64)));
    TG_HIP(hipMemset(ovf_slots, 0, 2 * sizeof(u64)));
    TG_TRY(dalloc(arena, &dist, (size_t)n * kSlots));
    hipLaunchKernelGGL(k_fill_i32_all, dim3(2048), dim3(BLOCK), 0, s, dist, n * kSlots, TG_INF);
    TG_HIP(hipGetLastError());
  }
  if (!h_alive) TG_HIP(hipHostMalloc((void **)&h_alive, STAT_SPAN * sizeof(u64), hipHostMallocDefault));
  if (!h_ovf) TG_HIP(hipHostMalloc((void **)&h_ovf, 2 * sizeof(u64), hipHostMallocDefault));
  TG_HIP(hipMemset(ws.bits_a, 0, ws.nwords * sizeof(uint32_t)));
  TG_HIP(hipMemset(ws.counters, 0, 64 * sizeof(uint32_t)));
  memset(&tab, 0, sizeof(tab));
  busy = 0;
  step = 0;
  have_queue = false;
  // the clears above are on the null stream, not ordered before work on a
  // non-blocking stream such as a server lane's
  TG_HIP(hipDeviceSynchronize());
  return TG_OK;
}

int SlotEngine::free_slot() const {
  for (int k = 0; k < kSlots; ++k)
    if (!((busy >> k) & 1ull)) return k;
  return -1;
}

int SlotEngine::join(int slot, int32_t root_local, int32_t *out_global) {
  const GpuPart &g = p->gpu;
  tab.out[slot] = out_global;
  // the root settles (level 0) in the next superstep, which first advances
  // the counter if a frontier is in flight
  tab.join[slot] = (int32_t)(have_queue ? step + 1 : step);
  busy |= 1ull << slot;
  if (kind == kSlotBfs && out_global)
    hipLaunchKernelGGL(k_fill_i32_out, dim3(nblk(std::min<int64_t>(g.n_global, 1 << 20))), dim3(BLOCK), 0, s,
                       out_global, g.n_global, TG_INF);
  hipLaunchKernelGGL(k_ms_join, dim3(1), dim3(64), 0, s, next, ws.bits_a, kind == kSlotSssp ? dist : nullptr,
                     root_local, slot);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int SlotEngine::superstep(u64 *finished) {
  TG_TRY(launch_step());
  return finish_step(finished);
}

int SlotEngine::launch_step() {
  const GpuPart &g = p->gpu;
  const Tuning &t = p->tune;
  if (have_queue && ws.h_plan->count > 0 && ws.h_plan->vb[NBIN] > 0) {
    const int grid = launch_grid(ws.h_plan->vb[NBIN]);
    const int tk = ktimer_start(s);
    if (kind == kSlotBfs)
      hipLaunchKernelGGL(k_ms_bfs_expand, dim3(grid), dim3(BLOCK), 0, s, ws.plan, ws.queue, ws.hubpref, g.out.off,
                         g.out.col, frontier, visited, next, ws.bits_a, t.hub_chunk);
    else
      hipLaunchKernelGGL(k_ms_sssp_expand, dim3(grid), dim3(BLOCK), 0, s, ws.plan, ws.queue, ws.hubpref,
                         g.out.off, g.out.col, g.out.w, frontier, dist, next, ws.bits_a, ovf, ovf_slots,
                         t.hub_chunk);
    ktimer_stop(tk, s, kind == kSlotBfs ? "msbfs_expand" : "mssssp_expand");
    hipLaunchKernelGGL(k_ms_clear, dim3(nblk(std::min<int64_t>(ws.h_plan->count, 1 << 20))), dim3(BLOCK), 0, s,
                       ws.plan, ws.queue, frontier);
    TG_HIP(hipGetLastError());
    ++step;
  } else if (have_queue) {
    ++step;
  }
  // next frontier: every vertex that received a slot bit (mode 1 takes and clears)
  TG_TRY(frontier_compact(g, ws, 1, ws.bits_a, nullptr, ws.queue, nullptr, 0, s));
  TG_TRY(frontier_plan(g, ws, ws.queue, t, s, false));
  TG_HIP(hipMemsetAsync(alive, 0, STAT_SPAN * sizeof(u64), s));
  const unsigned fgrid = nblk(std::min<int64_t>(g.n, 1 << 20));
  if (kind == kSlotBfs)
    hipLaunchKernelGGL(k_ms_bfs_finalize, dim3(fgrid), dim3(BLOCK), 0, s, ws.plan, ws.queue, visited, frontier, next,
                       g.g_of_l, tab, (int32_t)step, alive);
  else
    hipLaunchKernelGGL(k_ms_sssp_finalize, dim3(fgrid), dim3(BLOCK), 0, s, ws.plan, ws.queue, frontier, next, alive);
  TG_HIP(hipGetLastError());
  TG_HIP(hipMemcpyAsync(ws.h_plan, ws.plan, sizeof(Plan), hipMemcpyDeviceToHost, s));
  TG_HIP(hipMemcpyAsync(h_alive, alive, STAT_SPAN * sizeof(u64), hipMemcpyDeviceToHost, s));
  return TG_OK;
}

int SlotEngine::finish_step(u64 *finished) {
  TG_HIP(hipStreamSynchronize(s));
  ktimer_flush();
  have_queue = true;
  ++supersteps;
  // a busy slot with no bit on the new frontier has finished
  u64 any = 0;
  for (int i = 0; i < STAT_SLOTS; ++i) any |= h_alive[(size_t)i * STAT_STRIDE];
  *finished = busy & ~any;
  return TG_OK;
}

int SlotEngine::retire(u64 mask, u64 *overflow) {
  const GpuPart &g = p->gpu;
  if (overflow) *overflow = 0;
  if (!mask) return TG_OK;
  const unsigned grid = nblk(std::min<int64_t>(g.n, 1 << 20));
  if (kind == kSlotSssp) {
    for (int k = 0; k < kSlots; ++k)
      if ((mask >> k) & 1ull) {
        if (tab.out[k])
          hipLaunchKernelGGL(k_ms_sssp_collect, dim3(grid), dim3(BLOCK), 0, s, dist, g.n, k, g.g_of_l, tab.out[k]);
      }
    // slots that saw an overflowing candidate get the exact verdict
    TG_HIP(hipMemcpyAsync(h_ovf, ovf_slots, sizeof(u64), hipMemcpyDeviceToHost, s));
    TG_HIP(hipStreamSynchronize(s));
    const u64 flagged = h_ovf[0] & mask;
    if (flagged) {
      TG_HIP(hipMemsetAsync(ovf_slots + 1, 0, sizeof(u64), s));
      hipLaunchKernelGGL(k_ms_ovf_check, dim3(grid), dim3(BLOCK), 0, s, ovf, dist, g.n, flagged, ovf_slots + 1);
      hipLaunchKernelGGL(k_clear_bits64, dim3(1), dim3(64), 0, s, ovf_slots, flagged);
      TG_HIP(hipMemcpyAsync(h_ovf + 1, ovf_slots + 1, sizeof(u64), hipMemcpyDeviceToHost, s));
    }
    hipLaunchKernelGGL(k_ms_release, dim3(grid), dim3(BLOCK), 0, s, nullptr, dist, flagged ? ovf : nullptr, g.n,
                       mask);
    TG_HIP(hipGetLastError());
    TG_HIP(hipStreamSynchronize(s));
    if (flagged && overflow) *overflow = h_ovf[1] & flagged;
  } else {
    hipLaunchKernelGGL(k_ms_release, dim3(grid), dim3(BLOCK), 0, s, visited, nullptr, nullptr, g.n, mask);
    TG_HIP(hipGetLastError());
    TG_HIP(hipStreamSynchronize(s));
  }
  busy &= ~mask;
  for (int k = 0; k < kSlots; ++k)
    if ((mask >> k) & 1ull) tab.out[k] = nullptr;
  return TG_OK;
}

// Batched BFS / SSSP from a fixed list of roots: chunks of 64 slots that all
// join at superstep 0.
int slots_run_batch(tg_partition *p, int kind, const int32_t *roots, int32_t nr, int32_t *out, hipStream_t s,
                    int64_t *supersteps_out) {
  if (!p->slots[kind]) {
    p->slots[kind] = new (std::nothrow) SlotEngine();
    if (!p->slots[kind]) return set_error(TG_ENOMEM, "slot engine: out of host memory");
  }
  SlotEngine &E = *p->slots[kind];
  TG_TRY(E.init(p, kind, s));
  const int64_t V = p->g->n;
  int64_t total = 0;
  for (int32_t c0 = 0; c0 < nr; c0 += kSlots) {
    const int32_t cn = std::min<int32_t>(kSlots, nr - c0);
    for (int32_t k = 0; k < cn; ++k)
      TG_TRY(E.join(k, p->h_l_of_g[roots[c0 + k]], kind == kSlotBfs ? out + (int64_t)(c0 + k) * V : nullptr));
    u64 pending = E.busy;
    for (int64_t it = 0; pending; ++it) {
      if (it > p->gpu.n + 2) return set_error(TG_EDEVICE, "batched run: no convergence");
      u64 fin = 0;
      TG_TRY(E.superstep(&fin));
      if (fin) {
        if (kind == kSlotSssp)
          for (int k = 0; k < kSlots; ++k)
            if ((fin >> k) & 1ull) E.tab.out[k] = out + (int64_t)(c0 + k) * V;
        u64 ovf = 0;
        TG_TRY(E.retire(fin, &ovf));
        if (ovf) {
          const int k = __builtin_ctzll(ovf);
          return set_error(TG_ERANGE, "sssp_batched: the distances from root %d do not fit below INT32_MAX",
                           roots[c0 + k]);
        }
        pending &= ~fin;
      }
    }
    total += E.step;
    E.step = 0;
    E.have_queue = false;
  }
  if (supersteps_out) *supersteps_out = total;
  return TG_OK;
}

}  // namespace tg

// SSSP superstep: frontier Bellman-Ford (section 7.3, Figure 20).  Every
// active vertex relaxes its out-edges with an atomic minimum on the
// neighbour's distance; a neighbour whose distance dropped becomes active for
// the next superstep.  The run ends when no vertex is active.
//
// The atomic minimum returns nothing, so a lane never waits on it: a lane
// whose candidate beats the distance it read marks the neighbour active,
// whether or not its own minimum was the one that won.  The compaction keeps
// a marked vertex only if its distance is below the one it last relaxed with
// (`settled`), so every real improvement is expanded exactly as with a
// returned previous value, and stale marks are dropped.
//
// Per-XCD destination classes (tuning `sssp_xcd`): the out-edges are split by the
// 128-byte line of the destination's distance (class_csr.hip) and workgroups
// of XCD k relax only class k, so each XCD's L2 serves an eighth of the
// distance array.  Frontier vertices take lanes by the degree bin of
// ceil(deg / 8) (about one class row), hubs are chunked by their longest
// class row.
//
// Distances are int32 with INT32_MAX meaning unreachable.  A candidate
// distance >= INT32_MAX is never stored; the vertex is marked in an overflow
// bitmap instead, and the call fails with TG_ERANGE if such a vertex ends up
// without a finite distance (its true distance does not fit in int32).
#include <string.h>

#include <algorithm>
#include <atomic>
#include <string>
#include <thread>
#include <vector>

#include "tg_internal.h"

using namespace tgk;

namespace {

__global__ void k_set_i32(int32_t *p, int64_t i, int32_t v) {
  if (threadIdx.x == 0) p[i] = v;
}

// The next non-empty bitmap of the ring after bitmap `cur`: the blocks scan
// bitmaps cur+1, cur+2, ... (mod k) in turn, each block its share of every
// word range, and any[b] = 1 marks bitmap b as having a set bit (any zeroed
// before).  A block stops once a nearer bitmap is marked: then no later one
// can be the next.  Every block scans each bitmap up to and including the
// nearest non-empty one, so that one is always marked; marks beyond it may
// be missing, and the caller takes the nearest mark.
__global__ __launch_bounds__(BLOCK) void k_ring_next(const uint32_t *__restrict__ ring, int64_t nwords, int k,
                                                     int cur, uint32_t *any) {
  for (int j = 1; j < k; ++j) {
    bool nearer = false;
    if (threadIdx.x == 0)
      for (int m = 1; m < j; ++m)
        nearer |= __hip_atomic_load(any + (cur + m) % k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    if (__syncthreads_or(nearer)) return;
    const int b = (cur + j) % k;
    const uint32_t *bits = ring + (int64_t)b * nwords;
    uint32_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * BLOCK)
      acc |= bits[i];
    if (__syncthreads_or(acc != 0u) && threadIdx.x == 0)
      __hip_atomic_store(any + b, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Per vertex: how many of its packed out-edges (row sorted by weight) are
// lighter than delta (< 256), and how many are not.
__global__ void k_light_counts(const int64_t *__restrict__ off, const uint32_t *__restrict__ cw, int64_t n,
                               uint32_t bound, int32_t *__restrict__ lcnt, int32_t *__restrict__ hcnt) {
  const int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v >= n) return;
  int64_t lo = off[v], hi = off[v + 1];
  const int64_t b = lo, e = hi;
  while (lo < hi) {  // first word >= bound (weight >= delta)
    const int64_t mid = (lo + hi) >> 1;
    if (cw[mid] < bound) lo = mid + 1;
    else hi = mid;
  }
  lcnt[v] = (int32_t)(lo - b);
  hcnt[v] = (int32_t)(e - lo);
}

// Where an improved vertex is marked active: one bitmap, or (near/far with
// a bucket ring) bitmap (d / delta) mod k of the ring, nwords words apart.
struct ActiveSet {
  uint32_t *base;
  int32_t delta;
  int32_t k;  // 0: one bitmap
  int64_t nwords;
  __device__ __forceinline__ uint32_t *of(int32_t d) const {
    return k ? base + (int64_t)((d / delta) % k) * nwords : base;
  }
};

// Relax one edge.  `cur` is the neighbour's distance as this block knows it:
// an LDS snapshot for the hottest vertices (never below the true value, since
// distances only decrease) or the global value.
__device__ __forceinline__ void relax(int32_t *dist, int32_t *lds_d, int32_t hot, const ActiveSet &act, uint32_t *ovf,
                                      uint32_t *flags, int32_t dv, int32_t nb, int32_t wt, int32_t cur) {
  const int64_t nd = (int64_t)dv + (int64_t)wt;
  const uint32_t bit = 1u << (nb & 31);
  if (nd >= (int64_t)TG_INF) {
    // cannot improve a finite distance; matters only if nb stays unreached
    if (dist[nb] == TG_INF) {
      atomicOr(ovf + (nb >> 5), bit);
      flags[0] = 1u;
    }
    return;
  }
  if (nd < (int64_t)cur) {
    atomicMin(dist + nb, (int32_t)nd);  // no return value: nothing waits on it
    if (nb < hot) atomicMin(lds_d + nb, (int32_t)nd);
    atomicOr(act.of((int32_t)nd) + (nb >> 5), bit);
  }
}

__device__ __forceinline__ const int32_t *dist_ptr(const int32_t *dist, const int32_t *lds_d, int32_t hot, int32_t nb) {
  return nb < hot ? lds_d + nb : dist + nb;  // generic pointer: one load for LDS or HBM
}

// An edge's neighbour and weight: from the packed word (id | w << 24) or
// from the two arrays.
template <bool PACKED>
__device__ __forceinline__ void load_edge(const int32_t *__restrict__ col, const int32_t *__restrict__ wgt,
                                          const uint32_t *__restrict__ cw, int64_t e, int32_t &nb, int32_t &wt) {
  if (PACKED) {
    const uint32_t x = stream_load(cw + e);
    nb = (int32_t)(x & 0xFFFFFFu);
    wt = (int32_t)(x >> 24);
  } else {
    nb = stream_load(col + e);
    wt = stream_load(wgt + e);
  }
}

// Which edges of a frontier vertex relax: its whole row, or (packed rows,
// sorted by weight) its first lcnt[v] edges (lighter than the step) or the
// rest.
enum RelaxRange { ROW_ALL = 0, ROW_LIGHT = 1, ROW_HEAVY = 2 };

template <bool PACKED, int RANGE>
__global__ __launch_bounds__(BLOCK) void k_sssp_relax(const Plan *__restrict__ Pp,
                                                      const int32_t *__restrict__ queue,
                                                      const int64_t *__restrict__ hubpref,
                                                      const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ col,
                                                      const int32_t *__restrict__ wgt,
                                                      const uint32_t *__restrict__ cw, int32_t *dist,
                                                      const ActiveSet act, uint32_t *ovf, uint32_t *flags,
                                                      int64_t hub_chunk, unsigned long long *work, int32_t hot,
                                                      int vb_bin_lo, const int32_t *__restrict__ lcnt) {
  extern __shared__ int32_t lds_d[];
  for (int32_t i = threadIdx.x; i < hot; i += BLOCK) lds_d[i] = dist[i];
  const Plan &P = load_plan(Pp);  // (its barrier also publishes lds_d)
  const int64_t total = P.vb[NBIN];
  unsigned long long n_edges = 0, n_verts = 0;
  // virtual blocks of bins vb_bin_lo.. only
  for (int64_t vb = P.vb[vb_bin_lo] + blockIdx.x; vb < total; vb += gridDim.x) {
    const auto first = [off, lcnt](int32_t v) -> int64_t {
      return RANGE == ROW_HEAVY ? stream_load(off + v) + (int64_t)lcnt[v] : stream_load(off + v);
    };
    const auto last = [off, lcnt](int32_t v) -> int64_t {
      return RANGE == ROW_LIGHT ? stream_load(off + v) + (int64_t)lcnt[v] : stream_load(off + v + 1);
    };
    const Assign a = assign_work_range(vb, P, queue, nullptr, hubpref, first, last, hub_chunk);
    if (!a.ok) continue;
    if (a.lane == 0) {
      n_edges += (unsigned long long)(a.e_end - a.e_begin);
      n_verts += (a.bin != BIN_HUB || a.e_begin == first(a.v)) ? 1 : 0;
    }
    const int32_t dv = dist[a.v];
    const int64_t st = a.stride;
    int64_t e = a.e_begin + a.lane;
    // four edges per lane in flight: ids and weights, then the neighbours'
    // distances, then the (non-returning) atomics
    for (; e + 3 * st < a.e_end; e += 4 * st) {
      int32_t nb[4], wt[4], cur[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) load_edge<PACKED>(col, wgt, cw, e + k * st, nb[k], wt[k]);
#pragma unroll
      for (int k = 0; k < 4; ++k) cur[k] = *dist_ptr(dist, lds_d, hot, nb[k]);
#pragma unroll
      for (int k = 0; k < 4; ++k) relax(dist, lds_d, hot, act, ovf, flags, dv, nb[k], wt[k], cur[k]);
    }
    for (; e < a.e_end; e += st) {
      int32_t n0, w0;
      load_edge<PACKED>(col, wgt, cw, e, n0, w0);
      relax(dist, lds_d, hot, act, ovf, flags, dv, n0, w0, *dist_ptr(dist, lds_d, hot, n0));
    }
  }
  n_edges = block_sum(n_edges);
  n_verts = block_sum(n_verts);
  if (threadIdx.x == 0 && n_edges + n_verts > 0) {
    stat_add(stat_counter(work, 0), n_edges);
    stat_add(stat_counter(work, 1), n_verts);
  }
}

// The heavy edges of a settled bucket, pulled (symmetric graphs only: a
// vertex's out-edges are its in-edges, with the same weights).  The queue
// holds every vertex whose distance is not yet final; each takes the least
// dist[u] + w over its heavy edges from members u of the bucket.  A heavy
// candidate is at least the bucket's end, so final vertices could not gain
// and are skipped, which is what makes the pull cheaper than the push when
// the bucket's members hold more edges than the unsettled rest.  Each lane
// folds its share of a row and lowers the distance once, with the bit of the
// new distance's bucket set as a push relaxation would set it.
__global__ __launch_bounds__(BLOCK) void k_sssp_pull_heavy(const Plan *__restrict__ Pp,
                                                           const int32_t *__restrict__ queue,
                                                           const int64_t *__restrict__ hubpref,
                                                           const int64_t *__restrict__ off,
                                                           const uint32_t *__restrict__ cw,
                                                           const int32_t *__restrict__ lcnt, int32_t *dist,
                                                           const uint32_t *__restrict__ members, const ActiveSet act,
                                                           uint32_t *ovf, uint32_t *flags, int64_t hub_chunk,
                                                           unsigned long long *work) {
  const Plan &P = load_plan(Pp);
  const int64_t total = P.vb[NBIN];
  unsigned long long n_edges = 0, n_verts = 0;
  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const auto first = [off, lcnt](int32_t v) -> int64_t { return stream_load(off + v) + (int64_t)lcnt[v]; };
    const auto last = [off](int32_t v) -> int64_t { return stream_load(off + v + 1); };
    const Assign a = assign_work_range(vb, P, queue, nullptr, hubpref, first, last, hub_chunk);
    if (!a.ok) continue;
    if (a.lane == 0) {
      n_edges += (unsigned long long)(a.e_end - a.e_begin);
      n_verts += (a.bin != BIN_HUB || a.e_begin == first(a.v)) ? 1 : 0;
    }
    int64_t best = INT64_MAX;
    const int64_t st = a.stride;
    int64_t e = a.e_begin + a.lane;
    // four edges per lane in flight: words, then member bits, then the
    // members' distances
    for (; e + 3 * st < a.e_end; e += 4 * st) {
      uint32_t x[4], mw[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) x[k] = stream_load(cw + e + k * st);
#pragma unroll
      for (int k = 0; k < 4; ++k) mw[k] = members[(x[k] & 0xFFFFFFu) >> 5];
      int32_t du[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t u = x[k] & 0xFFFFFFu;
        du[k] = ((mw[k] >> (u & 31)) & 1u) ? dist[u] : TG_INF;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (du[k] < TG_INF) best = min(best, (int64_t)du[k] + (int64_t)(x[k] >> 24));
    }
    for (; e < a.e_end; e += st) {
      const uint32_t x = stream_load(cw + e);
      const uint32_t u = x & 0xFFFFFFu;
      if ((members[u >> 5] >> (u & 31)) & 1u) {
        const int32_t du = dist[u];
        if (du < TG_INF) best = min(best, (int64_t)du + (int64_t)(x >> 24));
      }
    }
    if (best == INT64_MAX) continue;
    const int32_t v = a.v;
    const uint32_t bit = 1u << (v & 31);
    const int32_t cur = dist[v];
    if (best >= (int64_t)TG_INF) {
      // cannot improve a finite distance; matters only if v stays unreached
      if (cur == TG_INF) {
        atomicOr(ovf + (v >> 5), bit);
        flags[0] = 1u;
      }
    } else if (best < (int64_t)cur) {
      atomicMin(dist + v, (int32_t)best);
      atomicOr(act.of((int32_t)best) + (v >> 5), bit);
    }
  }
  n_edges = block_sum(n_edges);
  n_verts = block_sum(n_verts);
  if (threadIdx.x == 0 && n_edges + n_verts > 0) {
    stat_add(stat_counter(work, 2), n_edges);
    stat_add(stat_counter(work, 3), n_verts);
  }
}

// One class per XCD: workgroup i relaxes class (i mod 8) of every frontier
// vertex's out-edges.
__global__ __launch_bounds__(BLOCK) void k_sssp_relax_cls(const Plan *__restrict__ Pp,
                                                          const int32_t *__restrict__ queue,
                                                          const int64_t *__restrict__ hubpref,
                                                          const int32_t *__restrict__ soff, tg::ClassBase cb,
                                                          const int32_t *__restrict__ scol,
                                                          const int32_t *__restrict__ sw, int64_t n, int32_t *dist,
                                                          uint32_t *active, uint32_t *ovf, uint32_t *flags,
                                                          int64_t hub_chunk, unsigned long long *work,
                                                          int vb_bin_hi) {
  const Plan &P = load_plan(Pp);
  const int k = (int)(blockIdx.x & 7);
  const int64_t jb = blockIdx.x >> 3, nb = gridDim.x >> 3;
  const int32_t *so = soff + (int64_t)k * (n + 1);
  const int64_t base = cb.base[k];
  const int64_t total = P.vb[vb_bin_hi];  // virtual blocks of bins ..vb_bin_hi-1 only
  unsigned long long n_edges = 0, n_verts = 0;
  for (int64_t vb = jb; vb < total; vb += nb) {
    const Assign a = assign_work_rows(vb, P, queue, nullptr, hubpref,
                                      [so, base](int64_t i) { return base + (int64_t)stream_load(so + i); },
                                      hub_chunk);
    if (!a.ok || a.e_begin >= a.e_end) continue;
    if (a.lane == 0) {
      n_edges += (unsigned long long)(a.e_end - a.e_begin);
      n_verts += (k == 0 && (a.bin != BIN_HUB || a.e_begin == base + so[a.v])) ? 1 : 0;
    }
    const int32_t dv = dist[a.v];
    const int64_t st = a.stride;
    int64_t e = a.e_begin + a.lane;
    for (; e + 3 * st < a.e_end; e += 4 * st) {
      int32_t nb4[4], wt[4], cur[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        nb4[q] = stream_load(scol + e + q * st);
        wt[q] = stream_load(sw + e + q * st);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) cur[q] = dist[nb4[q]];
#pragma unroll
      for (int q = 0; q < 4; ++q) relax(dist, nullptr, 0, ActiveSet{active, 0, 0, 0}, ovf, flags, dv, nb4[q], wt[q], cur[q]);
    }
    for (; e < a.e_end; e += st) {
      const int32_t n0 = stream_load(scol + e);
      relax(dist, nullptr, 0, ActiveSet{active, 0, 0, 0}, ovf, flags, dv, n0, stream_load(sw + e), dist[n0]);
    }
  }
  n_edges = block_sum(n_edges);
  n_verts = block_sum(n_verts);
  if (threadIdx.x == 0 && n_edges + n_verts > 0) {
    stat_add(stat_counter(work, 0), n_edges);
    stat_add(stat_counter(work, 1), n_verts);
  }
}

// flags[1] = 1 if some vertex with an overflowing candidate stayed unreached
__global__ __launch_bounds__(BLOCK) void k_overflow_check(const uint32_t *__restrict__ ovf,
                                                          const int32_t *__restrict__ dist, int64_t n,
                                                          uint32_t *flags) {
  const int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v >= n) return;
  if (((ovf[v >> 5] >> (v & 31)) & 1u) && dist[v] == TG_INF) flags[1] = 1u;
}

}  // namespace

namespace tg {

int sssp_relax_launch(const GpuPart &g, Workspace &ws, const int32_t *queue, int64_t vblocks, const Tuning &t,
                      hipStream_t s, int32_t bucket_delta, int32_t bucket_k, int range) {
  if (vblocks <= 0) return TG_OK;
  const int32_t hot = (int32_t)std::min<int64_t>(t.sssp_lds_verts, g.n);
  const int grid = hot > 0 ? (int)std::min<int64_t>(launch_grid(vblocks), t.sssp_grid) : launch_grid(vblocks);
  // improved vertices: the active bitmap, or the bucket ring of their new distance
  const ActiveSet act = bucket_k > 0 ? ActiveSet{ws.buckets, bucket_delta, bucket_k, ws.nwords}
                                     : ActiveSet{ws.bits_a, 0, 0, 0};
  const size_t lds = (size_t)hot * sizeof(int32_t);
  const int tk = ktimer_start(s);
  if (range == ROW_LIGHT || range == ROW_HEAVY) {
    // the split needs the packed rows sorted by weight and the light counts
    if (!g.out.cw || !g.lcnt) return set_error(TG_EDEVICE, "sssp: light/heavy relaxation without packed rows");
    if (range == ROW_LIGHT)
      hipLaunchKernelGGL((k_sssp_relax<true, ROW_LIGHT>), dim3(grid), dim3(BLOCK), lds, s, ws.plan, queue,
                         ws.hubpref, g.out.off, g.out.col, g.out.w, g.out.cw, ws.state, act, ws.bits_c, ws.counters,
                         t.hub_chunk, ws.work, hot, 0, g.lcnt);
    else
      hipLaunchKernelGGL((k_sssp_relax<true, ROW_HEAVY>), dim3(grid), dim3(BLOCK), lds, s, ws.plan, queue,
                         ws.hubpref, g.out.off, g.out.col, g.out.w, g.out.cw, ws.state, act, ws.bits_c, ws.counters,
                         t.hub_chunk, ws.work, hot, 0, g.lcnt);
  } else if (t.sssp_packed && g.out.cw) {
    hipLaunchKernelGGL((k_sssp_relax<true, ROW_ALL>), dim3(grid), dim3(BLOCK), lds, s, ws.plan, queue, ws.hubpref,
                       g.out.off, g.out.col, g.out.w, g.out.cw, ws.state, act, ws.bits_c, ws.counters, t.hub_chunk,
                       ws.work, hot, 0, nullptr);
  } else {
    hipLaunchKernelGGL((k_sssp_relax<false, ROW_ALL>), dim3(grid), dim3(BLOCK), lds, s, ws.plan, queue, ws.hubpref,
                       g.out.off, g.out.col, g.out.w, g.out.cw, ws.state, act, ws.bits_c, ws.counters, t.hub_chunk,
                       ws.work, hot, 0, nullptr);
  }
  ktimer_stop(tk, s, "sssp_relax");
  TG_HIP(hipGetLastError());
  return TG_OK;
}

// The pull form of a bucket's heavy pass over the queue of unsettled
// vertices (k_sssp_pull_heavy); `members` is the bucket's member bitmap.
int sssp_pull_heavy_launch(const GpuPart &g, Workspace &ws, const int32_t *queue, int64_t vblocks,
                           const uint32_t *members, const Tuning &t, hipStream_t s, int32_t bucket_delta,
                           int32_t bucket_k) {
  if (vblocks <= 0) return TG_OK;
  if (!g.out.cw || !g.lcnt || !g.in_alias)
    return set_error(TG_EDEVICE, "sssp: heavy pull needs packed rows, light counts and a symmetric graph");
  const ActiveSet act{ws.buckets, bucket_delta, bucket_k, ws.nwords};
  const int tk = ktimer_start(s);
  hipLaunchKernelGGL(k_sssp_pull_heavy, dim3(launch_grid(vblocks)), dim3(BLOCK), 0, s, ws.plan, queue, ws.hubpref,
                     g.out.off, g.out.cw, g.lcnt, ws.state, members, act, ws.bits_c, ws.counters, t.hub_chunk,
                     ws.work);
  ktimer_stop(tk, s, "sssp_pull");
  TG_HIP(hipGetLastError());
  return TG_OK;
}

// After the last superstep: ws.h_flags[1] = 1 iff some vertex had an
// overflowing candidate distance and stayed unreached.  Waits on `s`.
int sssp_overflow_check(const GpuPart &g, Workspace &ws, hipStream_t s) {
  TG_HIP(hipMemcpyAsync(ws.h_flags, ws.counters, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  if (ws.h_flags[0] && g.n > 0) {
    hipLaunchKernelGGL(k_overflow_check, dim3((unsigned)((g.n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s,
                       ws.bits_c, ws.state, g.n, ws.counters);
    TG_HIP(hipGetLastError());
    TG_HIP(hipMemcpyAsync(ws.h_flags, ws.counters, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    TG_HIP(hipStreamSynchronize(s));
  }
  return TG_OK;
}

struct SsspSlices {
  ClassCsr cc;               // out-edges and weights by destination class
  int32_t *maxlen = nullptr; // per vertex: its longest class row (hub chunking)
  DevArena arena;
  BinBounds bins{};          // bins of ceil(deg / 8) over the degree-sorted ids
  Tuning built_for{};
  bool built = false;
};

void sssp_slices_free(GpuPart &g) {
  delete g.sslices;
  g.sslices = nullptr;
}

int build_sssp_slices(tg_partition *p, hipStream_t s) {
  GpuPart &g = p->gpu;
  const Tuning &t = p->tune;
  if (g.sslices && g.sslices->built) {
    // the bins follow the tuning's thresholds
    if (memcmp(g.sslices->built_for.min_deg, t.min_deg, sizeof(t.min_deg)) != 0) {
      g.sslices->bins = BinBounds{};
      const int64_t n = g.n;
      int64_t i = 0;
      for (int b = 0; b < NBIN; ++b) {
        while (i < n && bin_of_degree((g.h_deg[i] + 7) / 8, t) < b) ++i;
        g.sslices->bins.bstart[b] = i;
      }
      g.sslices->bins.bstart[NBIN] = n;
      g.sslices->built_for = t;
    }
    return TG_OK;
  }
  sssp_slices_free(g);
  g.sslices = new (std::nothrow) SsspSlices();
  if (!g.sslices) return set_error(TG_ENOMEM, "sssp: out of host memory");
  SsspSlices &S = *g.sslices;
  const int64_t n = g.n;
  std::vector<int32_t> hsoff, hcnt;
  TG_TRY(build_class_csr(g.out.off, g.out.col, g.out.w, n, g.m, S.cc, hsoff, hcnt, s));
  std::vector<int32_t> ml((size_t)std::max<int64_t>(n, 1), 0);
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    int32_t m = 0;
    for (int k = 0; k < 8; ++k) m = std::max(m, hcnt[(size_t)k * n + v]);
    ml[v] = m;
  }
  TG_TRY(dalloc(S.arena, &S.maxlen, ml.size()));
  TG_HIP(hipMemcpy(S.maxlen, ml.data(), ml.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  TG_HIP(hipDeviceSynchronize());  // the copy is on the null stream
  int64_t i = 0;
  for (int b = 0; b < NBIN; ++b) {
    while (i < n && bin_of_degree((g.h_deg[i] + 7) / 8, t) < b) ++i;
    S.bins.bstart[b] = i;
  }
  S.bins.bstart[NBIN] = n;
  S.built_for = t;
  S.built = true;
  return TG_OK;
}

// Class mode: vertices of the HUB, BLOCK and WAVE bins (about a wave or more
// per class row) relax through the per-XCD classes; the lower bins, whose
// rows are too short to split eight ways, relax their whole rows in one pass.
static int sssp_relax_cls_launch(const GpuPart &g, Workspace &ws, const int32_t *queue, const Plan &hp,
                                 const Tuning &t, hipStream_t s) {
  const SsspSlices &S = *g.sslices;
  const int64_t vb_hi = hp.vb[BIN_G16], vb_lo_n = hp.vb[NBIN] - hp.vb[BIN_G16];
  const int tk = ktimer_start(s);
  if (vb_hi > 0) {
    // every class walks every virtual block: up to sssp_grid blocks per class
    const int grid = (int)(8 * std::min<int64_t>(vb_hi, std::max<int64_t>(t.sssp_grid, 1)));
    hipLaunchKernelGGL(k_sssp_relax_cls, dim3(grid), dim3(BLOCK), 0, s, ws.plan, queue, ws.hubpref, S.cc.soff,
                       S.cc.cb, S.cc.scol, S.cc.sw, g.n, ws.state, ws.bits_a, ws.bits_c, ws.counters, t.hub_chunk,
                       ws.work, (int)BIN_G16);
  }
  if (vb_lo_n > 0)
    hipLaunchKernelGGL((k_sssp_relax<false, ROW_ALL>), dim3(launch_grid(vb_lo_n)), dim3(BLOCK), 0, s, ws.plan,
                       queue, ws.hubpref, g.out.off, g.out.col, g.out.w, g.out.cw, ws.state,
                       ActiveSet{ws.bits_a, 0, 0, 0}, ws.bits_c, ws.counters, t.hub_chunk, ws.work, 0, (int)BIN_G16,
                       nullptr);
  ktimer_stop(tk, s, "sssp_relax");
  TG_HIP(hipGetLastError());
  return TG_OK;
}

namespace {

// Whether the ring schedule splits rows into light and heavy parts.
bool sssp_split_on(const tg_partition *p) {
  const Tuning &t = p->tune;
  return t.sssp_split && t.sssp_packed && p->gpu.out.cw && t.sssp_delta > 0 && t.sssp_delta < 256;
}

// The near/far schedule over a ring of k bucket bitmaps (see gpu_sssp).
// Distances, settled values and overflow marks are set up by the caller.
// With the light/heavy split (Meyer and Sanders' delta-stepping): while a
// bucket is processed its vertices relax only their edges lighter than
// delta, which may land in the same bucket; once it is empty its members'
// distances are final and each relaxes its heavy edges once, into later
// buckets.
int gpu_sssp_ring(tg_partition *p, Workspace &ws, int32_t root, hipStream_t s, int32_t k, int64_t *rounds_out,
                  int64_t *pulls_out) {
  GpuPart &g = p->gpu;
  const int64_t delta = p->tune.sssp_delta;
  const bool split = sssp_split_on(p) && g.lcnt && g.split_delta == delta;
  const BinBounds &bb = split ? g.light_bins : g.out_bins;
  // heavy passes may pull (symmetric graphs): then the vertices whose
  // distance is final are tracked too
  const bool hpull = split && g.in_alias && p->tune.sssp_hpull > 0;
  const int kb = k + (split ? 1 : 0) + (hpull ? 1 : 0);  // the bucket's members, then the final set, after the ring
  if (!ws.buckets || ws.buckets_k < kb) {
    TG_TRY(dalloc(ws.arena, &ws.buckets, (size_t)kb * ws.nwords));
    ws.buckets_k = kb;
  }
  uint32_t *members = split ? ws.buckets + (int64_t)k * ws.nwords : nullptr;
  uint32_t *done = hpull ? ws.buckets + (int64_t)(k + 1) * ws.nwords : nullptr;
  int64_t done_deg = 0, hpulls = 0;  // out-degree sum of the final set; pulled heavy passes
  TG_HIP(hipMemsetAsync(ws.buckets, 0, (size_t)kb * ws.nwords * sizeof(uint32_t), s));
  TG_TRY(set_bit(ws.buckets, root, s));  // bucket 0: distance 0
  int64_t lo = 0, rounds = 0;
  for (;;) {
    if (rounds > 4 * g.n + 4 || lo > (int64_t)TG_INF)
      return set_error(TG_EDEVICE, "sssp: no convergence after %lld rounds", (long long)rounds);
    uint32_t *bits = ws.buckets + ((lo / delta) % k) * ws.nwords;
    // every unsettled bit of the current bucket is in [lo, lo + delta): all are taken
    // (with the split, a vertex without light edges joins the bucket's
    // members but not the light pass)
    TG_TRY(frontier_compact_sssp(g, ws, bits, ws.queue, ws.state, ws.settled, TG_INF, false, bb, s, nullptr,
                                 members, split ? g.lcnt : nullptr));
    TG_TRY(frontier_plan_bins(g, ws, ws.queue, bb, split ? g.lcnt : nullptr, p->tune, s, true));
    if (ws.h_plan->count > 0) {
      ++rounds;
      TG_TRY(sssp_relax_launch(g, ws, ws.queue, ws.h_plan->vb[NBIN], p->tune, s, (int32_t)delta, k,
                               split ? 1 : 0));
      continue;
    }
    if (hpull) {
      // the bucket is settled: its members' heavy edges are relaxed once,
      // pushed from the members or pulled by the vertices not yet final,
      // whichever side holds fewer edges (out-degree sums; the pull's
      // weighted by sssp_hpull percent)
      TG_TRY(stat_zero(ws, 4, s));
      TG_TRY(frontier_compact_bucket_end(g, ws, members, done, false, ws.queue, stat_counter(ws.work, 4), s));
      TG_TRY(stat_fetch(ws, 4, s));
      TG_TRY(frontier_plan_bins(g, ws, ws.queue, g.out_bins, g.hcnt, p->tune, s, true));
      const int64_t push_deg = (int64_t)stat_sum(ws, 4);
      const int64_t pull_deg = g.m - done_deg - push_deg;
      done_deg += push_deg;
      if (ws.h_plan->count > 0 && pull_deg * 100 < push_deg * (int64_t)p->tune.sssp_hpull) {
        TG_TRY(frontier_compact_bucket_end(g, ws, members, done, true, ws.queue, nullptr, s));
        TG_TRY(frontier_plan_bins(g, ws, ws.queue, g.out_bins, g.hcnt, p->tune, s, true));
        if (ws.h_plan->count > 0) {
          ++rounds;
          ++hpulls;
          TG_TRY(sssp_pull_heavy_launch(g, ws, ws.queue, ws.h_plan->vb[NBIN], members, p->tune, s, (int32_t)delta,
                                        k));
        }
      } else if (ws.h_plan->count > 0) {
        ++rounds;
        TG_TRY(sssp_relax_launch(g, ws, ws.queue, ws.h_plan->vb[NBIN], p->tune, s, (int32_t)delta, k, 2));
      }
      TG_TRY(bitmap_merge_clear(ws, done, members, s));
    } else if (split) {
      // the bucket is settled: its members relax their heavy edges once
      TG_TRY(frontier_compact(g, ws, 1, members, nullptr, ws.queue, nullptr, 0, s));
      TG_TRY(frontier_plan_bins(g, ws, ws.queue, g.out_bins, g.hcnt, p->tune, s, true));
      if (ws.h_plan->count > 0) {
        ++rounds;
        TG_TRY(sssp_relax_launch(g, ws, ws.queue, ws.h_plan->vb[NBIN], p->tune, s, (int32_t)delta, k, 2));
      }
    }
    // the current bucket is empty: move to the next bucket with a set bit,
    // if any (the ring holds every active vertex)
    const int64_t cur = (lo / delta) % k;
    TG_HIP(hipMemsetAsync(ws.counters + 16, 0, (size_t)k * sizeof(uint32_t), s));
    const unsigned bx = (unsigned)std::min<int64_t>((ws.nwords + 8 * BLOCK - 1) / (8 * BLOCK), 512);
    hipLaunchKernelGGL(k_ring_next, dim3(bx), dim3(BLOCK), 0, s, ws.buckets, ws.nwords, (int)k, (int)cur,
                       ws.counters + 16);
    TG_HIP(hipGetLastError());
    TG_HIP(hipMemcpyAsync(ws.h_flags + 16, ws.counters + 16, (size_t)k * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    TG_HIP(hipStreamSynchronize(s));
    int64_t step = 0;
    for (int64_t j = 1; j < k && step == 0; ++j)
      if (ws.h_flags[16 + (cur + j) % k]) step = j;
    if (step == 0) break;  // no active vertex left
    lo += step * delta;
  }
  if (pulls_out) *pulls_out = hpulls;
  TG_TRY(sssp_overflow_check(g, ws, s));
  if (ws.h_flags[1]) return set_error(TG_ERANGE, "sssp: a shortest-path distance does not fit below INT32_MAX");
  if (rounds_out) *rounds_out = rounds;
  return TG_OK;
}

}  // namespace

// Light counts and light-degree bins for the split at the current step
// (once per partition and step, before lanes share them).  The bins place
// vertex v by its expected light degree, deg(v) times the graph's share of
// light edges (at least 1 for a vertex with edges): a contiguous id range
// per bin, as the compaction needs.
int sssp_split_prepare(tg_partition *p, hipStream_t s) {
  GpuPart &g = p->gpu;
  const Tuning &t = p->tune;
  if (!sssp_split_on(p) || g.split_delta == t.sssp_delta) return TG_OK;
  const int64_t n = g.n;
  if (!g.lcnt) {
    TG_TRY(dalloc(p->arena, &g.lcnt, (size_t)std::max<int64_t>(n, 1)));
    TG_TRY(dalloc(p->arena, &g.hcnt, (size_t)std::max<int64_t>(n, 1)));
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_light_counts, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, g.out.off,
                       g.out.cw, n, (uint32_t)t.sssp_delta << 24, g.lcnt, g.hcnt);
    TG_HIP(hipGetLastError());
  }
  std::vector<int32_t> lc((size_t)n);
  if (n > 0) TG_HIP(hipMemcpyAsync(lc.data(), g.lcnt, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  double light = 0;
  for (int32_t c : lc) light += c;
  const double frac = g.m > 0 ? light / (double)g.m : 0.0;
  int64_t i = 0;
  BinBounds bb{};
  // at least one: the degree-0 bin gets no work, and a vertex with edges
  // may have light ones whatever its expected count
  const auto light_deg = [&](int64_t i) {
    const int64_t d = g.h_deg[i];
    return d > 0 ? std::max<int64_t>(1, (int64_t)((double)d * frac + 0.5)) : (int64_t)0;
  };
  for (int b = 0; b < NBIN; ++b) {
    while (i < n && bin_of_degree(light_deg(i), t) < b) ++i;
    bb.bstart[b] = i;
  }
  bb.bstart[NBIN] = n;
  g.light_bins = bb;
  g.split_delta = t.sssp_delta;
  return TG_OK;
}

int gpu_sssp(tg_partition *p, Workspace &ws, int32_t root, hipStream_t s, int64_t *rounds_out, int64_t *pulls_out) {
  GpuPart &g = p->gpu;
  if (!g.out.w) return set_error(TG_EUNSUPPORTED, "sssp: the graph was loaded without weights");
  TG_TRY(ws.ensure(g, 0));
  uint32_t *active = ws.bits_a, *ovf = ws.bits_c;
  int32_t *dist = ws.state;
  TG_TRY(fill_i32(dist, g.n, TG_INF, s));
  TG_TRY(fill_i32(ws.settled, g.n, TG_INF, s));
  hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(64), 0, s, dist, (int64_t)root, 0);
  TG_HIP(hipMemsetAsync(active, 0, ws.nwords * sizeof(uint32_t), s));
  TG_HIP(hipMemsetAsync(ovf, 0, ws.nwords * sizeof(uint32_t), s));
  TG_HIP(hipMemsetAsync(ws.counters, 0, 4 * sizeof(uint32_t), s));
  TG_TRY(set_bit(active, root, s));
  int64_t rounds = 0;
  const int64_t delta = p->tune.sssp_delta;
  const bool cls = p->tune.sssp_xcd != 0;
  if (cls) TG_TRY(build_sssp_slices(p, s));
  const BinBounds &bb = cls ? g.sslices->bins : g.out_bins;
  const int32_t *len = cls ? g.sslices->maxlen : nullptr;
  // near/far over a ring of bucket bitmaps (plain push steps): while the
  // bucket of distances [lo, lo + delta) is processed, a relaxation yields at
  // most lo + delta - 1 + max_w, so every active vertex lies within
  // ceil((max_w + 1) / delta) + 1 buckets of lo and bitmap (d / delta) mod k
  // of a ring of that many holds it; a superstep filters only the current
  // bucket, and the ones beyond wait untouched
  const int64_t ring_k = delta > 0 ? (g.max_w + 1 + delta - 1) / delta + 1 : 0;
  if (p->tune.sssp_ring && delta > 0 && !cls && !(p->tune.sssp_pull > 0 && sssp_pull_supported(g)) && ring_k <= 16)
    return gpu_sssp_ring(p, ws, root, s, (int32_t)ring_k, rounds_out, pulls_out);
  int64_t thresh = delta;  // near/far: only active vertices below thresh relax
  // pull supersteps for frontiers with a large share of the edges: the
  // compaction sums the frontier's out-degrees (spread counter 4)
  const bool pull = p->tune.sssp_pull > 0 && !cls && sssp_pull_supported(g);
  unsigned long long *degsum = pull ? stat_counter(ws.work, 4) : nullptr;
  int64_t pulls = 0;
  for (;; ++rounds) {
    // a frontier Bellman-Ford settles within |V| - 1 rounds (per threshold step)
    if (rounds > 2 * g.n + 2) return set_error(TG_EDEVICE, "sssp: no convergence after %lld rounds", (long long)rounds);
    if (pull) TG_TRY(stat_zero(ws, 4, s));
    if (delta <= 0) {
      TG_TRY(frontier_compact_sssp(g, ws, active, ws.queue, dist, ws.settled, TG_INF, false, bb, s, degsum));
      if (pull) TG_TRY(stat_fetch(ws, 4, s));
      TG_TRY(frontier_plan_bins(g, ws, ws.queue, bb, len, p->tune, s, true));
      if (ws.h_plan->count == 0) break;
    } else {
      TG_TRY(frontier_compact_sssp(g, ws, active, ws.queue, dist, ws.settled,
                                   (int32_t)std::min<int64_t>(thresh, TG_INF), true, bb, s, degsum));
      TG_TRY(stat_fetch(ws, 5, s));
      TG_TRY(stat_fetch(ws, 6, s));
      if (pull) TG_TRY(stat_fetch(ws, 4, s));
      TG_TRY(frontier_plan_bins(g, ws, ws.queue, bb, len, p->tune, s, true));
      if (ws.h_plan->count == 0) {
        if (stat_sum(ws, 5) == 0) break;  // nothing left beyond the threshold either
        // jump to the least distance still waiting
        unsigned long long m = ~0ull;
        const unsigned long long *mins = stat_counter(ws.h_stat, 6);
        for (int i = 0; i < STAT_SLOTS; ++i) m = std::min(m, mins[(size_t)i * STAT_STRIDE]);
        thresh = (int64_t)m + delta;
        continue;
      }
    }
    if (pull && (double)stat_sum(ws, 4) * 100.0 > (double)p->tune.sssp_pull * (double)g.m) {
      // the taken frontier is in ws.bits_b (the compaction's filtered set)
      TG_TRY(sssp_pull_launch(p, ws, ws.bits_b, s));
      ++pulls;
    } else if (cls) {
      TG_TRY(sssp_relax_cls_launch(g, ws, ws.queue, *ws.h_plan, p->tune, s));
    } else {
      TG_TRY(sssp_relax_launch(g, ws, ws.queue, ws.h_plan->vb[NBIN], p->tune, s));
    }
  }
  if (pulls_out) *pulls_out = pulls;
  TG_TRY(sssp_overflow_check(g, ws, s));
  if (ws.h_flags[1]) return set_error(TG_ERANGE, "sssp: a shortest-path distance does not fit below INT32_MAX");
  if (rounds_out) *rounds_out = rounds;
  return TG_OK;
}

namespace {

struct LaneResult {
  int rc = TG_OK;
  std::string msg;
  int64_t rounds = 0, pulls = 0;
  unsigned long long relax = 0, act = 0, pull_checks = 0, pull_verts = 0;
  KTimes timers;
};

// One lane: searches from the shared root counter until none is left or a
// search fails, each collected into its row of dist.
void sssp_lane(tg_partition *p, int lane, hipStream_t s, const int32_t *roots_local, int32_t nr, int32_t *dist,
               std::atomic<int32_t> *next, std::atomic<bool> *failed, LaneResult *res, hipEvent_t ref) {
  if (lane > 0) {
    ktimer_reset();
    ktimer_set_ref(ref);
  }
  auto run = [&]() -> int {
    if (hipSetDevice(p->device) != hipSuccess) return set_error(TG_EDEVICE, "sssp: hipSetDevice failed");
    Workspace *ws = nullptr;
    TG_TRY(lane_workspace(p, lane, &ws));
    TG_TRY(ws->ensure(p->gpu, 0));
    TG_TRY(stat_zero_all(*ws, s));
    const int64_t V = p->gpu.n_global;
    while (!failed->load()) {
      const int32_t r = next->fetch_add(1);
      if (r >= nr) break;
      int64_t rounds = 0, pulls = 0;
      TG_TRY(gpu_sssp(p, *ws, roots_local[r], s, &rounds, &pulls));
      res->rounds += rounds;
      res->pulls += pulls;
      TG_TRY(collect_i32(p->gpu, ws->state, dist + (int64_t)r * V, s));
    }
    for (int k = 0; k < 4; ++k) TG_TRY(stat_fetch(*ws, k, s));
    TG_HIP(hipStreamSynchronize(s));
    res->relax = stat_sum(*ws, 0);
    res->act = stat_sum(*ws, 1);
    res->pull_checks = stat_sum(*ws, 2);
    res->pull_verts = stat_sum(*ws, 3);
    return TG_OK;
  };
  res->rc = run();
  if (res->rc != TG_OK) {
    res->msg = tg_last_error();
    failed->store(true);
    TG_QUIET(hipStreamSynchronize(s));
  }
  if (lane > 0) res->timers = ktimer_export();
}

}  // namespace

int sssp_prepare(tg_partition *p, hipStream_t s) {
  const Tuning &t = p->tune;
  if (t.sssp_xcd) TG_TRY(build_sssp_slices(p, s));
  if (t.sssp_pull > 0 && t.sssp_xcd == 0 && sssp_pull_supported(p->gpu)) TG_TRY(sssp_pull_prepare(p, s));
  TG_TRY(sssp_split_prepare(p, s));
  return TG_OK;
}

int gpu_sssp_roots(tg_partition *p, const int32_t *roots_local, int32_t nr, int32_t *dist, hipStream_t s,
                   int64_t *rounds, int64_t *pulls) {
  const Tuning &t = p->tune;
  // per-partition layouts are built here, once, before lanes share them
  TG_TRY(sssp_prepare(p, s));
  const int nl = (int)std::max<int64_t>(1, std::min<int64_t>(t.sssp_lanes, nr));
  hipStream_t st[MAX_LANES];
  for (int l = 0; l < nl; ++l) TG_TRY(lane_stream(p, l, s, &st[l]));
  for (int l = 1; l < nl; ++l) {
    Workspace *ws = nullptr;
    TG_TRY(lane_workspace(p, l, &ws));  // created here, not in the lane threads
  }
  hipEvent_t ev[MAX_LANES] = {};
  for (int l = 0; l < nl; ++l) TG_HIP(hipEventCreateWithFlags(&ev[l], hipEventDisableTiming));
  int rc = TG_OK;
  // the reference event of this call's kernel timings (with timing on),
  // recorded on s before any lane starts
  const hipEvent_t ref = ktimer_ensure_ref(s);
  // lanes 1.. start after the caller's earlier work on s
  if (hipEventRecord(ev[0], s) != hipSuccess) rc = set_error(TG_EDEVICE, "sssp: hipEventRecord failed");
  for (int l = 1; l < nl && rc == TG_OK; ++l)
    if (hipStreamWaitEvent(st[l], ev[0], 0) != hipSuccess) rc = set_error(TG_EDEVICE, "sssp: stream ordering failed");
  // the reference event of this call's kernel timings, recorded on s before
  // any lane starts
  if (rc == TG_OK) {
    std::atomic<int32_t> next{0};
    std::atomic<bool> failed{false};
    LaneResult res[MAX_LANES];
    std::vector<std::thread> th;
    try {
      for (int l = 1; l < nl; ++l)
        th.emplace_back(sssp_lane, p, l, st[l], roots_local, nr, dist, &next, &failed, &res[l], ref);
    } catch (const std::system_error &) {
      failed.store(true);
      res[0].rc = set_error(TG_EDEVICE, "sssp: could not start a lane thread");
    }
    if (res[0].rc == TG_OK) sssp_lane(p, 0, s, roots_local, nr, dist, &next, &failed, &res[0], ref);
    for (auto &x : th) x.join();
    int64_t rd = 0, pl = 0;
    unsigned long long rx = 0, ac = 0, pc = 0, pv = 0;
    for (int l = 0; l < nl; ++l) {
      if (rc == TG_OK && res[l].rc != TG_OK) rc = set_error(res[l].rc, "%s", res[l].msg.c_str());
      rd += res[l].rounds;
      pl += res[l].pulls;
      rx += res[l].relax;
      ac += res[l].act;
      pc += res[l].pull_checks;
      pv += res[l].pull_verts;
      if (l > 0) ktimer_import(res[l].timers);
    }
    *rounds = rd;
    *pulls = pl;
    stats_add("relaxations", (double)rx);
    stats_add("activations", (double)ac);
    stats_add("heavy_pull_edges_checked", (double)pc);
    stats_add("heavy_pull_vertices", (double)pv);
    stats_add("lanes", nl);
    // the caller's stream waits for the other lanes (already finished)
    for (int l = 1; l < nl && rc == TG_OK; ++l)
      if (hipEventRecord(ev[l], st[l]) != hipSuccess || hipStreamWaitEvent(s, ev[l], 0) != hipSuccess)
        rc = set_error(TG_EDEVICE, "sssp: stream ordering failed");
  }
  for (int l = 0; l < nl; ++l) TG_QUIET(hipEventDestroy(ev[l]));
  return rc;
}

}  // namespace tg

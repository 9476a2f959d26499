// Frontier compaction and planning.
//
// Each superstep's next frontier is a bitmap (one bit per local vertex).  It is
// compacted into a queue sorted by vertex id with a block-wide prefix scan over
// per-thread popcounts; because local ids are in decreasing-degree order, the
// queue is also sorted by degree and each degree bin is one queue segment.  The
// plan kernel then turns segment lengths into virtual-block counts (how many
// 256-thread blocks each bin needs) and, for hub vertices, a prefix over their
// edge chunks.
#include "tg_internal.h"

using namespace tgk;

namespace {

// Compaction kernels run 1024-thread blocks, one bitmap word per thread:
// at 2 MiB of bitmap per RMAT-24 frontier that is 512 blocks, enough waves
// to keep every SIMD busy, and a thread walks at most 32 bits serially.
constexpr int CT = 1024;  // threads per compaction block
constexpr int WPB = CT;   // bitmap words per block

// Sum over the compaction block; every thread gets the result.
template <typename T>
__device__ __forceinline__ T cblock_sum(T x) {
  __shared__ T red[CT / 64];
  x = wave_sum(x);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = x;
  __syncthreads();
  T s = red[0];
#pragma unroll
  for (int k = 1; k < CT / 64; ++k) s += red[k];
  return s;
}

// Exclusive prefix sum over the compaction block; `total` gets the sum.
__device__ __forceinline__ uint32_t cblock_exclusive_scan(uint32_t x, uint32_t &total) {
  __shared__ uint32_t wsum[CT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = x;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  __syncthreads();
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t before = 0;
  total = 0;
#pragma unroll
  for (int k = 0; k < CT / 64; ++k) {
    if (k < w) before += wsum[k];
    total += wsum[k];
  }
  return before + inc - x;
}

// SSSP filter over the set bits of a thread's N words.  A bit whose
// vertex has dist >= settled (the distance it had when it last relaxed its
// edges) is dropped: an attempt to lower it set the bit but found it already
// as low.  Of the rest, bits with dist < thresh are kept (the near set; their
// settled distance is updated here) and the others are counted, with their
// least distance, and stay active.  Eight set bits are handled at a time so
// that their distance loads are in flight together.
template <int N>
__device__ __forceinline__ void sssp_filter_words(uint32_t (&w)[N], int64_t word0, const int32_t *__restrict__ dist,
                                                  int32_t *__restrict__ settled, int32_t thresh, uint32_t (&keep)[N],
                                                  uint32_t (&dropped)[N], uint32_t &rest, int32_t &rest_min) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    keep[k] = 0;
    dropped[k] = 0;
    uint32_t x = w[k];
    const int64_t base = (word0 + k) * 32;
    while (x) {
      int b[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        b[j] = x ? __ffs(x) - 1 : -1;
        x &= x - 1;
      }
      int32_t d[8], st[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t v = base + (b[j] >= 0 ? b[j] : b[0]);
        d[j] = dist[v];
        st[j] = settled[v];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (b[j] < 0) continue;
        const uint32_t bit = 1u << b[j];
        if (d[j] >= st[j]) dropped[k] |= bit;
        else if (d[j] < thresh) {
          keep[k] |= bit;
          settled[base + b[j]] = d[j];  // the distance it relaxes with (at least)
        } else {
          ++rest;
          rest_min = d[j] < rest_min ? d[j] : rest_min;
        }
      }
    }
  }
}

// SSSP compaction, first pass: filter the active bitmap (sssp_filter_words),
// leave the untaken active bits in `bits`, the taken ones in `keep_out`, and
// each block's count in bcount.  With rest_cnt, the vertices left active
// beyond the threshold are counted into it and their least distance goes
// into rest_min (both spread counters; rest_min's slots start all ones).
__global__ __launch_bounds__(CT) void k_sssp_filter(uint32_t *__restrict__ bits, uint32_t *__restrict__ keep_out,
                                                    uint32_t *__restrict__ bcount, const int32_t *__restrict__ dist,
                                                    int32_t *__restrict__ settled, int32_t thresh,
                                                    unsigned long long *rest_cnt, unsigned long long *rest_min) {
  const int64_t q = (int64_t)blockIdx.x * CT + threadIdx.x;  // word index
  const uint32_t v = bits[q];
  uint32_t w[1] = {v}, keep[1], dr[1];
  uint32_t r = 0;
  int32_t rmin = TG_INF;
  sssp_filter_words<1>(w, q, dist, settled, thresh, keep, dr, r, rmin);
  bits[q] = v & ~(keep[0] | dr[0]);
  keep_out[q] = keep[0];
  if (rest_cnt) {
    r = cblock_sum(r);
    for (int o = 32; o > 0; o >>= 1) {
      const int32_t y = __shfl_xor(rmin, o, 64);
      rmin = y < rmin ? y : rmin;
    }
    if ((threadIdx.x & 63) == 0 && rmin < TG_INF)
      atomicMin(rest_min + (size_t)(blockIdx.x & (STAT_SLOTS - 1)) * STAT_STRIDE, (unsigned long long)rmin);
    if (threadIdx.x == 0 && r) stat_add(rest_cnt, (unsigned long long)r);
  }
  const uint32_t c = cblock_sum((uint32_t)__popc(keep[0]));
  if (threadIdx.x == 0) bcount[blockIdx.x] = c;
}

__global__ __launch_bounds__(CT) void k_compact_count(const uint32_t *__restrict__ bits,
                                                      const uint32_t *__restrict__ prev,
                                                      uint32_t *__restrict__ bcount) {
  const int64_t q = (int64_t)blockIdx.x * CT + threadIdx.x;  // word index
  uint32_t v = bits[q];
  if (prev) v &= ~prev[q];
  const uint32_t c = cblock_sum((uint32_t)__popc(v));
  if (threadIdx.x == 0) bcount[blockIdx.x] = c;
}

__global__ __launch_bounds__(CT) void k_compact_write(uint32_t *__restrict__ bits, uint32_t *__restrict__ prev,
                                                      int mode, const uint32_t *__restrict__ bcount,
                                                      int32_t *__restrict__ queue, int32_t *__restrict__ level,
                                                      int32_t level_value, BinBounds bb, int64_t n,
                                                      Plan *__restrict__ plan, uint32_t *__restrict__ fbits,
                                                      const int64_t *__restrict__ off, unsigned long long *degsum) {
  const int64_t q = (int64_t)blockIdx.x * CT + threadIdx.x;  // word index
  const uint32_t v = bits[q];
  // this block's offset: sum of the counts of all earlier blocks
  uint32_t part = 0;
  for (uint32_t i = threadIdx.x; i < blockIdx.x; i += CT) part += bcount[i];
  const uint32_t base = cblock_sum(part);

  uint32_t nw = v;
  if (mode == 0) {
    nw &= ~prev[q];
    prev[q] = v;             // prev := visited
    if (fbits) fbits[q] = nw;  // the new frontier
  } else if (mode == 4) {
    // a bitmap already filtered (k_sssp_filter): take it as it is
  } else {
    if (mode == 2) prev[q] = v;  // prev := the set taken
    bits[q] = 0;
  }
  uint32_t total;
  const uint32_t excl = base + cblock_exclusive_scan((uint32_t)__popc(nw), total);

  // queue positions of the bin boundaries that fall inside this thread's word
#pragma unroll
  for (int b = 0; b < NBIN; ++b) {
    const int64_t t = bb.bstart[b];
    if (t < n && (t >> 5) == q) plan->pos[b] = (int32_t)(excl + __popc(nw & ((1u << (t & 31)) - 1u)));
  }
  uint32_t o = excl;
  unsigned long long deg = 0;
  for (uint32_t w = nw; w; w &= w - 1) {
    const int32_t vtx = (int32_t)(q * 32 + (__ffs(w) - 1));
    queue[o++] = vtx;
    if (level) level[vtx] = level_value;
    if (degsum) deg += (unsigned long long)(off[vtx + 1] - off[vtx]);
  }
  if (degsum) {
    deg = cblock_sum(deg);
    if (threadIdx.x == 0 && deg) stat_add(degsum, deg);
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == CT - 1) plan->count = (int32_t)o;
}

// One block: fix up empty-tail positions, hub chunk prefix, virtual blocks.
__global__ __launch_bounds__(BLOCK) void k_plan(Plan *__restrict__ plan, BinBounds bb, int64_t n,
                                                const int32_t *__restrict__ queue,
                                                const int64_t *__restrict__ off, int64_t hub_chunk,
                                                int64_t *__restrict__ hubpref, int include_zero,
                                                const int32_t *__restrict__ len) {
  __shared__ int32_t pos[NBIN + 1];
  const int32_t count = plan->count;
  if (threadIdx.x <= NBIN) {
    const int b = threadIdx.x;
    pos[b] = (b == NBIN || bb.bstart[b] >= n) ? count : plan->pos[b];
  }
  __syncthreads();
  const int32_t nh = pos[1] - pos[0];
  // exclusive prefix of ceil(deg / hub_chunk) over the hub segment
  uint32_t carry = 0;  // fits: chunks <= E / hub_chunk
  int64_t carry64 = 0;
  for (int32_t i0 = 0; i0 < nh; i0 += BLOCK) {
    const int32_t i = i0 + threadIdx.x;
    uint32_t c = 0;
    if (i < nh) {
      const int32_t v = queue ? queue[pos[0] + i] : pos[0] + i;
      const int64_t d = len ? (int64_t)len[v] : off[v + 1] - off[v];  // edges to chunk
      c = (uint32_t)((d + hub_chunk - 1) / hub_chunk);
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(c, tot);
    if (i < nh) hubpref[i] = carry64 + ex;
    carry64 += tot;
    (void)carry;
  }
  if (threadIdx.x == 0) {
    hubpref[nh] = carry64;
    int64_t vb = 0;
    plan->vb[0] = 0;
    vb += carry64;
    plan->vb[1] = vb;
    for (int b = 1; b < NBIN; ++b) {
      const int64_t cnt = pos[b + 1] - pos[b];
      if (b != BIN_ZERO || include_zero) vb += (cnt + verts_per_vblock(b) - 1) / verts_per_vblock(b);
      plan->vb[b + 1] = vb;
    }
    for (int b = 0; b <= NBIN; ++b) plan->pos[b] = pos[b];
  }
}

}  // namespace

namespace tg {

int launch_grid(int64_t vblocks) {
  const int64_t cap = 16384;
  if (vblocks < 1) return 1;
  return (int)(vblocks < cap ? vblocks : cap);
}

int frontier_compact(const GpuPart &g, Workspace &ws, int mode, uint32_t *bits, uint32_t *prev,
                     int32_t *queue, int32_t *level, int32_t level_value, hipStream_t s) {
  const int blocks = (int)(ws.nwords / WPB);
  hipLaunchKernelGGL(k_compact_count, dim3(blocks), dim3(CT), 0, s, bits, mode == 0 ? prev : nullptr, ws.bcount);
  hipLaunchKernelGGL(k_compact_write, dim3(blocks), dim3(CT), 0, s, bits, prev, mode, ws.bcount, queue, level,
                     level_value, g.out_bins, g.n, ws.plan, nullptr, nullptr, nullptr);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int frontier_compact_bfs(const GpuPart &g, Workspace &ws, uint32_t *visited, uint32_t *prev, uint32_t *fbits,
                         int32_t *queue, int32_t *level, int32_t level_value, unsigned long long *degsum,
                         bool count_degrees, hipStream_t s) {
  const int blocks = (int)(ws.nwords / WPB);
  if (count_degrees) TG_HIP(hipMemsetAsync(degsum, 0, STAT_SPAN * sizeof(unsigned long long), s));
  hipLaunchKernelGGL(k_compact_count, dim3(blocks), dim3(CT), 0, s, visited, prev, ws.bcount);
  hipLaunchKernelGGL(k_compact_write, dim3(blocks), dim3(CT), 0, s, visited, prev, 0, ws.bcount, queue, level,
                     level_value, g.out_bins, g.n, ws.plan, fbits, g.out.off, count_degrees ? degsum : nullptr);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int frontier_compact_sssp(const GpuPart &g, Workspace &ws, uint32_t *bits, int32_t *queue, const int32_t *dist,
                          int32_t *settled, int32_t thresh, bool near, const BinBounds &bb, hipStream_t s) {
  const int blocks = (int)(ws.nwords / WPB);
  unsigned long long *rest_cnt = nullptr, *rest_min = nullptr;
  if (near) {
    // counter 5: active vertices left beyond the threshold; counter 6: their
    // least distance (all-ones slots: none)
    rest_cnt = stat_counter(ws.work, 5);
    rest_min = stat_counter(ws.work, 6);
    TG_TRY(stat_zero(ws, 5, s));
    TG_HIP(hipMemsetAsync(rest_min, 0xFF, STAT_SPAN * sizeof(unsigned long long), s));
  }
  // the taken bits go to bits_b (free during SSSP and connected components)
  hipLaunchKernelGGL(k_sssp_filter, dim3(blocks), dim3(CT), 0, s, bits, ws.bits_b, ws.bcount, dist, settled,
                     near ? thresh : TG_INF, rest_cnt, rest_min);
  hipLaunchKernelGGL(k_compact_write, dim3(blocks), dim3(CT), 0, s, ws.bits_b, nullptr, 4, ws.bcount, queue,
                     nullptr, 0, bb, g.n, ws.plan, nullptr, nullptr, nullptr);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int frontier_plan_bins(const GpuPart &g, Workspace &ws, const int32_t *queue, const BinBounds &bb,
                       const int32_t *len, const Tuning &t, hipStream_t s, bool sync) {
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(BLOCK), 0, s, ws.plan, bb, g.n, queue, g.out.off, t.hub_chunk,
                     ws.hubpref, 0, len);
  TG_HIP(hipGetLastError());
  if (sync) {
    TG_HIP(hipMemcpyAsync(ws.h_plan, ws.plan, sizeof(Plan), hipMemcpyDeviceToHost, s));
    TG_HIP(hipStreamSynchronize(s));
    ktimer_flush();
  }
  return TG_OK;
}

int frontier_plan(const GpuPart &g, Workspace &ws, const int32_t *queue, const Tuning &t,
                  hipStream_t s, bool sync) {
  return frontier_plan_off(g, ws, queue, g.out.off, t, s, sync, false);
}

int frontier_plan_off(const GpuPart &g, Workspace &ws, const int32_t *queue, const int64_t *off,
                      const Tuning &t, hipStream_t s, bool sync, bool include_zero) {
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(BLOCK), 0, s, ws.plan, g.out_bins, g.n, queue,
                     off, t.hub_chunk, ws.hubpref, include_zero ? 1 : 0, nullptr);
  TG_HIP(hipGetLastError());
  if (sync) {
    TG_HIP(hipMemcpyAsync(ws.h_plan, ws.plan, sizeof(Plan), hipMemcpyDeviceToHost, s));
    TG_HIP(hipStreamSynchronize(s));
    ktimer_flush();
  }
  return TG_OK;
}

}  // namespace tg

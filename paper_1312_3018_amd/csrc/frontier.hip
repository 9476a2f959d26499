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

// SSSP filter of one wave's 64 bitmap words (2048 vertices).  A set bit
// whose vertex has dist >= settled (the distance it had when it last relaxed
// its edges) is dropped: an attempt to lower it set the bit but found it
// already as low.  Of the rest, bits with dist < thresh are kept (the near
// set; their settled distance is updated here) and the others are counted,
// with their least distance, and stay active.  The wave walks its words two
// at a time, one vertex per lane, so that the distance and settled loads of
// 64 consecutive vertices are one coalesced access each; pairs of zero words
// are skipped, and up to four pairs are in flight at once.  Lane l ends with
// the keep and drop masks of its own word.  With `lcnt`, `queued` is the
// part of keep whose vertices have at least one light edge (the others have
// nothing to relax in a light pass); without, it equals keep.
__device__ __forceinline__ void sssp_filter_wave(uint32_t w, int64_t word0, const int32_t *__restrict__ dist,
                                                 int32_t *__restrict__ settled, const int32_t *__restrict__ lcnt,
                                                 int32_t thresh, uint32_t &keep, uint32_t &queued,
                                                 uint32_t &dropped, uint32_t &rest, int32_t &rest_min) {
  const int lane = threadIdx.x & 63;
  keep = 0;
  queued = 0;
  dropped = 0;
  // bit 2p: word 2p or 2p + 1 has a set bit
  const unsigned long long nz = __ballot(w != 0u);
  unsigned long long pairs = (nz | (nz >> 1)) & 0x5555555555555555ull;
  while (pairs) {
    int p[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      p[j] = pairs ? __ffsll((long long)pairs) - 1 : -1;
      pairs &= pairs - 1;
    }
    bool mine[4];
    int32_t d[4], st[4], lc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      mine[j] = false;
      if (p[j] < 0) continue;
      const uint32_t wa = (uint32_t)__builtin_amdgcn_readlane((int)w, p[j]);
      const uint32_t wb = (uint32_t)__builtin_amdgcn_readlane((int)w, p[j] + 1);
      mine[j] = ((lane < 32 ? wa >> lane : wb >> (lane - 32)) & 1u) != 0u;
      if (mine[j]) {
        const int64_t v = (word0 + p[j]) * 32 + lane;
        d[j] = dist[v];
        st[j] = settled[v];
        lc[j] = lcnt ? lcnt[v] : 1;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (p[j] < 0) continue;  // wave-uniform
      bool k = false, dr = false;
      if (mine[j]) {
        if (d[j] >= st[j]) {
          dr = true;
        } else if (d[j] < thresh) {
          k = true;
          settled[(word0 + p[j]) * 32 + lane] = d[j];  // the distance it relaxes with (at least)
        } else {
          ++rest;
          rest_min = d[j] < rest_min ? d[j] : rest_min;
        }
      }
      const unsigned long long km = __ballot(k), dm = __ballot(dr), qm = __ballot(k && lc[j] > 0);
      if (lane == p[j]) {
        keep = (uint32_t)km;
        queued = (uint32_t)qm;
        dropped = (uint32_t)dm;
      } else if (lane == p[j] + 1) {
        keep = (uint32_t)(km >> 32);
        queued = (uint32_t)(qm >> 32);
        dropped = (uint32_t)(dm >> 32);
      }
    }
  }
}

// SSSP compaction, first pass: filter the active bitmap (sssp_filter_wave),
// leave the untaken active bits in `bits`, the taken ones in `keep_out`
// (and, with `members`, also OR them into it), and each block's count in
// bcount.  With rest_cnt, the vertices left active beyond the threshold are
// counted into it and their least distance goes into rest_min (both spread
// counters; rest_min's slots start all ones).
__global__ __launch_bounds__(CT) void k_sssp_filter(uint32_t *__restrict__ bits, uint32_t *__restrict__ keep_out,
                                                    uint32_t *__restrict__ bcount, const int32_t *__restrict__ dist,
                                                    int32_t *__restrict__ settled, int32_t thresh,
                                                    unsigned long long *rest_cnt, unsigned long long *rest_min,
                                                    uint32_t *__restrict__ members,
                                                    const int32_t *__restrict__ lcnt) {
  const int64_t q = (int64_t)blockIdx.x * CT + threadIdx.x;  // word index
  const uint32_t v = bits[q];
  if (!__syncthreads_or(v != 0u)) {
    // no active bit in the block's words: nothing taken
    keep_out[q] = 0u;
    if (threadIdx.x == 0) bcount[blockIdx.x] = 0u;
    return;
  }
  uint32_t keep, queued, dr;
  uint32_t r = 0;
  int32_t rmin = TG_INF;
  sssp_filter_wave(v, q - (threadIdx.x & 63), dist, settled, lcnt, thresh, keep, queued, dr, r, rmin);
  bits[q] = v & ~(keep | dr);
  keep_out[q] = queued;
  if (members && keep) members[q] |= keep;
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
  const uint32_t c = cblock_sum((uint32_t)__popc(queued));
  if (threadIdx.x == 0) bcount[blockIdx.x] = c;
}

// Bits of word q that stand for vertices below n.
__device__ __forceinline__ uint32_t valid_bits(int64_t q, int64_t n) {
  const int64_t lo = q * 32;
  return lo + 32 <= n ? 0xFFFFFFFFu : lo >= n ? 0u : (1u << (n - lo)) - 1u;
}

// With a BFS control block (`ctl`), a search that has ended skips the pass.
// `invert` counts the vertices below n in neither bitmap (bits nor prev).
__global__ __launch_bounds__(CT) void k_compact_count(const uint32_t *__restrict__ bits,
                                                      const uint32_t *__restrict__ prev,
                                                      uint32_t *__restrict__ bcount,
                                                      const BfsCtl *__restrict__ ctl, int invert, int64_t n) {
  if (ctl && !ctl->active) return;
  const int64_t q = (int64_t)blockIdx.x * CT + threadIdx.x;  // word index
  uint32_t v = bits[q];
  if (invert) v = ~(v | prev[q]) & valid_bits(q, n);
  else if (prev) v &= ~prev[q];
  const uint32_t c = cblock_sum((uint32_t)__popc(v));
  if (threadIdx.x == 0) bcount[blockIdx.x] = c;
}

__global__ __launch_bounds__(CT) void k_compact_write(uint32_t *__restrict__ bits, uint32_t *__restrict__ prev,
                                                      int mode, const uint32_t *__restrict__ bcount,
                                                      int32_t *__restrict__ queue, int32_t *__restrict__ level,
                                                      int32_t level_value, BinBounds bb, int64_t n,
                                                      Plan *__restrict__ plan, uint32_t *__restrict__ fbits,
                                                      const int64_t *__restrict__ off, unsigned long long *degsum,
                                                      const BfsCtl *__restrict__ ctl, int64_t skip_min,
                                                      int64_t valid_n) {
  bool bu = false;
  if (ctl) {
    // device-resident BFS: the level and whether to sum degrees come from
    // the control block (a bottom-up step sums its joins' degrees and
    // writes their levels itself)
    if (!ctl->active) return;
    level_value = ctl->L + 1;
    bu = ctl->bottom_up != 0;
    if (bu) {
      degsum = nullptr;
      level = nullptr;
    }
  }
  if (mode == 4 && bcount[blockIdx.x] == 0u && blockIdx.x != gridDim.x - 1) {
    // a filtered block with nothing taken writes nothing, unless a degree
    // bin starts in its words (the bin's queue position is set here)
    bool starts = false;
#pragma unroll
    for (int b = 0; b < NBIN; ++b) {
      const int64_t w = bb.bstart[b] >> 5;
      starts |= bb.bstart[b] < n && w >= (int64_t)blockIdx.x * CT && w < ((int64_t)blockIdx.x + 1) * CT;
    }
    if (!starts) return;
  }
  const int64_t q = (int64_t)blockIdx.x * CT + threadIdx.x;  // word index
  const uint32_t v = bits[q];
  // this block's offset: sum of the counts of all earlier blocks; after a
  // bottom-up step also the frontier's total
  uint32_t part = 0, rest = 0;
  for (uint32_t i = threadIdx.x; i < gridDim.x; i += CT) {
    const uint32_t c = (i < blockIdx.x || bu) ? bcount[i] : 0u;
    if (i < blockIdx.x) part += c;
    else rest += c;
  }
  const uint32_t base = cblock_sum(part);
  // A frontier of at least skip_min vertices after a bottom-up step keeps
  // the next step bottom-up (Beamer's rule), which reads the frontier bitmap
  // only: no queue is written for it.
  const bool skip_queue = bu && (int64_t)base + (int64_t)cblock_sum(rest) >= skip_min;

  uint32_t nw = v;
  if (mode == 0) {
    nw &= ~prev[q];
    prev[q] = v;             // prev := visited
    if (fbits) fbits[q] = nw;  // the new frontier
  } else if (mode == 4) {
    // a bitmap already filtered (k_sssp_filter): take it as it is
  } else if (mode == 5) {
    // the vertices below valid_n in neither bitmap; both stay as they are
    nw = ~(v | prev[q]) & valid_bits(q, valid_n);
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
  uint32_t o = excl + (uint32_t)__popc(nw);
  unsigned long long deg = 0;
  if (!skip_queue || level || degsum) {
    // the wave's words two at a time, one vertex per lane: a vertex's queue
    // slot is its word pair's first slot plus the set bits below it, so the
    // queue, level and offset accesses of a pair are coalesced; pairs of
    // zero words are skipped and up to four pairs are in flight at once
    const int lane = threadIdx.x & 63;
    const int64_t word0 = q - lane;
    const unsigned long long below = (1ull << lane) - 1ull;
    const unsigned long long nz = __ballot(nw != 0u);
    unsigned long long pairs = (nz | (nz >> 1)) & 0x5555555555555555ull;
    while (pairs) {
      int32_t vv[4];
      uint32_t pos[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        vv[j] = -1;
        if (!pairs) continue;
        const int pr = __ffsll((long long)pairs) - 1;
        pairs &= pairs - 1;
        const unsigned long long m = (unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)nw, pr) |
                                     ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)nw, pr + 1) << 32);
        if ((m >> lane) & 1ull) {
          vv[j] = (int32_t)((word0 + pr) * 32 + lane);
          pos[j] = (uint32_t)__builtin_amdgcn_readlane((int)excl, pr) + (uint32_t)__popcll(m & below);
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (vv[j] >= 0 && !skip_queue) queue[pos[j]] = vv[j];
      if (level) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (vv[j] >= 0) level[vv[j]] = level_value;
      }
      if (degsum) {
        int64_t a[4], b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int32_t x = vv[j] >= 0 ? vv[j] : 0;
          a[j] = off[x];
          b[j] = off[x + 1];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (vv[j] >= 0) deg += (unsigned long long)(b[j] - a[j]);
      }
    }
  }
  if (degsum) {
    deg = cblock_sum(deg);
    if (threadIdx.x == 0 && deg) stat_add(degsum, deg);
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == CT - 1) {
    plan->count = (int32_t)o;
    if (ctl) plan->queue_skipped = skip_queue ? 1 : 0;
  }
}

// done |= members; members := 0.
__global__ __launch_bounds__(BLOCK) void k_bits_merge_clear(uint32_t *__restrict__ done, uint32_t *__restrict__ members,
                                                            int64_t nwords) {
  const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (q >= nwords) return;
  const uint32_t m = members[q];
  if (m) {
    done[q] |= m;
    members[q] = 0u;
  }
}

// One block: fix up empty-tail positions, hub chunk prefix, virtual blocks.
__device__ __forceinline__ void plan_body(Plan *__restrict__ plan, const BinBounds &bb, int64_t n,
                                          const int32_t *__restrict__ queue, const int64_t *__restrict__ off,
                                          int64_t hub_chunk, int64_t *__restrict__ hubpref, int include_zero,
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

__global__ __launch_bounds__(BLOCK) void k_plan(Plan *__restrict__ plan, BinBounds bb, int64_t n,
                                                const int32_t *__restrict__ queue,
                                                const int64_t *__restrict__ off, int64_t hub_chunk,
                                                int64_t *__restrict__ hubpref, int include_zero,
                                                const int32_t *__restrict__ len) {
  plan_body(plan, bb, n, queue, off, hub_chunk, hubpref, include_zero, len);
}

// The plan of a device-resident BFS superstep, then the superstep's
// decisions in the control block: an empty frontier ends the search;
// otherwise the level advances, the frontier's out-degree sum (the spread
// counter `degsum`, zeroed here for the next step) leaves m_u, and Beamer's
// switch picks the direction: bottom-up while m_f > m_u / alpha, back to
// top-down once n_f < n / beta.  Bottom-up steps are counted in `bu_steps`.
__global__ __launch_bounds__(BLOCK) void k_plan_bfs(Plan *__restrict__ plan, BinBounds bb, int64_t n,
                                                    const int32_t *__restrict__ queue,
                                                    const int64_t *__restrict__ off, int64_t hub_chunk,
                                                    int64_t *__restrict__ hubpref, BfsCtl *__restrict__ ctl,
                                                    unsigned long long *__restrict__ degsum,
                                                    unsigned long long *__restrict__ bu_steps, int64_t alpha,
                                                    int64_t beta, int do_switch) {
  if (!ctl->active) return;  // the search has ended: nothing changes any more
  __shared__ unsigned long long m_f;
  __shared__ int32_t dir;  // -1: ended, 0: top-down, 1: bottom-up
  if (threadIdx.x < STAT_SLOTS) {
    const unsigned long long x = wave_sum(degsum[(size_t)threadIdx.x * STAT_STRIDE]);
    degsum[(size_t)threadIdx.x * STAT_STRIDE] = 0ull;
    if (threadIdx.x == 0) m_f = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int32_t n_f = plan->count;
    if (n_f == 0) {
      ctl->active = 0;
      dir = -1;
    } else {
      ctl->L += 1;
      ctl->steps += 1;
      const int64_t m_u = ctl->m_u - (int64_t)m_f;
      ctl->m_u = m_u;
      int32_t bu = ctl->bottom_up;
      if (do_switch) {
        if (!bu && (int64_t)m_f > m_u / alpha) bu = 1;
        else if (bu && (int64_t)n_f < n / beta) bu = 0;
      }
      // a frontier compacted without a queue can only be expanded bottom-up
      // (the compaction skips the queue exactly when the rule above keeps
      // the step bottom-up)
      if (plan->queue_skipped) bu = 1;
      ctl->bottom_up = bu;
      if (bu) *bu_steps += 1ull;  // one writer: this thread
      dir = bu;
    }
  }
  __syncthreads();
  // a top-down step walks the queue: its bins, hub chunks and virtual blocks
  if (dir == 0) plan_body(plan, bb, n, queue, off, hub_chunk, hubpref, 0, nullptr);
}

// Start of a device-resident BFS from `root`: the control block, the
// frontier degree-sum slots and the root's visited bit.
__global__ void k_bfs_ctl_init(BfsCtl *__restrict__ ctl, int64_t m, unsigned long long *__restrict__ degsum,
                               uint32_t *__restrict__ visited, int32_t root) {
  const int t = threadIdx.x;
  if (t < STAT_SLOTS) degsum[(size_t)t * STAT_STRIDE] = 0ull;
  if (t == 0) {
    ctl->m_u = m;
    ctl->L = -1;
    ctl->bottom_up = 0;
    ctl->active = 1;
    ctl->steps = 0;
    if (root >= 0) visited[root >> 5] |= 1u << (root & 31);
  }
}

// Superstep L of a search whose frontier may also grow from outside the
// partition (the hybrid split): the compaction that follows takes new
// vertices at level L + 1 even if this partition's own frontier at L was
// empty (which ended the search in the control block).
__global__ void k_bfs_ctl_resume(BfsCtl *__restrict__ ctl, int32_t L) {
  if (threadIdx.x == 0) {
    if (!ctl->active) {
      ctl->active = 1;
      ctl->bottom_up = 0;
    }
    ctl->L = L;
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
  hipLaunchKernelGGL(k_compact_count, dim3(blocks), dim3(CT), 0, s, bits, mode == 0 ? prev : nullptr, ws.bcount,
                     nullptr, 0, (int64_t)0);
  hipLaunchKernelGGL(k_compact_write, dim3(blocks), dim3(CT), 0, s, bits, prev, mode, ws.bcount, queue, level,
                     level_value, g.out_bins, g.n, ws.plan, nullptr, nullptr, nullptr, nullptr, (int64_t)0, g.n);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int bfs_dev_start(const GpuPart &g, Workspace &ws, int32_t root, hipStream_t s) {
  hipLaunchKernelGGL(k_bfs_ctl_init, dim3(1), dim3(64), 0, s, ws.ctl, g.m, stat_counter(ws.work, 4), ws.bits_a,
                     root);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int bfs_dev_resume(Workspace &ws, int32_t L, hipStream_t s) {
  hipLaunchKernelGGL(k_bfs_ctl_resume, dim3(1), dim3(64), 0, s, ws.ctl, L);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int frontier_compact_bfs_dev(const GpuPart &g, Workspace &ws, const Tuning &t, hipStream_t s) {
  const int blocks = (int)(ws.nwords / WPB);
  hipLaunchKernelGGL(k_compact_count, dim3(blocks), dim3(CT), 0, s, ws.bits_a, ws.bits_b, ws.bcount, ws.ctl, 0,
                     (int64_t)0);
  hipLaunchKernelGGL(k_compact_write, dim3(blocks), dim3(CT), 0, s, ws.bits_a, ws.bits_b, 0, ws.bcount, ws.queue,
                     ws.state, 0, g.out_bins, g.n, ws.plan, ws.bits_c, g.out.off, stat_counter(ws.work, 4), ws.ctl,
                     t.bfs_do ? g.n / t.bfs_beta : INT64_MAX, g.n);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int frontier_plan_bfs_dev(const GpuPart &g, Workspace &ws, const Tuning &t, hipStream_t s) {
  hipLaunchKernelGGL(k_plan_bfs, dim3(1), dim3(BLOCK), 0, s, ws.plan, g.out_bins, g.n, ws.queue, g.out.off,
                     t.hub_chunk, ws.hubpref, ws.ctl, stat_counter(ws.work, 4), stat_counter(ws.work, 3), t.bfs_alpha,
                     t.bfs_beta, (int)t.bfs_do);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int frontier_compact_bucket_end(const GpuPart &g, Workspace &ws, uint32_t *members, uint32_t *done, bool pull,
                                int32_t *queue, unsigned long long *degsum, hipStream_t s) {
  const int blocks = (int)(ws.nwords / WPB);
  // vertices of out-degree 0 (the last ids) have no edge to pull over
  const int64_t nz = g.out_bins.bstart[BIN_ZERO];
  hipLaunchKernelGGL(k_compact_count, dim3(blocks), dim3(CT), 0, s, members, pull ? done : nullptr, ws.bcount,
                     nullptr, pull ? 1 : 0, nz);
  hipLaunchKernelGGL(k_compact_write, dim3(blocks), dim3(CT), 0, s, members, done, pull ? 5 : 4, ws.bcount, queue,
                     nullptr, 0, g.out_bins, g.n, ws.plan, nullptr, degsum ? g.out.off : nullptr, degsum, nullptr,
                     (int64_t)0, nz);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int bitmap_merge_clear(Workspace &ws, uint32_t *done, uint32_t *members, hipStream_t s) {
  hipLaunchKernelGGL(k_bits_merge_clear, dim3((unsigned)((ws.nwords + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, done,
                     members, ws.nwords);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int frontier_compact_sssp(const GpuPart &g, Workspace &ws, uint32_t *bits, int32_t *queue, const int32_t *dist,
                          int32_t *settled, int32_t thresh, bool near, const BinBounds &bb, hipStream_t s,
                          unsigned long long *degsum, uint32_t *members, const int32_t *lcnt) {
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
                     near ? thresh : TG_INF, rest_cnt, rest_min, members, lcnt);
  hipLaunchKernelGGL(k_compact_write, dim3(blocks), dim3(CT), 0, s, ws.bits_b, nullptr, 4, ws.bcount, queue,
                     nullptr, 0, bb, g.n, ws.plan, nullptr, degsum ? g.out.off : nullptr, degsum, nullptr, (int64_t)0,
                     g.n);
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

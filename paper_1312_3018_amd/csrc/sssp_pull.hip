// SSSP superstep in the pull direction, for frontiers that hold a large
// share of the edges (section 7.3 relaxes every out-edge of every active
// vertex; when most vertices are active that is a sweep over nearly all
// edges, and a pull sweep does it without atomics on the hot path).
//
// Every destination v takes the least candidate fd(u) + w(u, v) over its
// in-edges, where fd(u) is u's distance if u is on this superstep's frontier
// and INT32_MAX otherwise; a candidate below dist(v) lowers it and makes v
// active for the next superstep, exactly as the push relaxation of those
// edges would.  The in-edges are split into the 8 per-XCD classes by the
// 128-byte line of fd(u) and cut into row blocks (the layout of the PageRank
// gather, pr_rows.hip): workgroups of XCD k walk class k, so each XCD's L2
// and LDS hold an eighth of fd.  A destination gets one candidate per class
// and takes it with an atomic minimum only when it beats the distance read.
//
// Candidates travel as uint32: a valid distance is below OVER, OVER marks a
// candidate that does not fit below INT32_MAX (the overflow rule of the push
// relaxation: such a vertex is marked and the call fails if it stays
// unreached) and NONE means no in-neighbour on the frontier.
#include <string.h>

#include <algorithm>
#include <vector>

#include "tg_internal.h"

using namespace tgk;

namespace tg {
namespace {

constexpr int NS = 8;     // classes (XCDs)
constexpr int LINE = 32;  // 4-byte values per 128-byte line
constexpr int WB = 1024;  // threads per workgroup
constexpr int U = 8;      // loads per lane per row block
constexpr int NNZ = 64 * U;
constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr uint32_t OVER = 0x7FFFFFFFu;

struct PullArgs {
  const RowBlk *rb;
  int64_t rb_base[NS];
  int64_t nb[NS];
  const int32_t *soff;  // class k's row offsets at soff + k * (n + 1), relative to ebase[k]
  int64_t ebase[NS];
  const int32_t *scol;
  const int32_t *sw;
  const int32_t *fd;  // frontier distances (TG_INF: not on the frontier)
  int32_t *dist;
  uint32_t *active;
  uint32_t *ovf;
  uint32_t *flags;
  uint32_t *chunk_part;  // per chunk block: its least candidate
  const int32_t *lr_b0, *lr_nch;
  const int64_t *lr_pos;
  int32_t nlr;
  int32_t lds_verts;
  int64_t n;
  unsigned long long *work;  // spread counter of candidates from frontier sources
};

__device__ __forceinline__ uint32_t umin32(uint32_t a, uint32_t b) { return a < b ? a : b; }

__device__ __forceinline__ uint32_t group_min(uint32_t x, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) x = umin32(x, __shfl_xor(x, o, 64));
  return x;
}

// The least candidate m of destination v is final for this class: apply it.
__device__ __forceinline__ void finish(const PullArgs &A, int64_t v, uint32_t m) {
  if (m < OVER) {
    if ((int32_t)m < A.dist[v]) {
      atomicMin(A.dist + v, (int32_t)m);
      atomicOr(A.active + (v >> 5), 1u << (v & 31));
    }
  } else if (m == OVER && A.dist[v] == TG_INF) {
    atomicOr(A.ovf + (v >> 5), 1u << (v & 31));
    A.flags[0] = 1u;
  }
}

__device__ __forceinline__ const int32_t *fd_ptr(const int32_t *hot, const int32_t *fd, int64_t H, int32_t u) {
  // generic pointer: one load instruction for the LDS or the global case
  return u < H ? hot + (((u >> 8) << 5) | (u & 31)) : fd + u;
}

struct Loads {
  int32_t o[U];
  int32_t u[U];
  int32_t w[U];
};

// Row offsets, source ids and weights of one row block, issued without a
// branch (lanes past an end re-read the last element).
__device__ __forceinline__ void issue(Loads &L, const RowBlk &me, const RowBlk &nx, const int32_t *off,
                                     const int32_t *col, const int32_t *wt, int lane) {
  const bool chunk = me.lr >= 0;
  const int32_t nr = chunk ? 1 : nx.r0 - me.r0 + 1;
  const int32_t ne = (int32_t)(nx.e0 - me.e0);
  const int64_t elast = ne > 0 ? me.e0 + ne - 1 : 0;
#pragma unroll
  for (int q = 0; q < U; ++q) {
    const int32_t i = q * 64 + lane;
    L.o[q] = off[me.r0 + min(i, nr - 1)];
    const int64_t e = min(me.e0 + i, elast);
    L.u[q] = stream_load(col + e);
    L.w[q] = stream_load(wt + e);
  }
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// One workgroup of WB threads per CU; each wave walks its own row blocks of
// class k = blockIdx mod 8 (the loads of block j+1 in flight with the
// gathers of block j), with the hottest class-k lines of fd in LDS.
__global__ __launch_bounds__(WB) void k_sssp_pull_rows(const PullArgs A) {
  extern __shared__ int32_t lds[];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  int32_t *hot = lds;
  uint32_t *vals = reinterpret_cast<uint32_t *>(lds + A.lds_verts + (int64_t)w * NNZ * 2);
  int32_t *loff = reinterpret_cast<int32_t *>(vals + NNZ);
  const int k = (int)(blockIdx.x & (NS - 1));
  const int64_t nwg = (int64_t)(gridDim.x >> 3);
  const int64_t j0 = (int64_t)(blockIdx.x >> 3) * (WB / 64) + w;
  const int64_t js = nwg * (WB / 64);
  for (int32_t i = t; i < A.lds_verts; i += WB) {
    const int64_t u = ((int64_t)(i / LINE) * NS + k) * LINE + (i % LINE);
    hot[i] = u < A.n ? A.fd[u] : TG_INF;
  }
  const int64_t H = (int64_t)A.lds_verts * NS;
  __syncthreads();
  const RowBlk *rb = A.rb + A.rb_base[k];
  const int32_t *off = A.soff + (int64_t)k * (A.n + 1);
  const int32_t *col = A.scol + A.ebase[k];
  const int32_t *wt = A.sw + A.ebase[k];
  unsigned long long relaxed = 0;
  const int64_t nbk = A.nb[k];
  if (j0 < nbk) {
    RowBlk cur = rb[j0], cur_nx = rb[j0 + 1];
    const int64_t i1 = min(j0 + js, nbk - 1);
    RowBlk nxt = rb[i1], nxt_nx = rb[i1 + 1];
    Loads L;
    issue(L, cur, cur_nx, off, col, wt, lane);
    for (int64_t j = j0; j < nbk; j += js) {
      const int64_t i2 = min(j + 2 * js, nbk - 1);
      const RowBlk nn = rb[i2], nn_nx = rb[i2 + 1];
      int32_t x[U];
#pragma unroll
      for (int q = 0; q < U; ++q) x[q] = *fd_ptr(hot, A.fd, H, L.u[q]);
      Loads L2;
      issue(L2, nxt, nxt_nx, off, col, wt, lane);
      const int32_t ne = (int32_t)(cur_nx.e0 - cur.e0);
      uint32_t c[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const bool live = q * 64 + lane < ne && x[q] != TG_INF;
        const int64_t s = (int64_t)x[q] + (int64_t)L.w[q];
        c[q] = !live ? NONE : (s >= (int64_t)TG_INF ? OVER : (uint32_t)s);
        relaxed += live ? 1ull : 0ull;
      }
      if (cur.lr >= 0) {
        // one chunk of a long row: its least candidate, finished by k_sssp_pull_long
        uint32_t m = c[0];
#pragma unroll
        for (int q = 1; q < U; ++q) m = umin32(m, c[q]);
        m = group_min(m, 64);
        if (lane == 0) A.chunk_part[A.rb_base[k] + j] = m;
      } else {
        const int32_t R = cur_nx.r0 - cur.r0;
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const int32_t i = q * 64 + lane;
          if (i <= R) loff[i] = (int32_t)((int64_t)L.o[q] - cur.e0);
          if (i < ne) vals[i] = c[q];
        }
        wave_lds_sync();
        // rows of this block, Lw lanes each (Lw about the mean row length)
        const int32_t avg = ne / R;
        const int lg = avg >= 48 ? 6 : avg >= 24 ? 5 : avg >= 12 ? 4 : avg >= 6 ? 3 : avg >= 3 ? 2 : avg >= 2 ? 1 : 0;
        const int Lw = 1 << lg;
        const int32_t grp = lane >> lg, sub = lane & (Lw - 1);
        for (int32_t rbase = 0; rbase < R; rbase += (64 >> lg)) {
          const int32_t r = rbase + grp;
          uint32_t m = NONE;
          if (r < R) {
            const int32_t lo = loff[r], hi = loff[r + 1];
            for (int32_t i = lo + sub; i < hi; i += Lw) m = umin32(m, vals[i]);
          }
          m = group_min(m, Lw);
          if (r < R && sub == 0 && m != NONE) finish(A, cur.r0 + r, m);
        }
        wave_lds_sync();
      }
      cur = nxt;
      cur_nx = nxt_nx;
      nxt = nn;
      nxt_nx = nn_nx;
      L = L2;
    }
  }
  // candidates from frontier sources (the push relaxations this sweep stands for)
  relaxed = wave_sum(relaxed);
  if (lane == 0 && relaxed) stat_add(A.work, relaxed);
}

// Long rows: one wave per row takes the least of its chunks' candidates.
__global__ __launch_bounds__(BLOCK) void k_sssp_pull_long(const PullArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * BLOCK) >> 6;
  for (int64_t lr = w0; lr < A.nlr; lr += nw) {
    const int64_t b0 = A.lr_b0[lr];
    const int32_t nch = A.lr_nch[lr];
    uint32_t m = NONE;
    for (int32_t c = lane; c < nch; c += 64) m = umin32(m, A.chunk_part[b0 + c]);
    m = group_min(m, 64);
    if (lane == 0 && m != NONE) finish(A, A.lr_pos[lr], m);
  }
}

// fd(v) = dist(v) for the vertices taken into this superstep's frontier
// (bit set in `taken`), INT32_MAX for the others.
// The frontier's size goes to the spread counter `nf` (the activations the
// push step would have counted).
__global__ __launch_bounds__(BLOCK) void k_sssp_fd(const uint32_t *__restrict__ taken, const int32_t *__restrict__ dist,
                                                   int64_t n, int32_t *__restrict__ fd, unsigned long long *nf) {
  const int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool on = v < n && ((taken[v >> 5] >> (v & 31)) & 1u);
  if (v < n) fd[v] = on ? dist[v] : TG_INF;
  const unsigned long long c = block_sum((unsigned long long)(on ? 1 : 0));
  if (threadIdx.x == 0 && c) stat_add(nf, c);
}

}  // namespace

// The pull layout of a partition: in-edges with weights split by the source's
// line class, row blocks per class, the frontier distance array.
struct SsspPull {
  ClassCsr cc;
  RowsDev rows;
  int64_t rb_base[NS] = {}, nb[NS] = {};
  int64_t nrows = 0;
  bool built = false;
};

void sssp_pull_free(GpuPart &g) {
  delete g.spull;
  g.spull = nullptr;
}

bool sssp_pull_supported(const GpuPart &g) {
  // in-edge weights: on a symmetric whole graph the in-edges are the out-edges
  return g.in_alias && g.out.w != nullptr && g.m > 0;
}

int sssp_pull_prepare(tg_partition *p, hipStream_t s) {
  GpuPart &g = p->gpu;
  if (g.spull && g.spull->built) return TG_OK;
  sssp_pull_free(g);
  g.spull = new (std::nothrow) SsspPull();
  if (!g.spull) return set_error(TG_ENOMEM, "sssp: out of host memory");
  SsspPull &S = *g.spull;
  const int64_t n = g.n;
  std::vector<int32_t> hsoff, hcnt;
  TG_TRY(build_class_csr(g.in.off, g.in.col, g.out.w, n, g.m, S.cc, hsoff, hcnt, s));
  // rows: destinations with in-edges (a symmetric whole graph ends them at
  // its degree-0 tail)
  S.nrows = g.in_bins.bstart[BIN_ZERO];
  RowBlocksHost all, hk;
  int64_t nlr = 0;
  for (int k = 0; k < NS; ++k) {
    S.rb_base[k] = (int64_t)all.rb.size();
    build_row_blocks(S.nrows, nullptr, hsoff.data() + (size_t)k * (n + 1), NNZ, S.rb_base[k], 0, hk);
    S.nb[k] = (int64_t)hk.rb.size() - 1;
    for (RowBlk &b : hk.rb)
      if (b.lr >= 0) b.lr += (int32_t)nlr;
    all.rb.insert(all.rb.end(), hk.rb.begin(), hk.rb.end());
    all.lr_b0.insert(all.lr_b0.end(), hk.lr_b0.begin(), hk.lr_b0.end());
    all.lr_nch.insert(all.lr_nch.end(), hk.lr_nch.begin(), hk.lr_nch.end());
    all.lr_pos.insert(all.lr_pos.end(), hk.lr_pos.begin(), hk.lr_pos.end());
    nlr += (int64_t)hk.lr_b0.size();
  }
  if ((int64_t)all.rb.size() >= ((int64_t)1 << 31)) return set_error(TG_EUNSUPPORTED, "sssp: too many row blocks");
  TG_TRY(rows_upload(S.rows, all));
  TG_HIP(hipStreamSynchronize(s));
  S.built = true;
  return TG_OK;
}

size_t sssp_pull_lds_bytes(int32_t lds_verts) {
  return (size_t)lds_verts * sizeof(int32_t) + (size_t)(WB / 64) * NNZ * sizeof(uint32_t) * 2;
}

int sssp_pull_launch(tg_partition *p, Workspace &ws, const uint32_t *taken, hipStream_t s) {
  GpuPart &g = p->gpu;
  const Tuning &t = p->tune;
  TG_TRY(sssp_pull_prepare(p, s));
  SsspPull &S = *g.spull;
  // per workspace: lanes of one partition run pull steps at the same time
  if (!ws.fd) TG_TRY(dalloc(ws.arena, &ws.fd, (size_t)std::max<int64_t>(g.n, 1)));
  if (ws.pull_part_cap < S.rows.nb_total) {
    TG_TRY(dalloc(ws.arena, &ws.pull_part, (size_t)S.rows.nb_total));
    ws.pull_part_cap = S.rows.nb_total;
  }
  const int tk = ktimer_start(s);
  hipLaunchKernelGGL(k_sssp_fd, dim3((unsigned)((g.n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, taken, ws.state, g.n,
                     ws.fd, stat_counter(ws.work, 1));
  PullArgs A;
  memset(&A, 0, sizeof(A));
  int64_t nbmax = 0;
  for (int c = 0; c < NS; ++c) {
    A.rb_base[c] = S.rb_base[c];
    A.nb[c] = S.nb[c];
    A.ebase[c] = S.cc.cb.base[c];
    nbmax = std::max<int64_t>(nbmax, S.nb[c]);
  }
  A.rb = S.rows.rb;
  A.soff = S.cc.soff;
  A.scol = S.cc.scol;
  A.sw = S.cc.sw;
  A.fd = ws.fd;
  A.dist = ws.state;
  A.active = ws.bits_a;
  A.ovf = ws.bits_c;
  A.flags = ws.counters;
  A.chunk_part = ws.pull_part;
  A.lr_b0 = S.rows.lr_b0;
  A.lr_nch = S.rows.lr_nch;
  A.lr_pos = S.rows.lr_pos;
  A.nlr = (int32_t)S.rows.nlr;
  A.n = g.n;
  A.work = stat_counter(ws.work, 0);
  // hot table: whole lines, no more than a class holds, and what fits in LDS
  const int64_t lines = std::min<int64_t>(t.pr_lds_verts / LINE, (g.n + (int64_t)LINE * NS - 1) / ((int64_t)LINE * NS));
  int32_t lv = (int32_t)(lines * LINE);
  while (lv > 0 && sssp_pull_lds_bytes(lv) > (size_t)rows_lds_limit()) lv -= LINE;
  A.lds_verts = lv;
  const int64_t per = std::max<int64_t>(1, std::min<int64_t>((nbmax + 15) / 16, std::max<int64_t>(t.pr_grid / NS, 1)));
  hipLaunchKernelGGL(k_sssp_pull_rows, dim3((unsigned)(per * NS)), dim3(WB), sssp_pull_lds_bytes(lv), s, A);
  if (A.nlr > 0)
    hipLaunchKernelGGL(k_sssp_pull_long, dim3((unsigned)long_grid(A.nlr)), dim3(BLOCK), 0, s, A);
  ktimer_stop(tk, s, "sssp_pull");
  TG_HIP(hipGetLastError());
  return TG_OK;
}

}  // namespace tg

// PageRank pull gather over row blocks (section 7.1, Figure 14).
//
// The in-edge CSR is cut once into row blocks: runs of consecutive
// destination rows holding at most `nnz` in-edges and at most `nnz` rows; a
// row longer than `nnz` becomes a run of chunk blocks of `nnz` edges each.  A
// workgroup takes one row block at a time.  Its lanes first stream the block's
// source ids (coalesced) and gather the contributions c(u) into LDS, up to
// eight independent gathers in flight per lane; then groups of 1 to 64 lanes,
// sized to the block's mean row length, sum the rows out of LDS.  The number
// of dependent memory round trips per block is fixed, however the block's
// edges are spread over its rows, which is what bounds the degree-bin walk on
// low-degree rows.
//
// The same kernel serves the per-XCD source classes: there every class has
// its own CSR and row blocks, workgroup i takes class i mod 8, and rows yield
// partial sums that a combine pass adds (see pr_sliced.hip).
//
// Blocks never wait on each other.  A chunk block stores its partial sum; a
// second launch finishes the long rows (one wave per row, a fixed reduction
// tree over its chunks) and a third sums the per-block dangling partials.
// Cross-block combines inside one launch would need device-scope fences,
// which on this multi-XCD part write back and invalidate the XCD's L2.
// Summation order is fixed by the row blocks, so results are deterministic
// for a fixed tuning.
#include <string.h>

#include <algorithm>
#include <vector>

#include "tg_internal.h"

using namespace tgk;

namespace tg {

void build_row_blocks(int64_t nrows, const int64_t *off64, const int32_t *off32, int32_t nnz, int64_t first_block,
                      int64_t pos_base, RowBlocksHost &out) {
  auto off = [&](int64_t r) -> int64_t { return off64 ? off64[r] : (int64_t)off32[r]; };
  out.rb.clear();
  out.lr_b0.clear();
  out.lr_nch.clear();
  out.lr_pos.clear();
  // segments of rows packed independently, then concatenated
  const int64_t nseg = std::max<int64_t>(1, std::min<int64_t>(64, nrows / 65536));
  std::vector<std::vector<RowBlk>> seg_rb((size_t)nseg);
  std::vector<std::vector<int32_t>> seg_lr_b0((size_t)nseg), seg_lr_nch((size_t)nseg), seg_lr_row((size_t)nseg);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t sg = 0; sg < nseg; ++sg) {
    const int64_t lo = nrows * sg / nseg, hi = nrows * (sg + 1) / nseg;
    std::vector<RowBlk> &rb = seg_rb[sg];
    int64_t start = lo;  // first row of the open block
    for (int64_t v = lo; v < hi; ++v) {
      const int64_t len = off(v + 1) - off(v);
      if (len > nnz) {
        if (start < v) rb.push_back(RowBlk{off(start), (int32_t)start, -1});
        const int64_t nch = (len + nnz - 1) / nnz;
        seg_lr_b0[sg].push_back((int32_t)rb.size());  // local for now
        seg_lr_nch[sg].push_back((int32_t)nch);
        seg_lr_row[sg].push_back((int32_t)v);
        const int32_t lr_local = (int32_t)seg_lr_b0[sg].size() - 1;
        for (int64_t c = 0; c < nch; ++c) rb.push_back(RowBlk{off(v) + c * nnz, (int32_t)v, lr_local});
        start = v + 1;
        continue;
      }
      // close the open block if row v does not fit in it
      if (start < v && (off(v + 1) - off(start) > nnz || v - start >= nnz)) {
        rb.push_back(RowBlk{off(start), (int32_t)start, -1});
        start = v;
      }
    }
    if (start < hi) rb.push_back(RowBlk{off(start), (int32_t)start, -1});
  }
  int64_t nb = 0, nlr = 0;
  for (int64_t sg = 0; sg < nseg; ++sg) {
    for (RowBlk &b : seg_rb[sg])
      if (b.lr >= 0) b.lr += (int32_t)nlr;
    for (size_t i = 0; i < seg_lr_b0[sg].size(); ++i) {
      out.lr_b0.push_back((int32_t)(first_block + nb + seg_lr_b0[sg][i]));
      out.lr_nch.push_back(seg_lr_nch[sg][i]);
      out.lr_pos.push_back(pos_base + seg_lr_row[sg][i]);
    }
    out.rb.insert(out.rb.end(), seg_rb[sg].begin(), seg_rb[sg].end());
    nb += (int64_t)seg_rb[sg].size();
    nlr += (int64_t)seg_lr_b0[sg].size();
  }
  out.rb.push_back(RowBlk{off(nrows), (int32_t)nrows, -1});  // sentinel
}

namespace {

constexpr int NS = 8;     // source classes (XCDs)
constexpr int LINE = 32;  // contributions per 128-byte line
constexpr int U = 8;      // edges per lane per pass

template <bool CLASSES>
__device__ __forceinline__ const float *contrib_ptr(const float *hot, const float *c_in, int64_t H, int32_t u) {
  // generic pointer: one load instruction for the LDS or the global case
  if (CLASSES) return u < H ? hot + (((u >> 8) << 5) | (u & 31)) : c_in + u;
  return u < H ? hot + u : c_in + u;
}

template <bool CLASSES, typename OffT>
__global__ __launch_bounds__(BLOCK) void k_pr_rows(const RowsArgs A) {
  extern __shared__ float lds[];
  float *hot = lds;
  float *vals = lds + A.lds_verts;
  int32_t *loff = reinterpret_cast<int32_t *>(vals + A.nnz);
  int32_t *lod = loff + A.nnz + 1;  // out-degrees of the rows (single mode, unless they equal the row lengths)
  const int t = threadIdx.x;
  const int k = CLASSES ? (int)(blockIdx.x & (NS - 1)) : 0;
  const int64_t j0 = CLASSES ? (int64_t)(blockIdx.x >> 3) : (int64_t)blockIdx.x;
  const int64_t js = CLASSES ? (int64_t)(gridDim.x >> 3) : (int64_t)gridDim.x;
  // hottest contributions: sources [0, lds_verts); in class mode the first
  // lds_verts/32 lines of class k (lines k, k+8, ...), so that every source
  // below H has its line in LDS
  for (int32_t i = t; i < A.lds_verts; i += BLOCK) {
    const int64_t u = CLASSES ? ((int64_t)(i / LINE) * NS + k) * LINE + (i % LINE) : (int64_t)i;
    hot[i] = u < A.n ? A.c_in[u] : 0.0f;
  }
  const int64_t H = CLASSES ? (int64_t)A.lds_verts * NS : (int64_t)A.lds_verts;
  __syncthreads();
  const RowBlk *rb = A.rb + A.rb_base[k];
  const OffT *off = static_cast<const OffT *>(A.off) + (int64_t)k * A.off_stride;
  const int32_t *col = A.col + A.ebase[k];
  float *psk = CLASSES ? A.ps + (int64_t)k * A.n : nullptr;
  const double add = CLASSES ? 0.0 : A.base + A.d * (A.drop ? 0.0 : *A.dsum_in) * A.inv_n;
  const bool stage_od = !CLASSES && !A.od_rows;
  double dang = 0.0;

  const int64_t nbk = A.nb[k];
  RowBlk me{}, nx{};
  if (j0 < nbk) {
    me = rb[j0];
    nx = rb[j0 + 1];
  }
  for (int64_t j = j0; j < nbk; j += js) {
    // next block's descriptor, fetched while this one is processed
    RowBlk me2{}, nx2{};
    if (j + js < nbk) {
      me2 = rb[j + js];
      nx2 = rb[j + js + 1];
    }
    const int32_t ne = (int32_t)(nx.e0 - me.e0);
    const bool chunk = me.lr >= 0;
    const int32_t R = chunk ? 1 : nx.r0 - me.r0;
    const int32_t nr = chunk ? 0 : R + 1;  // row offsets to stage
    // One round stages up to BLOCK*U row offsets (and out-degrees) and
    // BLOCK*U edges.  Every load of a round is issued before the first use and
    // without a branch: lanes past an end re-read the last element, and a
    // part with nothing left reads the arrays' first element.
    for (int32_t b0 = 0; b0 < nr || b0 < ne; b0 += BLOCK * U) {
      const bool do_r = b0 < nr, do_e = b0 < ne;
      OffT o[U];
      int64_t p0[U], p1[U];
      int32_t u[U];
      float x[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int32_t i = b0 + q * BLOCK + t;
        o[q] = *(do_r ? off + me.r0 + min(i, nr - 1) : off);
        if (stage_od) {
          const int64_t v = do_r ? me.r0 + min(i, R - 1) : 0;
          p0[q] = stream_load(A.out_off + v);
          p1[q] = stream_load(A.out_off + v + 1) + (A.extra_deg ? A.extra_deg[v] : 0);
        }
      }
#pragma unroll
      for (int q = 0; q < U; ++q) u[q] = stream_load(do_e ? col + me.e0 + min(b0 + q * BLOCK + t, ne - 1) : A.col);
#pragma unroll
      for (int q = 0; q < U; ++q) x[q] = *contrib_ptr<CLASSES>(hot, A.c_in, H, u[q]);
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int32_t i = b0 + q * BLOCK + t;
        if (i < nr) loff[i] = (int32_t)((int64_t)o[q] - me.e0);
        if (stage_od && i < R) lod[i] = (int32_t)(p1[q] - p0[q]);
        if (i < ne) vals[i] = x[q];
      }
    }
    __syncthreads();

    if (chunk) {
      // partial sum of one chunk of a long row, finished by k_pr_long
      double cs = 0.0;
      for (int32_t i = t; i < ne; i += BLOCK) cs += (double)vals[i];
      cs = block_sum(cs);
      if (t == 0) A.chunk_part[A.rb_base[k] + j] = cs;
      __syncthreads();
      me = me2;
      nx = nx2;
      continue;
    }

    // rows of this block, L lanes each (L about the mean row length)
    const int32_t avg = R > 0 ? ne / R : 0;
    const int lg = avg >= 48 ? 6 : avg >= 24 ? 5 : avg >= 12 ? 4 : avg >= 6 ? 3 : avg >= 3 ? 2 : avg >= 2 ? 1 : 0;
    const int L = 1 << lg;
    const int32_t grp = t >> lg, lane = t & (L - 1);
    for (int32_t rbase = 0; rbase < R; rbase += (BLOCK >> lg)) {
      const int32_t r = rbase + grp;
      double s = 0.0;
      int32_t lo = 0, hi = 0;
      if (r < R) {
        lo = loff[r];
        hi = loff[r + 1];
        for (int32_t i = lo + lane; i < hi; i += L) s += (double)vals[i];
      }
      s = group_sum(s, L);
      if (r < R && lane == 0) {
        const int32_t v = me.r0 + r;
        if (CLASSES) {
          __builtin_nontemporal_store((float)s, psk + v);
        } else {
          const double rv = add + A.d * (s + (A.ghost ? A.ghost[v] : 0.0));
          const int32_t od = stage_od ? lod[r] : hi - lo;
          if (A.last) A.rank_out[A.g_of_l[v]] = (float)rv;
          else if (od > 0) __builtin_nontemporal_store((float)(rv / (double)od), A.c_out + v);
          if (od == 0) dang += rv;
        }
      }
    }
    __syncthreads();
    me = me2;
    nx = nx2;
  }
  if (CLASSES) return;
  dang = block_sum(dang);
  if (t == 0) A.partials[blockIdx.x] = dang;
}

// Long rows: one wave per row sums the row's chunk partials (lane-strided,
// then a fixed butterfly) and finishes the row like k_pr_rows does.  Single
// mode leaves one dangling partial per block in long_part.
template <bool CLASSES>
__global__ __launch_bounds__(BLOCK) void k_pr_long(const RowsArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * BLOCK) >> 6;
  const double add = CLASSES ? 0.0 : A.base + A.d * (A.drop ? 0.0 : *A.dsum_in) * A.inv_n;
  double dang = 0.0;
  for (int64_t lr = w0; lr < A.nlr; lr += nw) {
    const int64_t b0 = A.lr_b0[lr];
    const int32_t nch = A.lr_nch[lr];
    double s = 0.0;
    for (int32_t c = lane; c < nch; c += 64) s += A.chunk_part[b0 + c];
    s = wave_sum(s);
    if (lane == 0) {
      const int64_t pos = A.lr_pos[lr];
      if (CLASSES) {
        A.ps[pos] = (float)s;
      } else {
        const int64_t v = pos;
        const double r = add + A.d * (s + (A.ghost ? A.ghost[v] : 0.0));
        const int64_t od = A.out_off[v + 1] - A.out_off[v] + (A.extra_deg ? A.extra_deg[v] : 0);
        if (A.last) A.rank_out[A.g_of_l[v]] = (float)r;
        else if (od > 0) A.c_out[v] = (float)(r / (double)od);
        if (od == 0) dang += r;
      }
    }
  }
  if (CLASSES) return;
  dang = block_sum(dang);
  if (threadIdx.x == 0) A.long_part[blockIdx.x] = dang;
}

// D' = sum of the dangling partials (a then b, each in block order) + the
// isolated vertices' share.  One block.
__global__ __launch_bounds__(BLOCK) void k_pr_dsum(const double *__restrict__ pa, int32_t na,
                                                   const double *__restrict__ pb, int32_t nb, double iso_count,
                                                   double base, double d, double inv_n, int32_t drop,
                                                   const double *__restrict__ dsum_in, double *__restrict__ dsum_out) {
  double acc = 0.0;
  for (int32_t i = threadIdx.x; i < na; i += BLOCK) acc += pa[i];
  for (int32_t i = threadIdx.x; i < nb; i += BLOCK) acc += pb[i];
  acc = block_sum(acc);
  if (threadIdx.x == 0) {
    const double add = base + d * (drop ? 0.0 : *dsum_in) * inv_n;
    *dsum_out = acc + iso_count * add;
  }
}

// Ranks of the isolated tail [n0, n) (no in- or out-edges): r = (1-d)/N + d D/N.
__global__ __launch_bounds__(BLOCK) void k_pr_tail(double base, double d, double inv_n, int32_t drop,
                                                   const double *__restrict__ dsum_in, int64_t n0, int64_t n,
                                                   const int32_t *__restrict__ g_of_l, float *__restrict__ rank_out) {
  const int64_t v = n0 + (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v >= n) return;
  const double add = base + d * (drop ? 0.0 : *dsum_in) * inv_n;
  rank_out[g_of_l[v]] = (float)add;
}

}  // namespace

int rows_upload(RowsDev &D, const RowBlocksHost &h) {
  D.arena.release();
  D.nb_total = (int64_t)h.rb.size();
  D.nlr = (int64_t)h.lr_b0.size();
  const size_t nl = std::max<size_t>(h.lr_b0.size(), 1);
  TG_TRY(dalloc(D.arena, &D.rb, h.rb.size()));
  TG_HIP(hipMemcpy(D.rb, h.rb.data(), h.rb.size() * sizeof(RowBlk), hipMemcpyHostToDevice));
  TG_TRY(dalloc(D.arena, &D.lr_b0, nl));
  TG_TRY(dalloc(D.arena, &D.lr_nch, nl));
  TG_TRY(dalloc(D.arena, &D.lr_pos, nl));
  if (!h.lr_b0.empty()) {
    TG_HIP(hipMemcpy(D.lr_b0, h.lr_b0.data(), h.lr_b0.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    TG_HIP(hipMemcpy(D.lr_nch, h.lr_nch.data(), h.lr_nch.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    TG_HIP(hipMemcpy(D.lr_pos, h.lr_pos.data(), h.lr_pos.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  }
  TG_TRY(dalloc(D.arena, &D.chunk_part, (size_t)D.nb_total));
  TG_TRY(dalloc(D.arena, &D.long_part, (size_t)LONG_GRID));
  return TG_OK;
}

size_t rows_lds_bytes(int32_t lds_verts, int32_t nnz, bool stage_od) {
  return (size_t)lds_verts * sizeof(float) + (size_t)nnz * sizeof(float) + (size_t)(nnz + 1) * sizeof(int32_t) +
         (stage_od ? (size_t)nnz * sizeof(int32_t) : 0);
}

int rows_launch(const RowsArgs &A, bool classes, bool off32, int grid, hipStream_t s) {
  const size_t lds = rows_lds_bytes(A.lds_verts, A.nnz, !classes && !A.od_rows);
  if (lds > 65536) return set_error(TG_EINVAL, "pagerank: row blocks need %zu bytes of LDS (limit 65536)", lds);
  if (classes != (bool)off32) return set_error(TG_EINVAL, "pagerank: row offset width does not match the mode");
  if (classes)
    hipLaunchKernelGGL((k_pr_rows<true, int32_t>), dim3(grid), dim3(BLOCK), lds, s, A);
  else
    hipLaunchKernelGGL((k_pr_rows<false, int64_t>), dim3(grid), dim3(BLOCK), lds, s, A);
  TG_HIP(hipGetLastError());
  if (A.nlr > 0 || !classes) {
    // single mode always runs it: it writes the long rows' dangling partials
    const int lg = long_grid(A.nlr);
    if (classes)
      hipLaunchKernelGGL((k_pr_long<true>), dim3(lg), dim3(BLOCK), 0, s, A);
    else
      hipLaunchKernelGGL((k_pr_long<false>), dim3(lg), dim3(BLOCK), 0, s, A);
    TG_HIP(hipGetLastError());
  }
  return TG_OK;
}

int long_grid(int64_t nlr) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((nlr + (BLOCK / 64) - 1) / (BLOCK / 64), LONG_GRID));
}

int pr_dsum_launch(const double *pa, int32_t na, const double *pb, int32_t nb, double iso_count, double base,
                   double d, double inv_n, int32_t drop, const double *dsum_in, double *dsum_out, hipStream_t s) {
  hipLaunchKernelGGL(k_pr_dsum, dim3(1), dim3(BLOCK), 0, s, pa, na, pb, nb, iso_count, base, d, inv_n, drop, dsum_in,
                     dsum_out);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

// Row blocks of the whole in-edge CSR.  Rows [0, nrows): all local vertices,
// except that a symmetric whole-graph partition leaves out its isolated tail.
struct PrRows {
  RowsDev dev;
  int64_t nrows = 0;
  int32_t nnz = 0;
};

void pr_rows_free(GpuPart &g) {
  delete g.rows;
  g.rows = nullptr;
}

static int build_rows(tg_partition *p) {
  GpuPart &g = p->gpu;
  const int32_t nnz = (int32_t)p->tune.pr_rows;
  if (g.rows && g.rows->nnz == nnz) return TG_OK;
  pr_rows_free(g);
  g.rows = new (std::nothrow) PrRows();
  if (!g.rows) return set_error(TG_ENOMEM, "pagerank: out of host memory");
  PrRows &R = *g.rows;
  R.nrows = g.in_alias ? g.in_bins.bstart[BIN_ZERO] : g.n;
  std::vector<int64_t> hoff((size_t)g.n + 1);
  TG_HIP(hipMemcpy(hoff.data(), g.in.off, hoff.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  RowBlocksHost h;
  build_row_blocks(R.nrows, hoff.data(), nullptr, nnz, 0, 0, h);
  TG_TRY(rows_upload(R.dev, h));
  R.nnz = nnz;
  return TG_OK;
}

int gpu_pagerank_rows_step(tg_partition *p, double damping, int mode, int32_t k, bool last, float *rank_out,
                           hipStream_t s, const double *ghost, const int32_t *extra_deg) {
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  TG_TRY(build_rows(p));
  PrRows &R = *g.rows;
  const double N = (double)g.n_global;
  RowsArgs A;
  memset(&A, 0, sizeof(A));
  A.rb = R.dev.rb;
  A.nb[0] = R.dev.nb_total - 1;  // without the sentinel
  A.off = g.in.off;
  A.col = g.in.col;
  A.lr_b0 = R.dev.lr_b0;
  A.lr_nch = R.dev.lr_nch;
  A.chunk_part = R.dev.chunk_part;
  A.lr_pos = R.dev.lr_pos;
  A.long_part = R.dev.long_part;
  A.nlr = (int32_t)R.dev.nlr;
  A.nnz = R.nnz;
  A.lds_verts = (int32_t)std::min<int64_t>(p->tune.pr_lds_verts, g.n);
  // symmetric whole graph: out-degree = in-degree = row length
  A.od_rows = g.in_alias ? 1 : 0;
  while (A.lds_verts > 0 && rows_lds_bytes(A.lds_verts, A.nnz, !A.od_rows) > 65536) A.lds_verts -= 256;
  if (A.lds_verts < 0) A.lds_verts = 0;
  A.c_in = ws.cbuf[k & 1];
  A.n = g.n;
  A.base = (1.0 - damping) / N;
  A.d = damping;
  A.inv_n = 1.0 / N;
  A.iso_count = (double)(g.n - R.nrows);  // the tail not walked (isolated: dangling)
  A.drop = mode == TG_PR_DANGLING_DROP ? 1 : 0;
  A.last = last ? 1 : 0;
  A.dsum_in = ws.scalars + (k & 1);
  A.dsum_out = ws.scalars + ((k + 1) & 1);
  A.partials = ws.partials;
  A.out_off = g.out.off;
  A.c_out = ws.cbuf[(k + 1) & 1];
  A.g_of_l = g.g_of_l;
  A.rank_out = rank_out;
  A.ghost = ghost;
  A.extra_deg = extra_deg;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(A.nb[0], p->tune.pr_grid));
  const int tk = ktimer_start(s);
  TG_TRY(rows_launch(A, false, false, grid, s));
  TG_TRY(pr_dsum_launch(ws.partials, grid, R.dev.long_part, long_grid(A.nlr), A.iso_count, A.base, A.d, A.inv_n,
                        A.drop, A.dsum_in, A.dsum_out, s));
  ktimer_stop(tk, s, "pr_rows");
  if (last && R.nrows < g.n) {
    const int64_t tail = g.n - R.nrows;
    hipLaunchKernelGGL(k_pr_tail, dim3((unsigned)((tail + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, A.base, A.d,
                       A.inv_n, A.drop, A.dsum_in, R.nrows, g.n, g.g_of_l, rank_out);
    TG_HIP(hipGetLastError());
  }
  return TG_OK;
}

}  // namespace tg

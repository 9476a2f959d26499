// XCD-aware PageRank pull gather.
//
// MI355X has 8 XCDs, each with its own 4 MB L2, and dispatches workgroup i to
// XCD i mod 8.  A plain gather makes every XCD cache the same hot
// contributions c(u).  Here the in-edges are split into 8 classes by the
// 128-byte line of c(u) that the source falls in (class = line mod 8, 32
// sources per line, so no line is shared between classes), each stored as its
// own CSR over the destinations; workgroups with blockIdx mod 8 == k gather
// only class k (the row-block kernel of pr_rows.hip in class mode), so each
// XCD's L2 and LDS hold one eighth of the contribution vector and cover eight
// times as many hot sources.  Each class writes a partial sum per
// destination; a combine pass adds the eight partials and applies the
// PageRank update (section 7.1, Figure 14).  Correctness does not depend on
// the XCD mapping, only the cache behaviour does.
#include <string.h>

#include <algorithm>
#include <vector>

#include "tg_internal.h"

using namespace tgk;

namespace tg {
namespace {

constexpr int NS = 8;     // source classes = XCDs
constexpr int LINE = 32;  // contributions per 128-byte cache line

struct CombineParams {
  double base, d, inv_n, iso_count;
  int32_t drop, last;
  int64_t n_walk;  // vertices [0, n_walk) are updated
  int64_t n;
};

// r(v) = (1-d)/N + d (sum of the 8 partials + D/N); contribution, rank and
// the dangling mass as in the plain gather.  Each block leaves its dangling
// partial in partials[blockIdx]; a one-block launch adds them.
__global__ __launch_bounds__(BLOCK) void k_pr_combine(CombineParams prm, const float *__restrict__ ps,
                                                      const int64_t *__restrict__ out_off,
                                                      const double *__restrict__ dsum_in,
                                                      double *__restrict__ partials, float *__restrict__ c_out,
                                                      const int32_t *__restrict__ g_of_l,
                                                      float *__restrict__ rank_out) {
  const double D = prm.drop ? 0.0 : *dsum_in;
  const double add = prm.base + prm.d * D * prm.inv_n;
  double dang = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < prm.n_walk; v += (int64_t)gridDim.x * BLOCK) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) s += (double)__builtin_nontemporal_load(ps + (int64_t)k * prm.n + v);
    const double r = add + prm.d * s;
    const int64_t od = stream_load(out_off + v + 1) - stream_load(out_off + v);
    if (prm.last) rank_out[g_of_l[v]] = (float)r;
    else if (od > 0) __builtin_nontemporal_store((float)(r / (double)od), c_out + v);
    if (od == 0) dang += r;
  }
  dang = block_sum(dang);
  if (threadIdx.x == 0) partials[blockIdx.x] = dang;
}

}  // namespace

struct PrSlices {
  DevArena arena;
  ClassCsr cc;              // in-edges by source class
  float *ps = nullptr;      // partial sums, class k at ps + k * n
  RowsDev rows;             // per-class row blocks
  int64_t rb_base[NS] = {}, nb[NS] = {};
  int64_t nrows = 0;
  int64_t built_nnz = 0;
  bool built = false;
};

void pr_slices_free(GpuPart &g) {
  delete g.slices;
  g.slices = nullptr;
}

// Build the class CSRs on the device (once per partition and tuning).
static int build_slices(tg_partition *p, hipStream_t s) {
  GpuPart &g = p->gpu;
  const Tuning &t = p->tune;
  if (g.slices && g.slices->built && g.slices->built_nnz == t.pr_rows) return TG_OK;
  pr_slices_free(g);
  g.slices = new (std::nothrow) PrSlices();
  if (!g.slices) return set_error(TG_ENOMEM, "pagerank: out of host memory");
  PrSlices &S = *g.slices;
  const int64_t n = g.n, m = g.in.m;
  std::vector<int32_t> hsoff, hc;
  TG_TRY(build_class_csr(g.in.off, g.in.col, nullptr, n, m, S.cc, hsoff, hc, s));
  {
    // row blocks of every class over rows [0, nrows) (a symmetric whole-graph
    // partition leaves out its isolated tail, whose partials stay 0)
    S.nrows = g.in_alias ? g.in_bins.bstart[BIN_ZERO] : n;
    RowBlocksHost all, hk;
    int64_t nlr = 0;
    for (int k = 0; k < NS; ++k) {
      S.rb_base[k] = (int64_t)all.rb.size();
      build_row_blocks(S.nrows, nullptr, hsoff.data() + (size_t)k * (n + 1), (int32_t)t.pr_rows, S.rb_base[k],
                       (int64_t)k * n, hk);
      S.nb[k] = (int64_t)hk.rb.size() - 1;
      for (RowBlk &b : hk.rb)
        if (b.lr >= 0) b.lr += (int32_t)nlr;
      all.rb.insert(all.rb.end(), hk.rb.begin(), hk.rb.end());
      all.lr_b0.insert(all.lr_b0.end(), hk.lr_b0.begin(), hk.lr_b0.end());
      all.lr_nch.insert(all.lr_nch.end(), hk.lr_nch.begin(), hk.lr_nch.end());
      all.lr_pos.insert(all.lr_pos.end(), hk.lr_pos.begin(), hk.lr_pos.end());
      nlr += (int64_t)hk.lr_b0.size();
    }
    if ((int64_t)all.rb.size() >= ((int64_t)1 << 31))
      return set_error(TG_EUNSUPPORTED, "pagerank: too many row blocks");
    TG_TRY(rows_upload(S.rows, all));
  }
  TG_TRY(dalloc(S.arena, &S.ps, (size_t)NS * std::max<int64_t>(n, 1)));
  // rows that are never walked keep partial 0
  TG_HIP(hipMemset(S.ps, 0, (size_t)NS * std::max<int64_t>(n, 1) * sizeof(float)));
  TG_HIP(hipDeviceSynchronize());  // the clear is on the null stream
  S.built_nnz = t.pr_rows;
  S.built = true;
  return TG_OK;
}

int gpu_pagerank_sliced_step(tg_partition *p, double damping, int mode, int32_t k, bool last, float *rank_out,
                             hipStream_t s) {
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  TG_TRY(build_slices(p, s));
  PrSlices &S = *g.slices;
  const Tuning &t = p->tune;
  const double N = (double)g.n_global;
  RowsArgs A;
  memset(&A, 0, sizeof(A));
  int64_t nbmax = 0;
  for (int c = 0; c < NS; ++c) {
    A.rb_base[c] = S.rb_base[c];
    A.nb[c] = S.nb[c];
    A.ebase[c] = S.cc.cb.base[c];
    nbmax = std::max<int64_t>(nbmax, S.nb[c]);
  }
  A.rb = S.rows.rb;
  A.off = S.cc.soff;
  A.off_stride = g.n + 1;
  A.col = S.cc.scol;
  A.lr_b0 = S.rows.lr_b0;
  A.lr_nch = S.rows.lr_nch;
  A.chunk_part = S.rows.chunk_part;
  A.lr_pos = S.rows.lr_pos;
  A.long_part = S.rows.long_part;
  A.nlr = (int32_t)S.rows.nlr;
  A.nnz = (int32_t)t.pr_rows;
  // hot table: whole lines, no more than a class holds, and what fits in LDS
  const int64_t lines = std::min<int64_t>(t.pr_lds_verts / LINE, (g.n + (int64_t)LINE * NS - 1) / ((int64_t)LINE * NS));
  int32_t lds = (int32_t)(lines * LINE);
  while (lds > 0 && rows_lds_bytes(lds, A.nnz, false) > (size_t)rows_lds_limit()) lds -= LINE;
  A.lds_verts = lds;
  A.c_in = ws.cbuf[k & 1];
  A.n = g.n;
  A.ps = S.ps;
  // workgroups per class: enough for every wave to get a block, at most pr_grid / 8
  const int64_t per = std::max<int64_t>(1, std::min<int64_t>((nbmax + 15) / 16, std::max<int64_t>(t.pr_grid / NS, 1)));
  const int tk = ktimer_start(s);
  TG_TRY(rows_launch(A, true, true, (int)(per * NS), s));
  ktimer_stop(tk, s, "pr_slice_gather");
  CombineParams cp;
  cp.base = (1.0 - damping) / N;
  cp.d = damping;
  cp.inv_n = 1.0 / N;
  cp.drop = mode == TG_PR_DANGLING_DROP ? 1 : 0;
  cp.last = last ? 1 : 0;
  cp.n = g.n;
  // isolated vertices (symmetric graphs: the in-degree-0 tail) are walked only
  // when ranks are written; their dangling share is added analytically
  const bool walk_all = !g.in_alias || last;
  cp.n_walk = walk_all ? g.n : g.in_bins.bstart[BIN_ZERO];
  cp.iso_count = walk_all ? 0.0 : (double)g.n_isolated;
  const int cgrid = (int)std::max<int64_t>(1, std::min<int64_t>((cp.n_walk + BLOCK - 1) / BLOCK, 4096));
  const int tk2 = ktimer_start(s);
  hipLaunchKernelGGL(k_pr_combine, dim3(cgrid), dim3(BLOCK), 0, s, cp, S.ps, g.out.off, ws.scalars + (k & 1),
                     ws.partials, ws.cbuf[(k + 1) & 1], g.g_of_l, rank_out);
  TG_HIP(hipGetLastError());
  TG_TRY(pr_dsum_launch(ws.partials, cgrid, nullptr, 0, cp.iso_count, cp.base, cp.d, cp.inv_n, cp.drop,
                        ws.scalars + (k & 1), ws.scalars + ((k + 1) & 1), s));
  ktimer_stop(tk2, s, "pr_combine");
  return TG_OK;
}

}  // namespace tg

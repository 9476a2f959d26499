// XCD-aware PageRank pull gather.
//
// MI355X has 8 XCDs, each with its own 4 MB L2, and dispatches workgroup i to
// XCD i mod 8.  The plain gather makes every XCD cache the same hot
// contributions c(u).  Here the in-edges are split into 8 classes by the
// 128-byte line of c(u) that the source falls in (class = line mod 8, 32
// sources per line, so no line is shared between classes), each stored as its
// own CSR over the destinations; workgroups with blockIdx mod 8 == k gather
// only class k, so each XCD's L2 holds one eighth of the contribution vector
// and covers eight times as many hot sources.  Each
// class writes a partial sum per destination; a combine pass adds the eight
// partials and applies the PageRank update (section 7.1, Figure 14) exactly as
// the plain gather does.  (Correctness does not depend on the XCD mapping,
// only the cache behaviour does.)
#include <string.h>

#include <algorithm>
#include <vector>

#include "tg_internal.h"

using namespace tgk;

namespace tg {
namespace {

constexpr int NS = 8;     // source classes = XCDs
constexpr int LINE = 32;  // contributions per 128-byte cache line

__host__ __device__ __forceinline__ int class_of(int32_t u) { return (u >> 5) & (NS - 1); }

struct SliceArgs {
  int64_t base[NS];     // first edge of class k in scol
  int64_t hp_off[NS];   // first hubpref entry of class k
  int64_t chunk0[NS];   // first hub chunk of class k
};

// Row of destination v in class k: [base[k] + soff[k][v], base[k] + soff[k][v+1]).
__global__ __launch_bounds__(BLOCK) void k_slice_count(const int64_t *__restrict__ ioff, const int32_t *__restrict__ icol,
                                                       int64_t n, int32_t *__restrict__ cnt) {
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK) {
    int32_t c[NS] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t e = ioff[v]; e < ioff[v + 1]; ++e) {
      const int k = class_of(icol[e]);
#pragma unroll
      for (int j = 0; j < NS; ++j) c[j] += (j == k) ? 1 : 0;
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) cnt[k * n + v] = c[k];
  }
}

__global__ __launch_bounds__(BLOCK) void k_slice_fill(const int64_t *__restrict__ ioff, const int32_t *__restrict__ icol,
                                                      int64_t n, const int32_t *__restrict__ soff, SliceArgs sa,
                                                      int32_t *__restrict__ scol) {
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLOCK) {
    int64_t pos[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) pos[k] = sa.base[k] + soff[k * (n + 1) + v];
    for (int64_t e = ioff[v]; e < ioff[v + 1]; ++e) {  // sources stay ascending within each class
      const int32_t u = icol[e];
      const int k = class_of(u);
      int64_t p = 0;
#pragma unroll
      for (int j = 0; j < NS; ++j)
        if (j == k) p = pos[j]++;
      scol[p] = u;
    }
  }
}

struct SAssign {
  int32_t v, qi;
  int64_t e_begin, e_end, chunk;
  int lane, stride, bin;
  bool ok;
};

// As assign_work, over one class's 32-bit row offsets.
__device__ __forceinline__ SAssign assign_slice(int64_t vb, const Plan &P, const int32_t *order,
                                                const int64_t *hubpref, const int32_t *soff, int64_t base,
                                                int64_t hub_chunk) {
  SAssign a;
  a.ok = false;
  a.chunk = -1;
  const int t = threadIdx.x;
  const int b = segment_of(vb, P);
  a.bin = b;
  const int64_t local = vb - P.vb[b];
  if (b == BIN_HUB) {
    int lo = 0, hi = P.pos[1] - P.pos[0];
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (hubpref[mid] <= local) lo = mid; else hi = mid;
    }
    a.qi = P.pos[0] + lo;
    a.v = order ? order[a.qi] : a.qi;
    const int64_t k = local - hubpref[lo];
    const int64_t rb = base + soff[a.v], re = base + soff[a.v + 1];
    a.e_begin = rb + k * hub_chunk;
    a.e_end = a.e_begin + hub_chunk < re ? a.e_begin + hub_chunk : re;
    a.lane = t;
    a.stride = BLOCK;
    a.chunk = local;
    a.ok = true;
    return a;
  }
  const int vpb = verts_per_vblock(b), lpv = lanes_per_vertex(b);
  a.qi = P.pos[b] + (int32_t)(local * vpb) + t / lpv;
  a.lane = t % lpv;
  a.stride = lpv;
  if (a.qi < P.pos[b + 1]) {
    a.v = order ? stream_load(order + a.qi) : a.qi;
    a.e_begin = base + stream_load(soff + a.v);
    a.e_end = base + stream_load(soff + a.v + 1);
    a.ok = true;
  }
  return a;
}

template <bool ORDER>
__global__ __launch_bounds__(BLOCK) void k_pr_slice(const Plan *__restrict__ plans, const int32_t *__restrict__ order,
                                                    const int64_t *__restrict__ hubpref, SliceArgs sa,
                                                    const int32_t *__restrict__ soff, const int32_t *__restrict__ scol,
                                                    int64_t n, const float *__restrict__ c_in, float *__restrict__ ps,
                                                    float *hub_partials, uint32_t *hub_counters, int32_t nh_max,
                                                    int64_t hub_chunk, int32_t lds_verts) {
  __shared__ int s_last;
  extern __shared__ float lds_c[];
  const int k = blockIdx.x & (NS - 1);
  const int64_t jb = blockIdx.x >> 3, nb = gridDim.x >> 3;
  // the hottest sources of class k: the first lds_verts/32 of its lines
  // (lines k, k+8, k+16, ...), kept line by line
  for (int32_t i = threadIdx.x; i < lds_verts; i += BLOCK) {
    const int64_t u = ((int64_t)(i / LINE) * NS + k) * LINE + (i % LINE);
    lds_c[i] = u < n ? c_in[u] : 0.0f;
  }
  const Plan &P = load_plan(plans + k);
  const int32_t *so = soff + (int64_t)k * (n + 1);
  const int64_t *hp = hubpref + sa.hp_off[k];
  float *psk = ps + (int64_t)k * n;
  const int64_t total = P.vb[NBIN];
  const int32_t H = lds_verts * NS;  // sources below H (every class) have their line in LDS
  // LDS slot of a class-k source u < H: line (u >> 5) is the (u >> 8)-th line of the class
  for (int64_t vb = jb; vb < total; vb += nb) {
    const SAssign a = assign_slice(vb, P, ORDER ? order : nullptr, hp, so, sa.base[k], hub_chunk);
    double s = 0.0;
    if (a.ok) {
      const int64_t st = a.stride;
      int64_t e = a.e_begin + a.lane;
      double s1 = 0.0;
      for (; e + st < a.e_end; e += 2 * st) {
        const int32_t u0 = stream_load(scol + e), u1 = stream_load(scol + e + st);
        const float *p0 = u0 < H ? lds_c + (((u0 >> 8) << 5) | (u0 & 31)) : c_in + u0;
        const float *p1 = u1 < H ? lds_c + (((u1 >> 8) << 5) | (u1 & 31)) : c_in + u1;
        s += (double)*p0;
        s1 += (double)*p1;
      }
      if (e < a.e_end) {
        const int32_t u0 = stream_load(scol + e);
        const float *p0 = u0 < H ? lds_c + (((u0 >> 8) << 5) | (u0 & 31)) : c_in + u0;
        s += (double)*p0;
      }
      s += s1;
    }
    if (a.bin == BIN_HUB) {
      s = block_sum(s);
      const int32_t hi = a.qi - P.pos[0];
      uint32_t *ctr = hub_counters + (int64_t)k * nh_max + hi;
      if (threadIdx.x == 0) {
        hub_partials[sa.chunk0[k] + a.chunk] = (float)s;
        __threadfence();
        const uint32_t nch = (uint32_t)(hp[hi + 1] - hp[hi]);
        s_last = (atomicAdd(ctr, 1u) == nch - 1) ? 1 : 0;
      }
      __syncthreads();
      if (s_last && threadIdx.x == 0) {
        __threadfence();
        double tot = 0.0;
        for (int64_t c = hp[hi]; c < hp[hi + 1]; ++c)
          tot += (double)__hip_atomic_load(hub_partials + sa.chunk0[k] + c, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
        psk[a.v] = (float)tot;
        *ctr = 0u;
      }
      __syncthreads();
      continue;
    }
    if (a.bin == BIN_BLOCK) s = block_sum(s);
    else s = group_sum(s, a.stride);
    if (a.ok && a.lane == 0) __builtin_nontemporal_store((float)s, psk + a.v);
  }
}

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
  int32_t *soff = nullptr, *scol = nullptr;
  float *ps = nullptr, *hub_partials = nullptr;
  uint32_t *hub_counters = nullptr;
  int64_t *hubpref = nullptr;
  Plan *d_plans = nullptr;
  Plan plans[NS];
  SliceArgs sa{};
  int32_t nh_max = 0;
  RowsDev rows;             // per-class row blocks (when tuned for row blocks)
  int64_t rb_base[NS] = {}, nb[NS] = {};
  int64_t nrows = 0;
  Tuning built_for{};
  bool built = false;
};

void pr_slices_free(GpuPart &g) {
  delete g.slices;
  g.slices = nullptr;
}

static int build_class_plans(tg_partition *p, PrSlices &S, const std::vector<int32_t> &hc);

// Build the class CSRs on the device (once per partition and tuning).
static int build_slices(tg_partition *p, hipStream_t s) {
  GpuPart &g = p->gpu;
  const Tuning &t = p->tune;
  if (g.slices && g.slices->built && memcmp(g.slices->built_for.min_deg, t.min_deg, sizeof(t.min_deg)) == 0 &&
      g.slices->built_for.hub_chunk == t.hub_chunk && g.slices->built_for.pr_rows == t.pr_rows)
    return TG_OK;
  pr_slices_free(g);
  g.slices = new (std::nothrow) PrSlices();
  if (!g.slices) return set_error(TG_ENOMEM, "pagerank: out of host memory");
  PrSlices &S = *g.slices;
  const int64_t n = g.n, m = g.in.m;
  if (m >= ((int64_t)1 << 31) * NS / 2)
    return set_error(TG_EUNSUPPORTED, "pagerank: too many edges for the sliced gather");
  int32_t *cnt = nullptr;
  TG_TRY(dalloc(S.arena, &cnt, (size_t)NS * n));
  const unsigned grid = (unsigned)std::min<int64_t>((n + BLOCK - 1) / BLOCK, 4096);
  hipLaunchKernelGGL(k_slice_count, dim3(std::max(grid, 1u)), dim3(BLOCK), 0, s, g.in.off, g.in.col, n, cnt);
  TG_HIP(hipGetLastError());
  std::vector<int32_t> hc((size_t)NS * n);
  TG_HIP(hipMemcpyAsync(hc.data(), cnt, hc.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> hsoff((size_t)NS * (n + 1));
  int64_t tot[NS];
#pragma omp parallel for schedule(static, 1)
  for (int k = 0; k < NS; ++k) {
    int64_t acc = 0;
    for (int64_t v = 0; v < n; ++v) {
      hsoff[(size_t)k * (n + 1) + v] = (int32_t)acc;
      acc += hc[(size_t)k * n + v];
    }
    hsoff[(size_t)k * (n + 1) + n] = (int32_t)acc;
    tot[k] = acc;
  }
  int64_t base = 0;
  for (int k = 0; k < NS; ++k) {
    if (tot[k] >= ((int64_t)1 << 31)) return set_error(TG_EUNSUPPORTED, "pagerank: a source class exceeds 2^31 edges");
    S.sa.base[k] = base;
    base += tot[k];
  }
  TG_TRY(dalloc(S.arena, &S.soff, hsoff.size()));
  TG_HIP(hipMemcpyAsync(S.soff, hsoff.data(), hsoff.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  TG_TRY(dalloc(S.arena, &S.scol, (size_t)std::max<int64_t>(m, 1)));
  hipLaunchKernelGGL(k_slice_fill, dim3(std::max(grid, 1u)), dim3(BLOCK), 0, s, g.in.off, g.in.col, n, S.soff, S.sa,
                     S.scol);
  TG_HIP(hipGetLastError());
  if (t.pr_rows) {
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
  } else {
    TG_TRY(build_class_plans(p, S, hc));
  }
  TG_TRY(dalloc(S.arena, &S.ps, (size_t)NS * std::max<int64_t>(n, 1)));
  // rows that are never walked keep partial 0
  TG_HIP(hipMemset(S.ps, 0, (size_t)NS * std::max<int64_t>(n, 1) * sizeof(float)));
  TG_HIP(hipStreamSynchronize(s));
  S.arena.release_one(cnt);
  S.built_for = t;
  S.built = true;
  return TG_OK;
}

// Per-class plans over the same positions as the plain gather (decreasing
// in-degree) for the degree-bin walk; bins follow the expected class row
// length ceil(indeg / 8), hub chunks the actual class rows.
static int build_class_plans(tg_partition *p, PrSlices &S, const std::vector<int32_t> &hc) {
  GpuPart &g = p->gpu;
  const Tuning &t = p->tune;
  const int64_t n = g.n;
  std::vector<int64_t> d8((size_t)n);
  for (int64_t i = 0; i < n; ++i) d8[i] = (g.h_in_deg[i] + NS - 1) / NS;
  BinBounds cb{};
  {
    int64_t i = 0;
    for (int b = 0; b < NBIN; ++b) {
      while (i < n && bin_of_degree(d8[i], t) < b) ++i;
      cb.bstart[b] = i;
    }
    cb.bstart[NBIN] = n;
  }
  const int64_t nh = cb.bstart[1];
  S.nh_max = (int32_t)std::max<int64_t>(nh, 1);
  std::vector<int32_t> horder;
  if (g.pr_order) {
    horder.resize((size_t)n);
    TG_HIP(hipMemcpy(horder.data(), g.pr_order, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost));
  }
  std::vector<int64_t> hubpref;
  int64_t chunks = 0;
  for (int k = 0; k < NS; ++k) {
    Plan &P = S.plans[k];
    memset(&P, 0, sizeof(P));
    P.count = (int32_t)n;
    for (int b = 0; b <= NBIN; ++b) P.pos[b] = (int32_t)cb.bstart[b];
    S.sa.hp_off[k] = (int64_t)hubpref.size();
    S.sa.chunk0[k] = chunks;
    int64_t acc = 0;
    hubpref.push_back(0);
    for (int64_t i = 0; i < nh; ++i) {
      const int64_t v = g.pr_order ? horder[i] : i;
      const int64_t len = hc[(size_t)k * n + v];
      // an empty class row still gets one block, which writes its zero partial
      acc += std::max<int64_t>((len + t.hub_chunk - 1) / t.hub_chunk, 1);
      hubpref.push_back(acc);
    }
    int64_t vb = acc;
    P.vb[0] = 0;
    P.vb[1] = vb;
    for (int b = 1; b < NBIN; ++b) {
      if (b != BIN_ZERO) vb += (P.pos[b + 1] - P.pos[b] + verts_per_vblock(b) - 1) / verts_per_vblock(b);
      P.vb[b + 1] = vb;
    }
    chunks += acc;
  }
  TG_TRY(dalloc(S.arena, &S.hubpref, hubpref.size()));
  TG_HIP(hipMemcpy(S.hubpref, hubpref.data(), hubpref.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  TG_TRY(dalloc(S.arena, &S.d_plans, NS));
  TG_HIP(hipMemcpy(S.d_plans, S.plans, sizeof(S.plans), hipMemcpyHostToDevice));
  TG_TRY(dalloc(S.arena, &S.hub_partials, (size_t)std::max<int64_t>(chunks, 1)));
  TG_TRY(dalloc(S.arena, &S.hub_counters, (size_t)NS * S.nh_max));
  TG_HIP(hipMemset(S.hub_counters, 0, (size_t)NS * S.nh_max * sizeof(uint32_t)));
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
  const bool ordered = g.pr_order != nullptr;
  // whole lines only, and no more than the class holds
  const int64_t lines = std::min<int64_t>(t.pr_lds_verts / LINE, (g.n + (int64_t)LINE * NS - 1) / ((int64_t)LINE * NS));
  int32_t lds = (int32_t)(lines * LINE);
  const int tk = ktimer_start(s);
  const float *cin = ws.cbuf[k & 1];
  if (t.pr_rows) {
    RowsArgs A;
    memset(&A, 0, sizeof(A));
    int64_t nbmax = 0;
    for (int c = 0; c < NS; ++c) {
      A.rb_base[c] = S.rb_base[c];
      A.nb[c] = S.nb[c];
      A.ebase[c] = S.sa.base[c];
      nbmax = std::max<int64_t>(nbmax, S.nb[c]);
    }
    A.rb = S.rows.rb;
    A.off = S.soff;
    A.off_stride = g.n + 1;
    A.col = S.scol;
    A.lr_b0 = S.rows.lr_b0;
    A.lr_nch = S.rows.lr_nch;
    A.chunk_part = S.rows.chunk_part;
    A.lr_pos = S.rows.lr_pos;
    A.long_part = S.rows.long_part;
    A.nlr = (int32_t)S.rows.nlr;
    A.nnz = (int32_t)t.pr_rows;
    while (lds > 0 && rows_lds_bytes(lds, A.nnz, false) > 65536) lds -= LINE;
    A.lds_verts = lds;
    A.c_in = cin;
    A.n = g.n;
    A.ps = S.ps;
    const int64_t per = std::max<int64_t>(1, std::min<int64_t>(nbmax, std::max<int64_t>(t.pr_grid / NS, 1)));
    TG_TRY(rows_launch(A, true, true, (int)(per * NS), s));
  } else {
    int64_t vbmax = 0;
    for (int c = 0; c < NS; ++c) vbmax = std::max<int64_t>(vbmax, S.plans[c].vb[NBIN]);
    const int64_t per = std::max<int64_t>(1, std::min<int64_t>(vbmax, std::max<int64_t>(t.pr_grid / NS, 1)));
    const int grid = (int)(per * NS);
    if (ordered)
    hipLaunchKernelGGL(k_pr_slice<true>, dim3(grid), dim3(BLOCK), (size_t)lds * sizeof(float), s, S.d_plans,
                       g.pr_order, S.hubpref, S.sa, S.soff, S.scol, g.n, cin, S.ps, S.hub_partials, S.hub_counters,
                       S.nh_max, t.hub_chunk, lds);
    else
      hipLaunchKernelGGL(k_pr_slice<false>, dim3(grid), dim3(BLOCK), (size_t)lds * sizeof(float), s, S.d_plans,
                         nullptr, S.hubpref, S.sa, S.soff, S.scol, g.n, cin, S.ps, S.hub_partials, S.hub_counters,
                         S.nh_max, t.hub_chunk, lds);
    TG_HIP(hipGetLastError());
  }
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
  const bool walk_all = ordered || last;
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

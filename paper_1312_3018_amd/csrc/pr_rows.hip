// PageRank pull gather over row blocks (section 7.1, Figure 14).
//
// The in-edge CSR is cut once into row blocks: runs of consecutive
// destination rows holding at most `nnz` in-edges and fewer than `nnz` rows;
// a row longer than `nnz` becomes a run of chunk blocks of `nnz` edges each.
// A workgroup takes one row block at a time.  Its lanes stream the block's
// row offsets and source ids (coalesced) and gather the contributions c(u)
// into LDS, nnz/256 independent loads per lane in flight; then groups of 1 to
// 64 lanes, sized to the block's mean row length, sum the rows out of LDS.
// The loads of the next block are issued while the current block's gathers
// are in flight, so a block costs one memory round trip whatever the spread
// of its edges over its rows -- the latency chain (offsets, then ids, then
// gathers) is what bounds a degree-bin walk on low-degree rows.
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
      if (start < v && (off(v + 1) - off(start) > nnz || v - start >= nnz - 1)) {
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
constexpr int WB = 1024;  // threads per workgroup of the row-block gather

template <bool CLASSES>
__device__ __forceinline__ const float *contrib_ptr(const float *hot, const float *c_in, int64_t H, int32_t u) {
  // generic pointer: one load instruction for the LDS or the global case
  if (CLASSES) return u < H ? hot + (((u >> 8) << 5) | (u & 31)) : c_in + u;
  return u < H ? hot + u : c_in + u;
}

// Loads of one row block (its row offsets, out-degrees when staged, and
// source ids) by one wave, issued without a branch: lanes past an end re-read
// the last element, and a chunk block re-reads its row's offset.
template <typename OffT, int U>
struct BlockLoads {
  OffT o[U];
  int32_t od[U];
  int32_t u[U];
};

template <typename OffT, int U>
__device__ __forceinline__ void issue_loads(BlockLoads<OffT, U> &L, const RowBlk &me, const RowBlk &nx,
                                            const OffT *off, const int32_t *col, const int32_t *od32,
                                            bool stage_od, int lane) {
  const bool chunk = me.lr >= 0;
  const int32_t R = chunk ? 1 : nx.r0 - me.r0;
  const int32_t nr = chunk ? 1 : R + 1;
  const int32_t ne = (int32_t)(nx.e0 - me.e0);
  const int64_t elast = ne > 0 ? me.e0 + ne - 1 : 0;
#pragma unroll
  for (int q = 0; q < U; ++q) {
    const int32_t i = q * 64 + lane;
    L.o[q] = off[me.r0 + min(i, nr - 1)];
    if (stage_od) L.od[q] = od32[me.r0 + min(i, R - 1)];
    L.u[q] = stream_load(col + min(me.e0 + i, elast));
  }
}

// Keeps the compiler from moving LDS accesses across this point; the LDS
// unit serves one wave's accesses in order, so lanes then see each other's
// writes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// One workgroup of WB threads per CU.  Its waves share one table of hot
// contributions in LDS (in class mode every workgroup of an XCD serves the
// same class, so the table covers 8x as many sources) and each wave walks its
// own row blocks of at most 64*U edges and 64*U - 1 rows, with no workgroup
// barrier.  Per wave the loads of block j+1 are issued right after the
// gathers of block j, so one memory round trip covers both.
template <bool CLASSES, typename OffT, int U>
__global__ __launch_bounds__(WB) void k_pr_rows(const RowsArgs A) {
  constexpr int NNZ = 64 * U;
  // all LDS is dynamic (sized by rows_lds_bytes): hot table, then one
  // region per wave, then (single mode) the waves' dangling partials
  extern __shared__ float lds[];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const bool stage_od = !CLASSES && !A.od_rows;
  float *hot = lds;
  double *s_dang = reinterpret_cast<double *>(lds + A.lds_verts + (int64_t)(WB / 64) * NNZ * (stage_od ? 3 : 2));
  float *vals = lds + A.lds_verts + (int64_t)w * NNZ * (stage_od ? 3 : 2);
  int32_t *loff = reinterpret_cast<int32_t *>(vals + NNZ);
  int32_t *lod = loff + NNZ;  // out-degrees of the rows (single mode, unless they equal the row lengths)
  const int k = CLASSES ? (int)(blockIdx.x & (NS - 1)) : 0;
  const int64_t nwg = CLASSES ? (int64_t)(gridDim.x >> 3) : (int64_t)gridDim.x;
  const int64_t j0 = (CLASSES ? (int64_t)(blockIdx.x >> 3) : (int64_t)blockIdx.x) * (WB / 64) + w;
  const int64_t js = nwg * (WB / 64);
  // hottest contributions: sources [0, lds_verts); in class mode the first
  // lds_verts/32 lines of class k (lines k, k+8, ...), so that every source
  // below H has its line in LDS
  for (int32_t i = t; i < A.lds_verts; i += WB) {
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
  double dang = 0.0;

  const int64_t nbk = A.nb[k];
  if (j0 < nbk) {
    // descriptors of the current and the next block (past the end the last
    // block's is re-read: its loads are issued but never used)
    RowBlk cur = rb[j0], cur_nx = rb[j0 + 1];
    const int64_t i1 = min(j0 + js, nbk - 1);
    RowBlk nxt = rb[i1], nxt_nx = rb[i1 + 1];
    BlockLoads<OffT, U> L;
    issue_loads<OffT, U>(L, cur, cur_nx, off, col, A.od32, stage_od, lane);
    for (int64_t j = j0; j < nbk; j += js) {
      const int64_t i2 = min(j + 2 * js, nbk - 1);
      const RowBlk nn = rb[i2], nn_nx = rb[i2 + 1];
      float x[U];
#pragma unroll
      for (int q = 0; q < U; ++q) x[q] = *contrib_ptr<CLASSES>(hot, A.c_in, H, L.u[q]);
      BlockLoads<OffT, U> L2;
      issue_loads<OffT, U>(L2, nxt, nxt_nx, off, col, A.od32, stage_od, lane);

      const int32_t ne = (int32_t)(cur_nx.e0 - cur.e0);
      const bool chunk = cur.lr >= 0;
      if (chunk) {
        // partial sum of one chunk of a long row, finished by k_pr_long
        double cs = 0.0;
#pragma unroll
        for (int q = 0; q < U; ++q) cs += (q * 64 + lane < ne) ? (double)x[q] : 0.0;
        cs = wave_sum(cs);
        if (lane == 0) A.chunk_part[A.rb_base[k] + j] = cs;
      } else {
        const int32_t R = cur_nx.r0 - cur.r0;
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const int32_t i = q * 64 + lane;
          if (i <= R) loff[i] = (int32_t)((int64_t)L.o[q] - cur.e0);
          if (stage_od && i < R) lod[i] = L.od[q];
          if (i < ne) vals[i] = x[q];
        }
        wave_lds_sync();
        // rows of this block, Lw lanes each (Lw about the mean row length)
        const int32_t avg = ne / R;
        const int lg = avg >= 48 ? 6 : avg >= 24 ? 5 : avg >= 12 ? 4 : avg >= 6 ? 3 : avg >= 3 ? 2 : avg >= 2 ? 1 : 0;
        const int Lw = 1 << lg;
        const int32_t grp = lane >> lg, sub = lane & (Lw - 1);
        for (int32_t rbase = 0; rbase < R; rbase += (64 >> lg)) {
          const int32_t r = rbase + grp;
          double sm = 0.0;
          int32_t lo = 0, hi = 0;
          if (r < R) {
            lo = loff[r];
            hi = loff[r + 1];
            for (int32_t i = lo + sub; i < hi; i += Lw) sm += (double)vals[i];
          }
          sm = group_sum(sm, Lw);
          if (r < R && sub == 0) {
            const int32_t v = cur.r0 + r;
            if (CLASSES) {
              __builtin_nontemporal_store((float)sm, psk + v);
            } else {
              const double rv = add + A.d * (sm + (A.ghost ? A.ghost[v] : 0.0));
              const int32_t od = stage_od ? lod[r] : hi - lo;
              if (A.last) A.rank_out[A.g_of_l[v]] = (float)rv;
              else if (od > 0) __builtin_nontemporal_store((float)(rv / (double)od), A.c_out + v);
              if (od == 0) dang += rv;
            }
          }
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
  if (CLASSES) return;
  // dangling partial of this workgroup, waves added in order
  dang = wave_sum(dang);
  if (lane == 0) s_dang[w] = dang;
  __syncthreads();
  if (t == 0) {
    double acc = 0.0;
    for (int i = 0; i < WB / 64; ++i) acc += s_dang[i];
    A.partials[blockIdx.x] = acc;
  }
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
        const int64_t od = A.od_rows ? A.out_off[v + 1] - A.out_off[v] : A.od32[v];
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

// od32[v] = out-degree of v, boundary out-edges included
__global__ __launch_bounds__(BLOCK) void k_pr_od(const int64_t *__restrict__ out_off,
                                                 const int32_t *__restrict__ extra_deg, int64_t n,
                                                 int32_t *__restrict__ od32) {
  const int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v < n) od32[v] = (int32_t)(out_off[v + 1] - out_off[v]) + (extra_deg ? extra_deg[v] : 0);
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
  TG_HIP(hipDeviceSynchronize());  // the copies above are on the null stream
  return TG_OK;
}

size_t rows_lds_bytes(int32_t lds_verts, int32_t nnz, bool stage_od) {
  // (lds_verts is even, so the trailing doubles stay 8-byte aligned)
  return (size_t)lds_verts * sizeof(float) + (size_t)(WB / 64) * nnz * sizeof(int32_t) * (stage_od ? 3 : 2) +
         (size_t)(WB / 64) * sizeof(double);
}

int rows_lds_limit() {
  static int limit[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
  if (!limit[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) v = 65536;
    limit[dev] = v;
  }
  return limit[dev];
}

int rows_launch(const RowsArgs &A, bool classes, bool off32, int grid, hipStream_t s) {
  const size_t lds = rows_lds_bytes(A.lds_verts, A.nnz, !classes && !A.od_rows);
  if (lds > (size_t)rows_lds_limit())
    return set_error(TG_EINVAL, "pagerank: row blocks need %zu bytes of LDS (limit %d)", lds, rows_lds_limit());
  if (classes != (bool)off32) return set_error(TG_EINVAL, "pagerank: row offset width does not match the mode");
  if (A.nnz != 256 && A.nnz != 512) return set_error(TG_EINVAL, "pagerank: row blocks of %d edges (256 or 512)", A.nnz);
  if (A.lds_verts % 2) return set_error(TG_EINVAL, "pagerank: odd hot-table size");
#define TG_ROWS_LAUNCH(C, T, UU) hipLaunchKernelGGL((k_pr_rows<C, T, UU>), dim3(grid), dim3(WB), lds, s, A)
  if (classes) {
    if (A.nnz == 256) TG_ROWS_LAUNCH(true, int32_t, 4);
    else TG_ROWS_LAUNCH(true, int32_t, 8);
  } else {
    if (A.nnz == 256) TG_ROWS_LAUNCH(false, int64_t, 4);
    else TG_ROWS_LAUNCH(false, int64_t, 8);
  }
#undef TG_ROWS_LAUNCH
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
  int32_t *od32 = nullptr;  // out-degrees (incl. boundary edges) when they differ from the row lengths
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
  if (!g.in_alias) TG_TRY(dalloc(R.dev.arena, &R.od32, (size_t)std::max<int64_t>(g.n, 1)));
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
  A.lds_verts = (int32_t)std::min<int64_t>(p->tune.pr_lds_verts, g.n) & ~1;
  // symmetric whole graph: out-degree = in-degree = row length
  A.od_rows = g.in_alias ? 1 : 0;
  A.od32 = R.od32;
  if (!g.in_alias && k == 0 && g.n > 0) {
    hipLaunchKernelGGL(k_pr_od, dim3((unsigned)((g.n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, g.out.off, extra_deg,
                       g.n, R.od32);
    TG_HIP(hipGetLastError());
  }
  while (A.lds_verts > 0 && rows_lds_bytes(A.lds_verts, A.nnz, !A.od_rows) > (size_t)rows_lds_limit())
    A.lds_verts -= 256;
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
  // workgroups: enough for every wave to get a block, at most pr_grid
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((A.nb[0] + 15) / 16, p->tune.pr_grid));
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

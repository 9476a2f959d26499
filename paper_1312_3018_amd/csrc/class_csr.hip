// Per-XCD edge classes of a CSR.
//
// MI355X dispatches workgroup i to XCD i mod 8, and each XCD has its own L2.
// A kernel whose edges gather (or update) the state of the vertex they point
// at gets an eighth of that state per XCD if the edges are split into 8
// classes by the 128-byte line of the target's 4-byte state (class = line mod
// 8, 32 vertices per line, so no line is shared between classes) and the
// workgroups of XCD k take class k only.  The split is stored as 8 CSRs over
// the same rows, back to back: class k's row v is
// [base[k] + soff[k][v], base[k] + soff[k][v+1]) in scol (and sw), targets
// ascending within each class row.
//
// Both set-up kernels take one wave per row; the wave walks the row 64 edges
// at a time and counts (or places) each class with a ballot, so the order
// within a class row is the row's order.
#include <string.h>

#include <algorithm>
#include <vector>

#include "tg_internal.h"

using namespace tgk;

namespace tg {
namespace {

constexpr int NS = 8;

__global__ __launch_bounds__(BLOCK) void k_class_count(const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                       int64_t n, int32_t *__restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * BLOCK) >> 6;
  for (int64_t v = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6; v < n; v += nw) {
    const int64_t e0 = off[v], e1 = off[v + 1];
    int32_t mine = 0;  // lane j < 8 keeps the count of class j
    for (int64_t e = e0; e < e1; e += 64) {
      const int k = e + lane < e1 ? line_class(col[e + lane]) : -1;
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const int c = __popcll(__ballot(k == j));
        if (lane == j) mine += c;
      }
    }
    if (lane < NS) cnt[(int64_t)lane * n + v] = mine;
  }
}

__global__ __launch_bounds__(BLOCK) void k_class_fill(const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                      const int32_t *__restrict__ w, int64_t n,
                                                      const int32_t *__restrict__ soff, ClassBase cb,
                                                      int32_t *__restrict__ scol, int32_t *__restrict__ sw) {
  const int lane = threadIdx.x & 63;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));  // lanes under this one
  const int64_t nw = ((int64_t)gridDim.x * BLOCK) >> 6;
  for (int64_t v = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6; v < n; v += nw) {
    const int64_t e0 = off[v], e1 = off[v + 1];
    int64_t pos = lane < NS ? cb.base[lane] + soff[(int64_t)lane * (n + 1) + v] : 0;  // lane j: next slot of class j
    for (int64_t e = e0; e < e1; e += 64) {
      const bool live = e + lane < e1;
      const int32_t u = live ? col[e + lane] : 0;
      const int k = live ? line_class(u) : -1;
      int64_t dst = 0;
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const uint64_t mk = __ballot(k == j);
        const int64_t pj = __shfl(pos, j, 64);
        if (k == j) dst = pj + __popcll(mk & below);
        if (lane == j) pos += __popcll(mk);
      }
      if (live) {
        scol[dst] = u;
        if (sw) sw[dst] = w[e + lane];
      }
    }
  }
}

}  // namespace

int build_class_csr(const int64_t *off, const int32_t *col, const int32_t *w, int64_t n, int64_t m, ClassCsr &C,
                    std::vector<int32_t> &hsoff, std::vector<int32_t> &hcnt, hipStream_t s) {
  C.arena.release();
  C.n = n;
  C.m = m;
  if (m >= ((int64_t)1 << 31) * NS / 2) return set_error(TG_EUNSUPPORTED, "edge classes: too many edges");
  int32_t *cnt = nullptr;
  TG_TRY(dalloc(C.arena, &cnt, (size_t)NS * std::max<int64_t>(n, 1)));
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n * 64 + BLOCK - 1) / BLOCK, 8192));
  hipLaunchKernelGGL(k_class_count, dim3(grid), dim3(BLOCK), 0, s, off, col, n, cnt);
  TG_HIP(hipGetLastError());
  hcnt.resize((size_t)NS * n);
  TG_HIP(hipMemcpyAsync(hcnt.data(), cnt, hcnt.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  hsoff.resize((size_t)NS * (n + 1));
  int64_t tot[NS];
#pragma omp parallel for schedule(static, 1)
  for (int k = 0; k < NS; ++k) {
    int64_t acc = 0;
    for (int64_t v = 0; v < n; ++v) {
      hsoff[(size_t)k * (n + 1) + v] = (int32_t)acc;
      acc += hcnt[(size_t)k * n + v];
    }
    hsoff[(size_t)k * (n + 1) + n] = (int32_t)acc;
    tot[k] = acc;
  }
  int64_t base = 0;
  for (int k = 0; k < NS; ++k) {
    if (tot[k] >= ((int64_t)1 << 31)) return set_error(TG_EUNSUPPORTED, "edge classes: a class exceeds 2^31 edges");
    C.cb.base[k] = base;
    base += tot[k];
  }
  TG_TRY(dalloc(C.arena, &C.soff, hsoff.size()));
  TG_HIP(hipMemcpyAsync(C.soff, hsoff.data(), hsoff.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  // padded: a block of a class without edges re-reads the class's first
  // slot, which for the last classes lies past every edge, and gathers at
  // the id it finds there (its value is discarded); the padding holds id 0
  // so that gather stays inside the vertex arrays
  TG_TRY(dalloc(C.arena, &C.scol, (size_t)m + 64));
  TG_HIP(hipMemsetAsync(C.scol + m, 0, 64 * sizeof(int32_t), s));
  if (w) {
    TG_TRY(dalloc(C.arena, &C.sw, (size_t)m + 64));
    TG_HIP(hipMemsetAsync(C.sw + m, 0, 64 * sizeof(int32_t), s));
  }
  hipLaunchKernelGGL(k_class_fill, dim3(grid), dim3(BLOCK), 0, s, off, col, w, n, C.soff, C.cb, C.scol, C.sw);
  TG_HIP(hipGetLastError());
  TG_HIP(hipStreamSynchronize(s));
  C.arena.release_one(cnt);
  return TG_OK;
}

}  // namespace tg

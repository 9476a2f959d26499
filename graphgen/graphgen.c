/*
 * graphgen — seeded synthetic graph inputs shared by the tests, the bench and
 * the oracle checks.  It holds no part of the graph algorithms themselves:
 * only edge-list generation (R-MAT and uniform G(n, m)), the edge list -> CSR
 * conversion (symmetrize, drop self-loops and duplicates, sort neighbours)
 * and per-edge weight draws.
 *
 * Randomness is counter based: every draw is a pure function of
 * (seed, stream, index), computed with the SplitMix64 finaliser of Steele,
 * Lea and Flood ("Fast splittable pseudorandom number generators", OOPSLA
 * 2014).  Output is therefore identical for any thread count.
 *
 * R-MAT follows Chakrabarti, Zhan and Faloutsos (SDM 2004): each edge picks
 * one of four quadrants per bit level with probabilities (a, b, c, d).  The
 * paper's workloads take (a, b, c) = (0.57, 0.19, 0.19), with 16 generated
 * edges per vertex on average (section 5, Table 2).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GG_OK 0
#define GG_ENOMEM -2
#define GG_EINVAL -1

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Draw number `i` of stream `stream` under `seed`. */
static inline uint64_t ctr_rand(uint64_t seed, uint64_t stream, uint64_t i) {
  uint64_t key = mix64(seed ^ mix64(stream + 0x632BE59BD9B4E019ULL));
  return mix64(key + (i + 1) * 0x9E3779B97F4A7C15ULL);
}

enum { ST_RMAT = 1, ST_PERM = 2, ST_UNIF = 3, ST_WEIGHT = 4 };

/* Keyed bijection on [0, 2^s): add, multiply by an odd constant and
 * xor-shift, each invertible modulo 2^s.  Used to relabel R-MAT ids so that
 * vertex id carries no degree information (as Graph500 does). */
static inline uint64_t perm_bits(uint64_t x, int s, uint64_t seed) {
  const uint64_t mask = (s >= 64) ? ~0ULL : ((1ULL << s) - 1);
  const int sh = (s + 1) / 2;
  for (int r = 0; r < 4; ++r) {
    uint64_t k = ctr_rand(seed, ST_PERM, (uint64_t)r);
    x = (x + k) & mask;
    x = (x * (k | 1ULL)) & mask;
    x ^= (x >> sh);
  }
  return x;
}

/* ---------------------------------------------------------------- sorting */

static void insertion_sort(int32_t *a, int64_t n) {
  for (int64_t i = 1; i < n; ++i) {
    int32_t v = a[i];
    int64_t j = i - 1;
    while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
    a[j + 1] = v;
  }
}

/* LSD radix sort of non-negative int32 keys, 4 passes of 8 bits. */
static int radix_sort(int32_t *a, int64_t n) {
  int32_t *tmp = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!tmp) return GG_ENOMEM;
  int32_t *src = a, *dst = tmp;
  for (int pass = 0; pass < 4; ++pass) {
    int64_t cnt[257];
    memset(cnt, 0, sizeof(cnt));
    const int sh = pass * 8;
    for (int64_t i = 0; i < n; ++i) cnt[((uint32_t)src[i] >> sh & 0xFF) + 1]++;
    for (int b = 0; b < 256; ++b) cnt[b + 1] += cnt[b];
    for (int64_t i = 0; i < n; ++i) dst[cnt[(uint32_t)src[i] >> sh & 0xFF]++] = src[i];
    int32_t *t = src; src = dst; dst = t;
  }
  /* four passes: result is back in `a` */
  free(tmp);
  return GG_OK;
}

static int sort_unique(int32_t *a, int64_t n, int64_t *out_n) {
  if (n <= 48) insertion_sort(a, n);
  else if (radix_sort(a, n) != GG_OK) return GG_ENOMEM;
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i)
    if (k == 0 || a[k - 1] != a[i]) a[k++] = a[i];
  *out_n = k;
  return GG_OK;
}

/* ------------------------------------------------------------ CSR handle */

typedef struct {
  int64_t n;
  int64_t nnz;
  int64_t *off;
  int32_t *col;
} gg_csr;

/* Edge list (src, dst) of length m over n vertices -> CSR with neighbours
 * sorted ascending, self-loops and duplicates removed; if `symmetrize`, each
 * edge is also inserted reversed.  Consumes nothing; returns a handle. */
static gg_csr *build_csr(int64_t n, int64_t m, const int32_t *src,
                         const int32_t *dst, int symmetrize, int *err) {
  *err = GG_OK;
  gg_csr *h = (gg_csr *)calloc(1, sizeof(gg_csr));
  uint32_t *deg = (uint32_t *)calloc((size_t)n + 1, sizeof(uint32_t));
  int64_t *off = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!h || !deg || !off) { *err = GG_ENOMEM; goto fail; }

#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    int32_t s = src[i], d = dst[i];
    if (s == d) continue;
    __atomic_fetch_add(&deg[s], 1u, __ATOMIC_RELAXED);
    if (symmetrize) __atomic_fetch_add(&deg[d], 1u, __ATOMIC_RELAXED);
  }
  off[0] = 0;
  for (int64_t v = 0; v < n; ++v) off[v + 1] = off[v] + deg[v];
  int64_t raw = off[n];
  int32_t *col = (int32_t *)malloc((size_t)(raw > 0 ? raw : 1) * sizeof(int32_t));
  if (!col) { *err = GG_ENOMEM; goto fail; }
  /* reuse deg as the per-row cursor */
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) deg[v] = 0;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    int32_t s = src[i], d = dst[i];
    if (s == d) continue;
    uint32_t p = __atomic_fetch_add(&deg[s], 1u, __ATOMIC_RELAXED);
    col[off[s] + p] = d;
    if (symmetrize) {
      uint32_t q = __atomic_fetch_add(&deg[d], 1u, __ATOMIC_RELAXED);
      col[off[d] + q] = s;
    }
  }
  int failed = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : failed)
  for (int64_t v = 0; v < n; ++v) {
    int64_t k = 0;
    if (sort_unique(col + off[v], off[v + 1] - off[v], &k) != GG_OK) failed |= 1;
    deg[v] = (uint32_t)k;
  }
  if (failed) { free(col); *err = GG_ENOMEM; goto fail; }
  int64_t *noff = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!noff) { free(col); *err = GG_ENOMEM; goto fail; }
  noff[0] = 0;
  for (int64_t v = 0; v < n; ++v) noff[v + 1] = noff[v] + deg[v];
  int64_t nnz = noff[n];
  int32_t *ncol = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
  if (!ncol) { free(col); free(noff); *err = GG_ENOMEM; goto fail; }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v)
    memcpy(ncol + noff[v], col + off[v], (size_t)deg[v] * sizeof(int32_t));
  free(col);
  free(off);
  free(deg);
  h->n = n;
  h->nnz = nnz;
  h->off = noff;
  h->col = ncol;
  return h;
fail:
  free(h);
  free(deg);
  free(off);
  return NULL;
}

/* R-MAT edge list at the given scale; returns a CSR handle (or NULL). */
void *gg_rmat_csr(int scale, int64_t edge_factor, double a, double b, double c,
                  uint64_t seed, int symmetrize, int permute, int64_t *nnz_out,
                  int *err_out) {
  *err_out = GG_OK;
  if (scale < 1 || scale > 30 || edge_factor < 1 || a < 0 || b < 0 || c < 0 ||
      a + b + c > 1.0) {
    *err_out = GG_EINVAL;
    return NULL;
  }
  const int64_t n = (int64_t)1 << scale;
  const int64_t m = edge_factor << scale;
  int32_t *src = (int32_t *)malloc((size_t)m * sizeof(int32_t));
  int32_t *dst = (int32_t *)malloc((size_t)m * sizeof(int32_t));
  if (!src || !dst) {
    free(src); free(dst);
    *err_out = GG_ENOMEM;
    return NULL;
  }
  /* thresholds in units of 2^-32 */
  const double two32 = 4294967296.0;
  const uint64_t ta = (uint64_t)(a * two32);
  const uint64_t tab = (uint64_t)((a + b) * two32);
  const uint64_t tabc = (uint64_t)((a + b + c) * two32);
  const int64_t words = (scale + 1) / 2; /* two 32-bit uniforms per draw */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    uint64_t u = 0, v = 0, r = 0;
    for (int k = 0; k < scale; ++k) {
      if ((k & 1) == 0) r = ctr_rand(seed, ST_RMAT, (uint64_t)i * words + k / 2);
      uint64_t x = (k & 1) ? (r >> 32) : (r & 0xFFFFFFFFULL);
      uint64_t bu, bv;
      if (x < ta) { bu = 0; bv = 0; }
      else if (x < tab) { bu = 0; bv = 1; }
      else if (x < tabc) { bu = 1; bv = 0; }
      else { bu = 1; bv = 1; }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    if (permute) {
      u = perm_bits(u, scale, seed);
      v = perm_bits(v, scale, seed);
    }
    src[i] = (int32_t)u;
    dst[i] = (int32_t)v;
  }
  gg_csr *h = build_csr(n, m, src, dst, symmetrize, err_out);
  free(src);
  free(dst);
  if (h) *nnz_out = h->nnz;
  return h;
}

/* Uniform random G(n, m): m endpoint pairs drawn uniformly. */
void *gg_uniform_csr(int64_t n, int64_t m, uint64_t seed, int symmetrize,
                     int64_t *nnz_out, int *err_out) {
  *err_out = GG_OK;
  if (n < 1 || n > 2147483647LL || m < 0) { *err_out = GG_EINVAL; return NULL; }
  int32_t *src = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  int32_t *dst = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  if (!src || !dst) { free(src); free(dst); *err_out = GG_ENOMEM; return NULL; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    src[i] = (int32_t)(ctr_rand(seed, ST_UNIF, 2 * (uint64_t)i) % (uint64_t)n);
    dst[i] = (int32_t)(ctr_rand(seed, ST_UNIF, 2 * (uint64_t)i + 1) % (uint64_t)n);
  }
  gg_csr *h = build_csr(n, m, src, dst, symmetrize, err_out);
  free(src);
  free(dst);
  if (h) *nnz_out = h->nnz;
  return h;
}

/* Arbitrary edge list -> CSR (used for hand-made test graphs). */
void *gg_edges_csr(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                   int symmetrize, int64_t *nnz_out, int *err_out) {
  *err_out = GG_OK;
  for (int64_t i = 0; i < m; ++i)
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) {
      *err_out = GG_EINVAL;
      return NULL;
    }
  gg_csr *h = build_csr(n, m, src, dst, symmetrize, err_out);
  if (h) *nnz_out = h->nnz;
  return h;
}

/* Copy the CSR into caller buffers (off: n+1 int64, col: nnz int32), free it. */
void gg_take(void *handle, int64_t *off, int32_t *col) {
  gg_csr *h = (gg_csr *)handle;
  if (!h) return;
  if (off) memcpy(off, h->off, ((size_t)h->n + 1) * sizeof(int64_t));
  if (col && h->nnz) memcpy(col, h->col, (size_t)h->nnz * sizeof(int32_t));
  free(h->off);
  free(h->col);
  free(h);
}

/* Per-edge integer weights uniform in [lo, hi].  With `symmetric`, the draw is
 * keyed by the unordered pair so that w(u, v) == w(v, u). */
void gg_weights(int64_t n, const int64_t *off, const int32_t *col, uint64_t seed,
                int symmetric, int32_t lo, int32_t hi, int32_t *w) {
  const uint64_t span = (uint64_t)((int64_t)hi - (int64_t)lo + 1);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t u = 0; u < n; ++u) {
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      uint64_t x = (uint64_t)u, y = (uint64_t)(uint32_t)col[e];
      if (symmetric && y < x) { uint64_t t = x; x = y; y = t; }
      uint64_t r = ctr_rand(seed, ST_WEIGHT, (x << 32) | y);
      w[e] = (int32_t)((int64_t)lo + (int64_t)(r % span));
    }
  }
}

/* Raw counter-based draws (exposed so Python can sample roots with the same
 * generator). */
void gg_draws(uint64_t seed, uint64_t stream, int64_t start, int64_t count,
              uint64_t *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i)
    out[i] = ctr_rand(seed, stream, (uint64_t)(start + i));
}

/*
 * oracle.c — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU implementations of what the GPU path
 * computes.  Only the tests, the smoke check and the bench's CPU baseline leg
 * may call this code; the product library never links or loads it, and it
 * shares no source with the GPU path.
 *
 * Every function computes the plain definition of its result:
 *   - BFS levels: fewest edges on a directed path from the root (section 6.3.2,
 *     Figure 11; in Appendix 1 the output is this hop count, called the
 *     level, for each vertex).  FIFO queue, first discoverer is the parent.
 *   - SSSP distances: least total weight over directed paths (section 7.3,
 *     Figure 20).  Dijkstra with a binary heap and 64-bit sums; plain
 *     Bellman-Ford (|V|-1 sweeps over every edge) as a second oracle.
 *   - PageRank: the synchronous power iteration of Page et al. cited in
 *     section 7.1 (Figure 14), in fp64, with the contribution of u divided by
 *     its out-degree and the rank of out-degree-0 vertices spread uniformly
 *     (or dropped, as Figure 14 read literally does).
 *   - Connected components (section 9.4; the algorithm runs on the undirected
 *     graph, section 9.4 / Table 5): two vertices share a component iff an
 *     undirected path joins them; each vertex is labelled with the smallest
 *     vertex id of its component (the fixed point of minimum-label
 *     propagation).  Union-find with path halving over every edge, then the
 *     minimum id per root.
 *   - Betweenness centrality: Brandes' algorithm cited in section 7.2
 *     (Figure 18): a BFS from each source counting shortest paths sigma, then
 *     dependencies delta(v) = sum over successors w of sigma_v/sigma_w *
 *     (1 + delta_w), accumulated for v != source, over ordered pairs, not
 *     halved, not normalised.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -2

#define LEVEL_INF INT32_MAX
#define DIST_INF INT64_MAX

/* ------------------------------------------------------------------ BFS */
int oracle_bfs(int64_t n, const int64_t *off, const int32_t *col, int32_t root,
               int32_t *level, int32_t *parent) {
  if (root < 0 || root >= n) return OR_EINVAL;
  int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!queue) return OR_ENOMEM;
  for (int64_t v = 0; v < n; ++v) {
    level[v] = LEVEL_INF;
    if (parent) parent[v] = -1;
  }
  int64_t head = 0, tail = 0;
  level[root] = 0;
  if (parent) parent[root] = root;
  queue[tail++] = root;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t v = col[e];
      if (level[v] == LEVEL_INF) {
        level[v] = level[u] + 1;
        if (parent) parent[v] = u;
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  return OR_OK;
}

/* ----------------------------------------------------------- SSSP: Dijkstra */
typedef struct { int64_t d; int32_t v; } heap_item;

static void heap_push(heap_item *h, int64_t *sz, heap_item x) {
  int64_t i = (*sz)++;
  h[i] = x;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].d <= h[i].d) break;
    heap_item t = h[p]; h[p] = h[i]; h[i] = t;
    i = p;
  }
}

static heap_item heap_pop(heap_item *h, int64_t *sz) {
  heap_item top = h[0];
  h[0] = h[--(*sz)];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, m = i;
    if (l < *sz && h[l].d < h[m].d) m = l;
    if (r < *sz && h[r].d < h[m].d) m = r;
    if (m == i) break;
    heap_item t = h[m]; h[m] = h[i]; h[i] = t;
    i = m;
  }
  return top;
}

/* dist[v] = least weight of a root->v path, DIST_INF if none (lazy deletion
 * heap: an entry is stale when its key exceeds the settled distance). */
int oracle_sssp_dijkstra(int64_t n, const int64_t *off, const int32_t *col,
                         const int32_t *w, int32_t root, int64_t *dist) {
  if (root < 0 || root >= n) return OR_EINVAL;
  int64_t cap = off[n] + 1;
  heap_item *h = (heap_item *)malloc((size_t)cap * sizeof(heap_item));
  uint8_t *done = (uint8_t *)calloc((size_t)n, 1);
  if (!h || !done) { free(h); free(done); return OR_ENOMEM; }
  for (int64_t v = 0; v < n; ++v) dist[v] = DIST_INF;
  int64_t sz = 0;
  dist[root] = 0;
  heap_item first = {0, root};
  heap_push(h, &sz, first);
  while (sz > 0) {
    heap_item it = heap_pop(h, &sz);
    int32_t u = it.v;
    if (done[u] || it.d != dist[u]) continue;
    done[u] = 1;
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t v = col[e];
      int64_t nd = dist[u] + (int64_t)w[e];
      if (nd < dist[v]) {
        dist[v] = nd;
        heap_item x = {nd, v};
        heap_push(h, &sz, x);
      }
    }
  }
  free(h);
  free(done);
  return OR_OK;
}

/* --------------------------------------------------- SSSP: Bellman-Ford */
int oracle_sssp_bellman_ford(int64_t n, const int64_t *off, const int32_t *col,
                             const int32_t *w, int32_t root, int64_t *dist) {
  if (root < 0 || root >= n) return OR_EINVAL;
  for (int64_t v = 0; v < n; ++v) dist[v] = DIST_INF;
  dist[root] = 0;
  for (int64_t round = 0; round + 1 < n; ++round) {
    int changed = 0;
    for (int64_t u = 0; u < n; ++u) {
      if (dist[u] == DIST_INF) continue;
      for (int64_t e = off[u]; e < off[u + 1]; ++e) {
        int64_t nd = dist[u] + (int64_t)w[e];
        if (nd < dist[col[e]]) { dist[col[e]] = nd; changed = 1; }
      }
    }
    if (!changed) break;
  }
  return OR_OK;
}

/* -------------------------------------------------------------- PageRank */
/* r_0 = 1/N; r_{k+1}[v] = (1-d)/N + d * (sum_{u->v} r_k[u]/outdeg(u) + D_k/N)
 * with D_k = sum of r_k over out-degree-0 vertices when dangling_mode == 0,
 * and D_k = 0 when dangling_mode == 1.  Returns r_K. */
int oracle_pagerank(int64_t n, const int64_t *off, const int32_t *col, double d,
                    int32_t iters, int32_t dangling_mode, double *rank) {
  if (n == 0) return OR_OK;
  if (iters < 0 || (dangling_mode != 0 && dangling_mode != 1)) return OR_EINVAL;
  double *acc = (double *)malloc((size_t)n * sizeof(double));
  if (!acc) return OR_ENOMEM;
  const double N = (double)n;
  for (int64_t v = 0; v < n; ++v) rank[v] = 1.0 / N;
  for (int32_t k = 0; k < iters; ++k) {
    double dangling = 0.0;
    for (int64_t v = 0; v < n; ++v) acc[v] = 0.0;
    for (int64_t u = 0; u < n; ++u) {
      int64_t deg = off[u + 1] - off[u];
      if (deg == 0) { dangling += rank[u]; continue; }
      double share = rank[u] / (double)deg;
      for (int64_t e = off[u]; e < off[u + 1]; ++e) acc[col[e]] += share;
    }
    if (dangling_mode == 1) dangling = 0.0;
    for (int64_t v = 0; v < n; ++v)
      rank[v] = (1.0 - d) / N + d * (acc[v] + dangling / N);
  }
  free(acc);
  return OR_OK;
}

/* ---------------------------------------------------------------- Brandes */
/* bc[v] = sum over the given sources s != v of delta_s(v); sigma_out, when
 * non-NULL, receives sigma from the last source (a test hook). */
int oracle_bc(int64_t n, const int64_t *off, const int32_t *col,
              const int32_t *sources, int32_t nsrc, double *bc,
              double *sigma_out) {
  for (int32_t i = 0; i < nsrc; ++i)
    if (sources[i] < 0 || sources[i] >= n) return OR_EINVAL;
  int32_t *order = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int32_t *dist = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  double *sigma = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double *delta = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  if (!order || !dist || !sigma || !delta) {
    free(order); free(dist); free(sigma); free(delta);
    return OR_ENOMEM;
  }
  for (int64_t v = 0; v < n; ++v) bc[v] = 0.0;
  for (int32_t i = 0; i < nsrc; ++i) {
    int32_t s = sources[i];
    for (int64_t v = 0; v < n; ++v) { dist[v] = -1; sigma[v] = 0.0; delta[v] = 0.0; }
    int64_t head = 0, tail = 0;
    dist[s] = 0;
    sigma[s] = 1.0;
    order[tail++] = s;
    while (head < tail) { /* BFS; `order` ends up in non-decreasing distance */
      int32_t u = order[head++];
      for (int64_t e = off[u]; e < off[u + 1]; ++e) {
        int32_t v = col[e];
        if (dist[v] < 0) { dist[v] = dist[u] + 1; order[tail++] = v; }
        if (dist[v] == dist[u] + 1) sigma[v] += sigma[u];
      }
    }
    for (int64_t k = tail - 1; k >= 0; --k) { /* farthest vertices first */
      int32_t v = order[k];
      double acc = 0.0;
      for (int64_t e = off[v]; e < off[v + 1]; ++e) {
        int32_t w = col[e];
        if (dist[w] == dist[v] + 1) acc += sigma[v] / sigma[w] * (1.0 + delta[w]);
      }
      delta[v] = acc;
      if (v != s) bc[v] += acc;
    }
    if (sigma_out && i == nsrc - 1)
      memcpy(sigma_out, sigma, (size_t)n * sizeof(double));
  }
  free(order); free(dist); free(sigma); free(delta);
  return OR_OK;
}

/* ------------------------------------------------------------------ CC */

static int32_t uf_find(int32_t *parent, int32_t x) {
  while (parent[x] != x) {
    parent[x] = parent[parent[x]]; /* path halving */
    x = parent[x];
  }
  return x;
}

/* labels[v] = smallest vertex id in v's (weakly) connected component; the
 * edge direction is ignored. */
int oracle_cc(int64_t n, const int64_t *off, const int32_t *col, int32_t *labels) {
  if (n < 0 || !off || (n > 0 && (!col || !labels))) return OR_EINVAL;
  int32_t *parent = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int32_t *minid = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  if (!parent || !minid) { free(parent); free(minid); return OR_ENOMEM; }
  for (int64_t v = 0; v < n; ++v) parent[v] = (int32_t)v;
  for (int64_t u = 0; u < n; ++u)
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t a = uf_find(parent, (int32_t)u), b = uf_find(parent, col[e]);
      if (a != b) parent[a < b ? b : a] = a < b ? a : b; /* union: smaller root wins */
    }
  for (int64_t v = 0; v < n; ++v) minid[v] = INT32_MAX;
  for (int64_t v = 0; v < n; ++v) {
    int32_t r = uf_find(parent, (int32_t)v);
    if ((int32_t)v < minid[r]) minid[r] = (int32_t)v;
  }
  for (int64_t v = 0; v < n; ++v) labels[v] = minid[uf_find(parent, (int32_t)v)];
  free(parent); free(minid);
  return OR_OK;
}

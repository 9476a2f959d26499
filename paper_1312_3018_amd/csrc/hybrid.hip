// The hybrid split (sections 3-4 and 6.3): one partition on the GPU, one on
// host threads, run as BSP supersteps (section 4.1).  In each superstep both
// partitions compute, each reduces the messages bound for every remote
// vertex into one value at the source (section 3.4), the two message arrays
// cross PCIe (only messages travel: the slot order is fixed at partition time,
// section 4.3.2), and each receiver folds its inbox into its vertex state.
//
// Partition choice (section 6.3.1): HIGH moves the highest-degree vertices to
// the host until it holds cpu_edge_share of the edges, LOW the lowest-degree
// ones, RAND a seeded random subset.
//
// Message reductions are atomic-free: every channel keeps, per outbox slot
// (one distinct remote vertex), the list of local sources — a reverse CSR —
// and the sender reduces each slot's list with the degree-binned gather.
#include <omp.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "gather.h"
#include "hybrid.h"

using namespace tgk;

namespace tg {

// ------------------------------------------------------------ host partition
struct CpuPart {
  int64_t n = 0, m = 0;
  std::vector<int64_t> off;
  std::vector<int32_t> col, w;    // local out-edges (host-local ids)
  std::vector<int64_t> ioff;
  std::vector<int32_t> icol;      // local in-edges
  std::vector<int32_t> g_of_l;    // host-local -> global id
  std::vector<int32_t> l_of_g;    // global id -> host-local id (-1 on the GPU side)
  std::vector<int32_t> bdeg;      // boundary out-degree per host vertex
  int64_t n_dangling = 0;
};

// Messages from a sender partition to a receiver over the boundary edges
// src (sender-local) -> dst (receiver-local).  One slot per distinct receiver
// vertex, in increasing receiver-local id; per slot, its sender-local sources.
struct Channel {
  int64_t nslots = 0;
  std::vector<int32_t> dst;   // slot -> receiver-local id (the receiver's inbox)
  std::vector<int64_t> roff;  // slot -> [roff[s], roff[s+1])
  std::vector<int32_t> rsrc;  // sender-local sources
  std::vector<int32_t> rw;    // their edge weights (if weighted)
  int64_t edges() const { return roff.empty() ? 0 : roff.back(); }
};

struct HybridState {
  CpuPart cpu;
  Channel g2c, c2g;
  int64_t raw_boundary_edges = 0;  // boundary edges before reduction (both directions)
  DevArena arena;
  // GPU-sent channel: reverse CSR and a static degree-binned plan over slots
  int64_t *d_roff = nullptr;
  int32_t *d_rsrc = nullptr, *d_rw = nullptr, *d_slot_order = nullptr;
  Plan h_splan{};
  Plan *d_splan = nullptr;
  int64_t splan_hub_chunk = 0;  // edges per hub chunk of the static slot plan (fixed at build)
  int64_t *d_shubpref = nullptr;
  double *d_shub_partials_f = nullptr;
  int64_t *d_shub_partials_i = nullptr;
  // messages
  int64_t *d_out_i = nullptr;   // GPU outbox (int64: level or distance)
  double *d_out_f = nullptr;    // GPU outbox (PageRank sums)
  int32_t *d_in_dst = nullptr;  // GPU inbox: GPU-local ids
  int64_t *d_in_i = nullptr;
  double *d_in_f = nullptr;
  int32_t *d_bdeg = nullptr;    // GPU vertices' boundary out-degree
  double *d_ghost = nullptr;    // PageRank: inbox sums per GPU vertex
  int32_t *d_cpu_g_of_l = nullptr;
  int32_t *d_stage = nullptr;   // host-partition results on their way to the output
  int64_t *h_out_i = nullptr, *h_in_i = nullptr;
  double *h_out_f = nullptr, *h_in_f = nullptr;
  int32_t *h_stage = nullptr;
  ~HybridState() {
    if (h_out_i) TG_QUIET(hipHostFree(h_out_i));
    if (h_in_i) TG_QUIET(hipHostFree(h_in_i));
    if (h_out_f) TG_QUIET(hipHostFree(h_out_f));
    if (h_in_f) TG_QUIET(hipHostFree(h_in_f));
    if (h_stage) TG_QUIET(hipHostFree(h_stage));
  }
};

namespace {

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t) { return std::chrono::duration<double, std::milli>(clk::now() - t).count(); }

uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Channel from per-source boundary lists (src_off over sender-local ids,
// global destinations) and the receiver's global -> local map.  Sources are
// ascending within each slot, so reductions over a slot add in a fixed order.
void build_channel(const std::vector<int64_t> &src_off, const std::vector<int32_t> &dstg,
                   const std::vector<int32_t> &wts, const std::vector<int32_t> &recv_l_of_g, int64_t recv_n,
                   Channel &ch) {
  const int64_t nsrc = (int64_t)src_off.size() - 1;
  const int64_t ne = (int64_t)dstg.size();
  const bool weighted = !wts.empty();
  std::vector<int64_t> cnt((size_t)recv_n + 1, 0);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < ne; ++e) __atomic_fetch_add(&cnt[(size_t)recv_l_of_g[dstg[e]] + 1], (int64_t)1, __ATOMIC_RELAXED);
  // slots: receiver vertices with at least one incoming boundary edge
  std::vector<int32_t> slot_of((size_t)recv_n, -1);
  ch.dst.clear();
  ch.roff.assign(1, 0);
  for (int64_t x = 0; x < recv_n; ++x)
    if (cnt[x + 1] > 0) {
      slot_of[x] = (int32_t)ch.dst.size();
      ch.dst.push_back((int32_t)x);
      ch.roff.push_back(ch.roff.back() + cnt[x + 1]);
    }
  ch.nslots = (int64_t)ch.dst.size();
  ch.rsrc.resize((size_t)ne);
  ch.rw.resize(weighted ? (size_t)ne : 0);
  std::vector<int64_t> cur(ch.roff.begin(), ch.roff.end() - 1);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t u = 0; u < nsrc; ++u)
    for (int64_t e = src_off[u]; e < src_off[u + 1]; ++e) {
      const int32_t sl = slot_of[recv_l_of_g[dstg[e]]];
      const int64_t k = __atomic_fetch_add(&cur[sl], (int64_t)1, __ATOMIC_RELAXED);
      ch.rsrc[k] = (int32_t)u;
      if (weighted) ch.rw[k] = wts[e];
    }
  // the scatter above fills each slot in no fixed order: sort it
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t sl = 0; sl < ch.nslots; ++sl) {
    const int64_t b = ch.roff[sl], en = ch.roff[sl + 1];
    if (!weighted) {
      std::sort(ch.rsrc.begin() + b, ch.rsrc.begin() + en);
      continue;
    }
    std::vector<int64_t> pr((size_t)(en - b));
    for (int64_t k = b; k < en; ++k) pr[k - b] = ((int64_t)ch.rsrc[k] << 32) | (uint32_t)ch.rw[k];
    std::sort(pr.begin(), pr.end());
    for (int64_t k = b; k < en; ++k) {
      ch.rsrc[k] = (int32_t)(pr[k - b] >> 32);
      ch.rw[k] = (int32_t)(uint32_t)(pr[k - b] & 0xFFFFFFFFu);
    }
  }
}

template <typename T>
int up(DevArena &a, T **d, const T *h, size_t n) {
  TG_TRY(dalloc(a, d, n));
  if (n) TG_HIP(hipMemcpy(*d, h, n * sizeof(T), hipMemcpyHostToDevice));
  return TG_OK;
}

}  // namespace

// ------------------------------------------------------------ static checks
// Every index the outbox, inbox and staging kernels take from the partition
// (not from a frontier) comes from the structures built here, so they are
// checked once, on the host: the channels' slot lists and reverse CSRs, the
// slot order and the static plan over slots, including a replay of the
// mapping from each virtual block of the plan to its slots and edge ranges
// (the arithmetic of assign_work_rows).
namespace {

int check_channel(const Channel &ch, int64_t sender_n, int64_t receiver_n, bool weighted, const char *name) {
  if ((int64_t)ch.dst.size() != ch.nslots || (int64_t)ch.roff.size() != ch.nslots + 1 || ch.roff[0] != 0)
    return set_error(TG_EDEVICE, "hybrid %s: slot arrays of inconsistent length", name);
  if (ch.roff.back() != (int64_t)ch.rsrc.size() || (weighted && ch.rw.size() != ch.rsrc.size()))
    return set_error(TG_EDEVICE, "hybrid %s: reverse CSR length", name);
  for (int64_t k = 0; k < ch.nslots; ++k) {
    if (ch.roff[k + 1] <= ch.roff[k]) return set_error(TG_EDEVICE, "hybrid %s: slot %lld has no source", name, (long long)k);
    if (ch.dst[k] < 0 || ch.dst[k] >= receiver_n || (k > 0 && ch.dst[k] <= ch.dst[k - 1]))
      return set_error(TG_EDEVICE, "hybrid %s: slot %lld receiver id out of range or not ascending", name,
                       (long long)k);
  }
  for (size_t e = 0; e < ch.rsrc.size(); ++e)
    if (ch.rsrc[e] < 0 || ch.rsrc[e] >= sender_n)
      return set_error(TG_EDEVICE, "hybrid %s: source %d of entry %zu out of range", name, ch.rsrc[e], e);
  return TG_OK;
}

int check_hybrid(const tg_partition &p, const std::vector<int32_t> &sorder, const std::vector<int64_t> &sdeg) {
  const HybridState &h = *p.hy;
  const CpuPart &C = h.cpu;
  const int64_t gn = p.gpu.n;
  TG_TRY(check_channel(h.g2c, gn, C.n, p.g->has_w, "GPU-to-host channel"));
  TG_TRY(check_channel(h.c2g, C.n, gn, p.g->has_w, "host-to-GPU channel"));
  const Channel &o = h.g2c;
  // slot order: a permutation, by non-increasing source count
  std::vector<char> seen((size_t)o.nslots, 0);
  for (int64_t i = 0; i < o.nslots; ++i) {
    const int32_t sl = sorder[i];
    if (sl < 0 || sl >= o.nslots || seen[sl]) return set_error(TG_EDEVICE, "hybrid: slot order is not a permutation");
    seen[sl] = 1;
    if (sdeg[i] != o.roff[sl + 1] - o.roff[sl] || (i > 0 && sdeg[i] > sdeg[i - 1]))
      return set_error(TG_EDEVICE, "hybrid: slot order is not by source count");
  }
  // the static plan and a replay of its virtual blocks
  const Plan &P = h.h_splan;
  if (P.count != o.nslots || P.pos[0] != 0 || P.pos[NBIN] != o.nslots)
    return set_error(TG_EDEVICE, "hybrid: slot plan does not cover the slots");
  for (int b = 0; b < NBIN; ++b)
    if (P.pos[b + 1] < P.pos[b] || P.vb[b + 1] < P.vb[b]) return set_error(TG_EDEVICE, "hybrid: slot plan not monotone");
  const int64_t nh = P.pos[1] - P.pos[0], hc = h.splan_hub_chunk;
  std::vector<int64_t> hubpref((size_t)nh + 1, 0);
  for (int64_t k = 0; k < nh; ++k) hubpref[k + 1] = hubpref[k] + (sdeg[k] + hc - 1) / hc;
  if (P.vb[1] != hubpref[nh]) return set_error(TG_EDEVICE, "hybrid: hub chunks of the slot plan");
  std::vector<int64_t> covered((size_t)o.nslots, 0);
  for (int64_t vb = 0; vb < P.vb[NBIN]; ++vb) {
    int b = 0;
    for (int k = 1; k < NBIN; ++k) b += vb >= P.vb[k] ? 1 : 0;
    const int64_t local = vb - P.vb[b];
    if (b == BIN_HUB) {
      const int64_t i = std::upper_bound(hubpref.begin(), hubpref.end(), local) - hubpref.begin() - 1;
      if (i < 0 || i >= nh || local >= hubpref[nh]) return set_error(TG_EDEVICE, "hybrid: hub virtual block %lld", (long long)vb);
      const int32_t sl = sorder[P.pos[0] + i];
      const int64_t e0 = o.roff[sl] + (local - hubpref[i]) * hc;
      const int64_t e1 = std::min<int64_t>(e0 + hc, o.roff[sl + 1]);
      if (e0 < o.roff[sl] || e0 >= e1) return set_error(TG_EDEVICE, "hybrid: hub chunk %lld of slot %d", (long long)vb, sl);
      covered[sl] += e1 - e0;
      continue;
    }
    if (b == BIN_ZERO) return set_error(TG_EDEVICE, "hybrid: a slot in the empty bin");
    for (int t = 0; t < BLOCK; t += lanes_per_vertex(b)) {
      const int64_t qi = P.pos[b] + local * verts_per_vblock(b) + t / lanes_per_vertex(b);
      if (qi >= P.pos[b + 1]) break;
      const int32_t sl = sorder[qi];
      covered[sl] += o.roff[sl + 1] - o.roff[sl];
    }
  }
  for (int64_t sl = 0; sl < o.nslots; ++sl)
    if (covered[sl] != o.roff[sl + 1] - o.roff[sl])
      return set_error(TG_EDEVICE, "hybrid: slot plan covers %lld of the %lld sources of slot %lld", (long long)covered[sl],
                       (long long)(o.roff[sl + 1] - o.roff[sl]), (long long)sl);
  // the host partition's own CSRs and id maps
  if ((int64_t)C.off.size() != C.n + 1 || C.off.back() != C.m || (int64_t)C.g_of_l.size() != C.n)
    return set_error(TG_EDEVICE, "hybrid: host partition CSR");
  for (int32_t x : C.col)
    if (x < 0 || x >= C.n) return set_error(TG_EDEVICE, "hybrid: host edge target out of range");
  for (int64_t i = 0; i < C.n; ++i)
    if (C.g_of_l[i] < 0 || C.g_of_l[i] >= p.g->n || p.h_l_of_g[C.g_of_l[i]] >= 0)
      return set_error(TG_EDEVICE, "hybrid: host vertex %lld is not a host-only vertex", (long long)i);
  return TG_OK;
}

}  // namespace

// ------------------------------------------------------------------ building
int build_hybrid(tg_partition *p, uint64_t seed) {
  const tg_graph &G = *p->g;
  const int64_t V = G.n;
  if (V == 0) return set_error(TG_EINVAL, "hybrid partition of an empty graph");
  std::vector<int32_t> order((size_t)V);
  for (int64_t v = 0; v < V; ++v) order[v] = (int32_t)v;
  auto deg = [&](int32_t v) { return G.off[v + 1] - G.off[v]; };
  if (p->strategy != TG_PART_RAND) {
    // by degree, ties by id: HIGH decreasing, LOW increasing (counting sort)
    std::vector<int64_t> key((size_t)V);
    int64_t maxd = 0;
    for (int64_t v = 0; v < V; ++v) maxd = std::max<int64_t>(maxd, deg((int32_t)v));
    for (int64_t v = 0; v < V; ++v) key[v] = p->strategy == TG_PART_HIGH ? deg((int32_t)v) : maxd - deg((int32_t)v);
    sort_desc_by_key(key, order);
  } else {
    std::vector<uint64_t> key((size_t)V);
    for (int64_t v = 0; v < V; ++v) key[v] = mix64(seed * 0x9E3779B97F4A7C15ULL + (uint64_t)v + 1);
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  }
  // host partition: whole vertices in strategy order until >= alpha * E edges
  const double want = p->alpha * (double)G.m;
  std::vector<char> on_cpu((size_t)V, 0);
  int64_t taken = 0, cpu_edges = 0;
  while (taken < V && (double)cpu_edges < want) {
    on_cpu[order[taken]] = 1;
    cpu_edges += deg(order[taken]);
    ++taken;
  }
  if (taken == 0) return set_error(TG_EINVAL, "cpu_edge_share too small to place any vertex on the host");
  if (taken == V) return set_error(TG_EINVAL, "cpu_edge_share leaves no vertex on the GPU");
  std::vector<int32_t> gpu_verts, cpu_verts;
  gpu_verts.reserve((size_t)(V - taken));
  cpu_verts.reserve((size_t)taken);
  for (int64_t v = 0; v < V; ++v) (on_cpu[v] ? cpu_verts : gpu_verts).push_back((int32_t)v);

  BoundaryEdges gb;
  TG_TRY(build_gpu_part(p, gpu_verts, &gb));

  auto *hy = new (std::nothrow) HybridState();
  if (!hy) return set_error(TG_ENOMEM, "hybrid: out of host memory");
  p->hy = hy;
  CpuPart &C = hy->cpu;
  // host-local ids by decreasing local out-degree
  std::vector<int32_t> c_l_of_g((size_t)V, -1);
  for (int32_t v : cpu_verts) c_l_of_g[v] = 0;
  std::vector<int64_t> ldeg((size_t)V, 0);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < (int64_t)cpu_verts.size(); ++i) {
    const int32_t u = cpu_verts[i];
    int64_t d = 0;
    for (int64_t e = G.off[u]; e < G.off[u + 1]; ++e) d += c_l_of_g[G.col[e]] >= 0;
    ldeg[u] = d;
  }
  C.g_of_l = cpu_verts;
  std::stable_sort(C.g_of_l.begin(), C.g_of_l.end(), [&](int32_t a, int32_t b) { return ldeg[a] > ldeg[b]; });
  C.n = (int64_t)C.g_of_l.size();
  for (int64_t i = 0; i < C.n; ++i) c_l_of_g[C.g_of_l[i]] = (int32_t)i;
  C.off.assign((size_t)C.n + 1, 0);
  std::vector<int64_t> cb_off((size_t)C.n + 1, 0);
  for (int64_t i = 0; i < C.n; ++i) {
    const int32_t u = C.g_of_l[i];
    C.off[i + 1] = C.off[i] + ldeg[u];
    cb_off[i + 1] = cb_off[i] + deg(u) - ldeg[u];
  }
  C.m = C.off[C.n];
  C.col.resize((size_t)C.m);
  if (G.has_w) C.w.resize((size_t)C.m);
  std::vector<int32_t> cb_dst((size_t)cb_off[C.n]), cb_w(G.has_w ? (size_t)cb_off[C.n] : 0);
  C.bdeg.resize((size_t)C.n);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < C.n; ++i) {
    const int32_t u = C.g_of_l[i];
    std::vector<std::pair<int32_t, int32_t>> loc;
    int64_t k = C.off[i], b = cb_off[i];
    for (int64_t e = G.off[u]; e < G.off[u + 1]; ++e) {
      const int32_t l = c_l_of_g[G.col[e]];
      if (l >= 0) {
        loc.emplace_back(l, G.has_w ? G.w[e] : 0);
      } else {
        cb_dst[b] = G.col[e];
        if (G.has_w) cb_w[b] = G.w[e];
        ++b;
      }
    }
    std::sort(loc.begin(), loc.end());
    for (auto &pr : loc) {
      C.col[k] = pr.first;
      if (G.has_w) C.w[k] = pr.second;
      ++k;
    }
    C.bdeg[i] = (int32_t)(cb_off[i + 1] - cb_off[i]);
  }
  // host in-edges
  transpose_csr(C.n, C.off, C.col, C.ioff, C.icol);
  for (int64_t i = 0; i < C.n; ++i) C.n_dangling += (C.off[i + 1] == C.off[i] && C.bdeg[i] == 0);

  // channels: GPU -> host uses the GPU's boundary edges, host -> GPU the host's
  build_channel(gb.src_off, gb.dst, gb.w, c_l_of_g, C.n, hy->g2c);
  build_channel(cb_off, cb_dst, cb_w, p->h_l_of_g, p->gpu.n, hy->c2g);
  C.l_of_g = std::move(c_l_of_g);
  hy->raw_boundary_edges = (int64_t)gb.dst.size() + (int64_t)cb_dst.size();

  // device side
  GpuPart &g = p->gpu;
  DevArena &A = hy->arena;
  Channel &o = hy->g2c;
  TG_TRY(up(A, &hy->d_roff, o.roff.data(), o.roff.size()));
  TG_TRY(up(A, &hy->d_rsrc, o.rsrc.data(), std::max<size_t>(o.rsrc.size(), 1)));
  if (G.has_w) TG_TRY(up(A, &hy->d_rw, o.rw.data(), std::max<size_t>(o.rw.size(), 1)));
  // slots ordered by decreasing source count: the gather's degree bins
  std::vector<int32_t> sorder((size_t)o.nslots);
  for (int64_t i = 0; i < o.nslots; ++i) sorder[i] = (int32_t)i;
  std::stable_sort(sorder.begin(), sorder.end(), [&](int32_t a, int32_t b) {
    return o.roff[a + 1] - o.roff[a] > o.roff[b + 1] - o.roff[b];
  });
  std::vector<int64_t> sdeg((size_t)o.nslots);
  for (int64_t i = 0; i < o.nslots; ++i) sdeg[i] = o.roff[sorder[i] + 1] - o.roff[sorder[i]];
  TG_TRY(up(A, &hy->d_slot_order, sorder.data(), std::max<size_t>(sorder.size(), 1)));
  {
    // static plan over the slots (same bins as the vertex kernels)
    BinBounds bb{};
    int64_t i = 0;
    for (int b = 0; b < NBIN; ++b) {
      while (i < o.nslots && bin_of_degree(sdeg[i], p->tune) < b) ++i;
      bb.bstart[b] = i;
    }
    bb.bstart[NBIN] = o.nslots;
    Plan &P = hy->h_splan;
    memset(&P, 0, sizeof(P));
    P.count = (int32_t)o.nslots;
    for (int b = 0; b <= NBIN; ++b) P.pos[b] = (int32_t)bb.bstart[b];
    const int64_t nh = bb.bstart[1];
    std::vector<int64_t> hubpref((size_t)nh + 1, 0);
    for (int64_t k = 0; k < nh; ++k) hubpref[k + 1] = hubpref[k] + (sdeg[k] + p->tune.hub_chunk - 1) / p->tune.hub_chunk;
    int64_t vb = hubpref[nh];
    P.vb[0] = 0;
    P.vb[1] = vb;
    for (int b = 1; b < NBIN; ++b) {
      if (b != BIN_ZERO) vb += (P.pos[b + 1] - P.pos[b] + verts_per_vblock(b) - 1) / verts_per_vblock(b);
      P.vb[b + 1] = vb;
    }
    hy->splan_hub_chunk = p->tune.hub_chunk;
    TG_TRY(up(A, &hy->d_shubpref, hubpref.data(), hubpref.size()));
    TG_TRY(up(A, &hy->d_splan, &P, 1));
    TG_TRY(dalloc(A, &hy->d_shub_partials_f, (size_t)hubpref[nh] + 1));
    TG_TRY(dalloc(A, &hy->d_shub_partials_i, (size_t)hubpref[nh] + 1));
  }
  const size_t no = (size_t)std::max<int64_t>(o.nslots, 1), ni = (size_t)std::max<int64_t>(hy->c2g.nslots, 1);
  TG_TRY(dalloc(A, &hy->d_out_i, no));
  TG_TRY(dalloc(A, &hy->d_out_f, no));
  TG_TRY(up(A, &hy->d_in_dst, hy->c2g.dst.data(), std::max<size_t>(hy->c2g.dst.size(), 1)));
  TG_TRY(dalloc(A, &hy->d_in_i, ni));
  TG_TRY(dalloc(A, &hy->d_in_f, ni));
  std::vector<int32_t> gb_deg((size_t)g.n);
  for (int64_t i = 0; i < g.n; ++i) gb_deg[i] = (int32_t)(gb.src_off[i + 1] - gb.src_off[i]);
  TG_TRY(up(A, &hy->d_bdeg, gb_deg.data(), std::max<size_t>(gb_deg.size(), 1)));
  TG_TRY(dalloc(A, &hy->d_ghost, (size_t)std::max<int64_t>(g.n, 1)));
  TG_TRY(up(A, &hy->d_cpu_g_of_l, C.g_of_l.data(), (size_t)C.n));
  TG_TRY(dalloc(A, &hy->d_stage, (size_t)C.n));
  TG_HIP(hipHostMalloc((void **)&hy->h_out_i, no * sizeof(int64_t), hipHostMallocDefault));
  TG_HIP(hipHostMalloc((void **)&hy->h_in_i, ni * sizeof(int64_t), hipHostMallocDefault));
  TG_HIP(hipHostMalloc((void **)&hy->h_out_f, no * sizeof(double), hipHostMallocDefault));
  TG_HIP(hipHostMalloc((void **)&hy->h_in_f, ni * sizeof(double), hipHostMallocDefault));
  TG_HIP(hipHostMalloc((void **)&hy->h_stage, (size_t)C.n * sizeof(int32_t), hipHostMallocDefault));
  return check_hybrid(*p, sorder, sdeg);
}

void hybrid_free(tg_partition *p) {
  delete p->hy;
  p->hy = nullptr;
}

std::string hybrid_info_json(const tg_partition *p) {
  if (!p->hy) return "";
  const HybridState &h = *p->hy;
  // space of a partition (section 4.3.3): eid*|V| + vid*|E| + w*|E| + (vid+s)*(|Vi| + |Vo|),
  // with 8-byte offsets, 4-byte ids, 4-byte weights and 4-byte messages
  auto space = [&](int64_t n, int64_t m, int64_t vin, int64_t vout) {
    return 8 * (n + 1) + 4 * m + (p->g->has_w ? 4 * m : 0) + 8 * (vin + vout);
  };
  char buf[1024];
  snprintf(buf, sizeof(buf),
           ",\"cpu_vertices\":%lld,\"cpu_edges\":%lld,\"cpu_boundary_edges\":%lld,\"boundary_edges\":%lld,"
           "\"outbox_gpu_to_cpu\":%lld,"
           "\"outbox_cpu_to_gpu\":%lld,\"beta_raw\":%.6f,\"beta_reduced\":%.6f,\"gpu_space_bytes\":%lld,"
           "\"cpu_space_bytes\":%lld",
           (long long)h.cpu.n, (long long)h.cpu.m, (long long)h.c2g.edges(), (long long)h.raw_boundary_edges,
           (long long)h.g2c.nslots,
           (long long)h.c2g.nslots, (double)h.raw_boundary_edges / (double)std::max<int64_t>(p->g->m, 1),
           (double)(h.g2c.nslots + h.c2g.nslots) / (double)std::max<int64_t>(p->g->m, 1),
           (long long)space(p->gpu.n, p->gpu.m, h.c2g.nslots, h.g2c.nslots),
           (long long)space(h.cpu.n, h.cpu.m, h.g2c.nslots, h.c2g.nslots));
  return buf;
}

// ------------------------------------------------------------- GPU kernels
namespace {

constexpr int64_t I64_INF = INT64_MAX;

// BFS outbox: a slot gets L+1 if any of its sources is on the frontier L.
struct BfsOutbox {
  using T = int64_t;
  const int32_t *rsrc;
  const int32_t *level;
  int32_t L;
  int64_t *msg;
  __device__ static int64_t identity() { return I64_INF; }
  __device__ static int64_t combine(int64_t a, int64_t b) { return a < b ? a : b; }
  __device__ int32_t vstate(int32_t) const { return 0; }
  __device__ int64_t term(int32_t, int64_t e) const { return level[rsrc[e]] == L ? (int64_t)L + 1 : I64_INF; }
  __device__ void finish(int32_t slot, int64_t r) const { msg[slot] = r; }
};

// SSSP outbox: least dist(src) + w over sources that relaxed this superstep.
struct SsspOutbox {
  using T = int64_t;
  const int32_t *rsrc;
  const int32_t *rw;
  const int32_t *dist;
  const uint32_t *cur;
  int64_t *msg;
  __device__ static int64_t identity() { return I64_INF; }
  __device__ static int64_t combine(int64_t a, int64_t b) { return a < b ? a : b; }
  __device__ int32_t vstate(int32_t) const { return 0; }
  __device__ int64_t term(int32_t, int64_t e) const {
    const int32_t u = rsrc[e];
    return ((cur[u >> 5] >> (u & 31)) & 1u) ? (int64_t)dist[u] + (int64_t)rw[e] : I64_INF;
  }
  __device__ void finish(int32_t slot, int64_t r) const { msg[slot] = r; }
};

// PageRank outbox: sum of contributions c(src) bound for one remote vertex.
struct PrOutbox : SumF64 {
  const int32_t *rsrc;
  const float *c;
  double *msg;
  __device__ int32_t vstate(int32_t) const { return 0; }
  __device__ double term(int32_t, int64_t e) const { return (double)c[rsrc[e]]; }
  __device__ void finish(int32_t slot, double r) const { msg[slot] = r; }
};

// Sets bit v of the bitmap for every lane with `on`.  Lanes with ascending
// ids hit the same 32-bit word in runs; each run ORs its bits together with
// shuffles and only its first lane issues the atomic, so one word gets one
// atomic instead of up to 32 (atomics on one address serialize).  Every lane
// of the wave must call it.
__device__ __forceinline__ void wave_or_bits(uint32_t *bits, int32_t v, bool on) {
  if (!__ballot(on)) return;  // the same for the whole wave
  const int lane = threadIdx.x & 63;
  const int32_t w = on ? (v >> 5) : -1;
  uint32_t b = on ? (1u << (v & 31)) : 0u;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t ow = __shfl_down(w, o, 64);
    const uint32_t ob = __shfl_down(b, o, 64);
    if (lane + o < 64 && ow == w) b |= ob;
  }
  const int32_t pw = __shfl_up(w, 1, 64);
  if (on && (lane == 0 || pw != w)) atomicOr(bits + w, b);
}

// Inbox vertices are ascending by slot, so a wave's visited bits come in
// runs on a few words (wave_or_bits).
__global__ __launch_bounds__(BLOCK) void k_inbox_bfs(const int32_t *__restrict__ dst,
                                                     const int64_t *__restrict__ msg, int64_t n, uint32_t *visited) {
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool on = k < n && msg[k] != I64_INF;
  wave_or_bits(visited, on ? dst[k] : 0, on);
}

__global__ __launch_bounds__(BLOCK) void k_inbox_sssp(const int32_t *__restrict__ dst,
                                                      const int64_t *__restrict__ msg, int64_t n, int32_t *dist,
                                                      uint32_t *active, uint32_t *ovf, uint32_t *flags) {
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  int32_t v = 0;
  bool act = false;
  if (k < n && msg[k] != I64_INF) {
    v = dst[k];
    const int64_t m = msg[k];
    if (m >= (int64_t)TG_INF) {
      if (dist[v] == TG_INF) {
        atomicOr(ovf + (v >> 5), 1u << (v & 31));
        flags[0] = 1u;
      }
    } else if (m < (int64_t)dist[v]) {  // inbox ids are distinct: no other writer
      dist[v] = (int32_t)m;
      act = true;
    }
  }
  wave_or_bits(active, v, act);
}

__global__ void k_inbox_pr(const int32_t *__restrict__ dst, const double *__restrict__ msg, int64_t n,
                           double *ghost) {
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k < n) ghost[dst[k]] = msg[k];
}

__global__ void k_scatter_stage_i32(const int32_t *__restrict__ g_of_l, const int32_t *__restrict__ st, int64_t n,
                                    int32_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) out[g_of_l[i]] = st[i];
}

__global__ void k_scatter_stage_f32(const int32_t *__restrict__ g_of_l, const float *__restrict__ st, int64_t n,
                                    float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) out[g_of_l[i]] = st[i];
}

__global__ void k_set_i32h(int32_t *p, int64_t i, int32_t v) {
  if (threadIdx.x == 0) p[i] = v;
}

inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>((n + BLOCK - 1) / BLOCK, 1); }

// The slot plan, its hub chunk prefix and the partials buffer were sized at
// partition time with splan_hub_chunk; a later retune must not change the
// chunking they were built for.
template <class Op>
int launch_outbox(HybridState &h, hipStream_t s, Op op, typename Op::T *partials) {
  if (h.g2c.nslots == 0) return TG_OK;
  hipLaunchKernelGGL(k_gather<Op>, dim3(launch_grid(h.h_splan.vb[NBIN])), dim3(BLOCK), 0, s, h.d_splan,
                     h.d_slot_order, h.d_shubpref, h.d_roff, h.splan_hub_chunk, partials, op);
  if (h.h_splan.pos[1] > h.h_splan.pos[0])
    hipLaunchKernelGGL(k_gather_hubs<Op>, dim3(64), dim3(BLOCK), 0, s, h.d_splan, h.d_slot_order, h.d_shubpref,
                       partials, op);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

// host-side atomics on plain arrays
inline bool test_and_set(uint8_t *flag) { return __atomic_exchange_n(flag, (uint8_t)1, __ATOMIC_RELAXED) != 0; }
inline bool atomic_min_i32(int32_t *p, int32_t v) {
  int32_t cur = __atomic_load_n(p, __ATOMIC_RELAXED);
  while (v < cur)
    if (__atomic_compare_exchange_n(p, &cur, v, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) return true;
  return false;
}

void concat(std::vector<std::vector<int32_t>> &parts, std::vector<int32_t> &out) {
  out.clear();
  for (auto &v : parts) {
    out.insert(out.end(), v.begin(), v.end());
    v.clear();
  }
}

// Per-call accounting.  cpu_edges: out-edges (local and boundary) of the
// host vertices the host processed; h2d_bytes: the host-to-GPU part of
// exchange_bytes, the part exchange_ms times (BFS).
struct Phase {
  double gpu_ms = 0, cpu_ms = 0, exchange_ms = 0, bytes = 0, cpu_edges = 0, h2d_bytes = 0;
  int64_t supersteps = 0;
};

void add_phase_stats(const Phase &ph) {
  stats_add("supersteps", (double)ph.supersteps);
  stats_add("gpu_ms", ph.gpu_ms);
  stats_add("cpu_ms", ph.cpu_ms);
  stats_add("exchange_ms", ph.exchange_ms);
  stats_add("exchange_bytes", ph.bytes);
  stats_add("exchange_h2d_bytes", ph.h2d_bytes);
  stats_add("cpu_edges", ph.cpu_edges);
}

// Out-edges of a host frontier, local and boundary.
double frontier_edges(const CpuPart &C, const std::vector<int32_t> &front) {
  double s = 0;
  for (int32_t v : front) s += (double)(C.off[v + 1] - C.off[v] + C.bdeg[v]);
  return s;
}

}  // namespace

// ------------------------------------------------------------------- BFS
int hybrid_bfs(tg_partition *p, const int32_t *roots, int32_t nr, int32_t *levels, int32_t *parents,
               hipStream_t s) {
  if (parents) return set_error(TG_EUNSUPPORTED, "bfs: parents are not produced on hybrid partitions");
  HybridState &h = *p->hy;
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  CpuPart &C = h.cpu;
  const Tuning &t = p->tune;
  TG_TRY(ws.ensure(g, 0));
  const int64_t V = p->g->n;
  std::vector<uint8_t> cvis((size_t)C.n);
  std::vector<int32_t> clev((size_t)C.n);
  std::vector<int32_t> cfront, cnext;
  std::vector<std::vector<int32_t>> tl((size_t)omp_get_max_threads());
  Phase ph;
  hipEvent_t e0, e1, e2, e3;
  TG_HIP(hipEventCreate(&e0));
  TG_HIP(hipEventCreate(&e1));
  TG_HIP(hipEventCreate(&e2));
  TG_HIP(hipEventCreate(&e3));
  int rc = TG_OK;
  for (int32_t r = 0; r < nr && rc == TG_OK; ++r) {
    const int32_t root = roots[r];
    const int32_t gl = p->h_l_of_g[root];
    uint32_t *visited = ws.bits_a, *prev = ws.bits_b;
    TG_HIP(hipMemsetAsync(visited, 0, ws.nwords * sizeof(uint32_t), s));
    TG_HIP(hipMemsetAsync(prev, 0, ws.nwords * sizeof(uint32_t), s));
    TG_TRY(fill_i32(ws.state, g.n, TG_INF, s));
    std::fill(cvis.begin(), cvis.end(), 0);
    std::fill(clev.begin(), clev.end(), TG_INF);
    cfront.clear();
    if (gl >= 0) {
      TG_TRY(set_bit(visited, gl, s));
    } else {
      const int32_t cl = C.l_of_g[root];
      if (cl < 0) return set_error(TG_EDEVICE, "hybrid bfs: root %d is on neither side", root);
      cvis[cl] = 1;
      clev[cl] = 0;
      cfront.push_back(cl);
    }
    TG_TRY(frontier_compact(g, ws, 0, visited, prev, ws.queue, ws.state, 0, s));
    TG_TRY(frontier_plan(g, ws, ws.queue, t, s, true));
    for (int32_t L = 0;; ++L) {
      if (ws.h_plan->count == 0 && cfront.empty()) break;
      if (L > V) return set_error(TG_EDEVICE, "hybrid bfs: more supersteps than vertices");
      ++ph.supersteps;
      // GPU: expand the local frontier, reduce the outbox, start its copy
      TG_HIP(hipEventRecord(e0, s));
      TG_TRY(bfs_expand_launch(g, ws, ws.queue, ws.h_plan->vb[NBIN], t, s));
      TG_TRY(launch_outbox(h, s, BfsOutbox{h.d_rsrc, ws.state, L, h.d_out_i}, h.d_shub_partials_i));
      TG_HIP(hipEventRecord(e1, s));
      if (h.g2c.nslots)
        TG_HIP(hipMemcpyAsync(h.h_out_i, h.d_out_i, h.g2c.nslots * sizeof(int64_t), hipMemcpyDeviceToHost, s));
      // host: expand its frontier and reduce its outbox while the GPU runs
      const auto tc = clk::now();
#pragma omp parallel
      {
        auto &mine = tl[omp_get_thread_num()];
#pragma omp for schedule(dynamic, 64)
        for (size_t i = 0; i < cfront.size(); ++i) {
          const int32_t v = cfront[i];
          for (int64_t e = C.off[v]; e < C.off[v + 1]; ++e) {
            const int32_t x = C.col[e];
            if (!cvis[x] && !test_and_set(&cvis[x])) {
              clev[x] = L + 1;
              mine.push_back(x);
            }
          }
        }
#pragma omp for schedule(dynamic, 256)
        for (int64_t k = 0; k < h.c2g.nslots; ++k) {
          int64_t m = I64_INF;
          for (int64_t e = h.c2g.roff[k]; e < h.c2g.roff[k + 1] && m == I64_INF; ++e)
            if (clev[h.c2g.rsrc[e]] == L) m = L + 1;
          h.h_in_i[k] = m;
        }
      }
      concat(tl, cnext);
      ph.cpu_ms += ms_since(tc);
      ph.cpu_edges += frontier_edges(C, cfront);
      // exchange: host messages to the GPU inbox; fold them in and compact
      TG_HIP(hipEventRecord(e2, s));
      if (h.c2g.nslots) {
        TG_HIP(hipMemcpyAsync(h.d_in_i, h.h_in_i, h.c2g.nslots * sizeof(int64_t), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_inbox_bfs, dim3(nblk(h.c2g.nslots)), dim3(BLOCK), 0, s, h.d_in_dst, h.d_in_i,
                           h.c2g.nslots, visited);
      }
      TG_HIP(hipEventRecord(e3, s));
      TG_TRY(frontier_compact(g, ws, 0, visited, prev, ws.queue, ws.state, L + 1, s));
      TG_TRY(frontier_plan(g, ws, ws.queue, t, s, true));  // waits: GPU messages are on the host
      float a = 0, b = 0;
      TG_QUIET(hipEventElapsedTime(&a, e0, e1));
      TG_QUIET(hipEventElapsedTime(&b, e2, e3));
      ph.gpu_ms += a;
      ph.exchange_ms += b;
      ph.bytes += (double)(h.g2c.nslots + h.c2g.nslots) * sizeof(int64_t);
      ph.h2d_bytes += (double)h.c2g.nslots * sizeof(int64_t);
      const auto tc2 = clk::now();
      for (int64_t k = 0; k < h.g2c.nslots; ++k) {
        if (h.h_out_i[k] == I64_INF) continue;
        const int32_t x = h.g2c.dst[k];
        if (!cvis[x]) {
          cvis[x] = 1;
          clev[x] = L + 1;
          cnext.push_back(x);
        }
      }
      cfront.swap(cnext);
      ph.cpu_ms += ms_since(tc2);
    }
    TG_TRY(collect_levels(g, ws.bits_a, ws.state, levels + (int64_t)r * V, s));
    memcpy(h.h_stage, clev.data(), (size_t)C.n * sizeof(int32_t));
    TG_HIP(hipMemcpyAsync(h.d_stage, h.h_stage, (size_t)C.n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_scatter_stage_i32, dim3(nblk(C.n)), dim3(BLOCK), 0, s, h.d_cpu_g_of_l, h.d_stage, C.n,
                       levels + (int64_t)r * V);
    TG_HIP(hipStreamSynchronize(s));
  }
  TG_QUIET(hipEventDestroy(e0));
  TG_QUIET(hipEventDestroy(e1));
  TG_QUIET(hipEventDestroy(e2));
  TG_QUIET(hipEventDestroy(e3));
  stats_add("roots", nr);
  add_phase_stats(ph);
  ktimer_emit();
  return rc;
}

// ------------------------------------------------------------------ SSSP
int hybrid_sssp(tg_partition *p, const int32_t *roots, int32_t nr, int32_t *dist_out, hipStream_t s) {
  HybridState &h = *p->hy;
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  CpuPart &C = h.cpu;
  const Tuning &t = p->tune;
  TG_TRY(ws.ensure(g, 0));
  const int64_t V = p->g->n;
  std::vector<int32_t> cdist((size_t)C.n);
  std::vector<uint8_t> cin_next((size_t)C.n), cin_cur((size_t)C.n), covf((size_t)C.n);
  std::vector<int32_t> cfront, cnext;
  std::vector<std::vector<int32_t>> tl((size_t)omp_get_max_threads());
  Phase ph;
  for (int32_t r = 0; r < nr; ++r) {
    const int32_t root = roots[r];
    const int32_t gl = p->h_l_of_g[root];
    uint32_t *active = ws.bits_a, *cur = ws.bits_b, *ovf = ws.bits_c;
    int32_t *dist = ws.state;
    TG_TRY(fill_i32(dist, g.n, TG_INF, s));
    TG_HIP(hipMemsetAsync(active, 0, ws.nwords * sizeof(uint32_t), s));
    TG_HIP(hipMemsetAsync(cur, 0, ws.nwords * sizeof(uint32_t), s));
    TG_HIP(hipMemsetAsync(ovf, 0, ws.nwords * sizeof(uint32_t), s));
    TG_HIP(hipMemsetAsync(ws.counters, 0, 4 * sizeof(uint32_t), s));
    std::fill(cdist.begin(), cdist.end(), TG_INF);
    std::fill(cin_next.begin(), cin_next.end(), 0);
    std::fill(covf.begin(), covf.end(), 0);
    cfront.clear();
    bool cpu_overflow_candidate = false;
    if (gl >= 0) {
      hipLaunchKernelGGL(k_set_i32h, dim3(1), dim3(64), 0, s, dist, (int64_t)gl, 0);
      TG_TRY(set_bit(active, gl, s));
    } else {
      const int32_t cl = C.l_of_g[root];
      if (cl < 0) return set_error(TG_EDEVICE, "hybrid sssp: root %d is on neither side", root);
      cdist[cl] = 0;
      cfront.push_back(cl);
    }
    TG_TRY(frontier_compact(g, ws, 2, active, cur, ws.queue, nullptr, 0, s));
    TG_TRY(frontier_plan(g, ws, ws.queue, t, s, true));
    for (int64_t step = 0;; ++step) {
      if (ws.h_plan->count == 0 && cfront.empty()) break;
      if (step > V) return set_error(TG_EDEVICE, "hybrid sssp: no convergence");
      ++ph.supersteps;
      const auto tg0 = clk::now();
      TG_TRY(sssp_relax_launch(g, ws, ws.queue, ws.h_plan->vb[NBIN], t, s));
      TG_TRY(launch_outbox(h, s, SsspOutbox{h.d_rsrc, h.d_rw, dist, cur, h.d_out_i}, h.d_shub_partials_i));
      if (h.g2c.nslots)
        TG_HIP(hipMemcpyAsync(h.h_out_i, h.d_out_i, h.g2c.nslots * sizeof(int64_t), hipMemcpyDeviceToHost, s));
      // host: relax its frontier, reduce its outbox
      const auto tc = clk::now();
      std::fill(cin_cur.begin(), cin_cur.end(), 0);
      for (int32_t v : cfront) cin_cur[v] = 1;
#pragma omp parallel
      {
        auto &mine = tl[omp_get_thread_num()];
#pragma omp for schedule(dynamic, 64)
        for (size_t i = 0; i < cfront.size(); ++i) {
          const int32_t v = cfront[i];
          const int64_t dv = __atomic_load_n(&cdist[v], __ATOMIC_RELAXED);
          for (int64_t e = C.off[v]; e < C.off[v + 1]; ++e) {
            const int32_t x = C.col[e];
            const int64_t nd = dv + C.w[e];
            if (nd >= (int64_t)TG_INF) {
              if (__atomic_load_n(&cdist[x], __ATOMIC_RELAXED) == TG_INF) covf[x] = 1;
              continue;
            }
            if (atomic_min_i32(&cdist[x], (int32_t)nd) && !test_and_set(&cin_next[x])) mine.push_back(x);
          }
        }
#pragma omp for schedule(dynamic, 256)
        for (int64_t k = 0; k < h.c2g.nslots; ++k) {
          int64_t m = I64_INF;
          for (int64_t e = h.c2g.roff[k]; e < h.c2g.roff[k + 1]; ++e) {
            const int32_t u = h.c2g.rsrc[e];
            if (cin_cur[u]) m = std::min<int64_t>(m, (int64_t)cdist[u] + h.c2g.rw[e]);
          }
          h.h_in_i[k] = m;
        }
      }
      concat(tl, cnext);
      ph.cpu_ms += ms_since(tc);
      ph.cpu_edges += frontier_edges(C, cfront);
      if (h.c2g.nslots) {
        TG_HIP(hipMemcpyAsync(h.d_in_i, h.h_in_i, h.c2g.nslots * sizeof(int64_t), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_inbox_sssp, dim3(nblk(h.c2g.nslots)), dim3(BLOCK), 0, s, h.d_in_dst, h.d_in_i,
                           h.c2g.nslots, dist, active, ovf, ws.counters);
      }
      TG_TRY(frontier_compact(g, ws, 2, active, cur, ws.queue, nullptr, 0, s));
      TG_TRY(frontier_plan(g, ws, ws.queue, t, s, true));
      ph.gpu_ms += ms_since(tg0);
      ph.bytes += (double)(h.g2c.nslots + h.c2g.nslots) * sizeof(int64_t);
      ph.h2d_bytes += (double)h.c2g.nslots * sizeof(int64_t);
      const auto tc2 = clk::now();
      for (int64_t k = 0; k < h.g2c.nslots; ++k) {
        const int64_t m = h.h_out_i[k];
        if (m == I64_INF) continue;
        const int32_t x = h.g2c.dst[k];
        if (m >= (int64_t)TG_INF) {
          if (cdist[x] == TG_INF) covf[x] = 1;
          continue;
        }
        if (m < cdist[x]) {
          cdist[x] = (int32_t)m;
          if (!cin_next[x]) {
            cin_next[x] = 1;
            cnext.push_back(x);
          }
        }
      }
      for (int32_t x : cnext) cin_next[x] = 0;
      cfront.swap(cnext);
      ph.cpu_ms += ms_since(tc2);
    }
    for (int64_t i = 0; i < C.n; ++i)
      if (covf[i] && cdist[i] == TG_INF) cpu_overflow_candidate = true;
    TG_TRY(sssp_overflow_check(g, ws, s));
    if (ws.h_flags[1] || cpu_overflow_candidate)
      return set_error(TG_ERANGE, "sssp: a shortest-path distance does not fit below INT32_MAX");
    TG_TRY(collect_i32(g, dist, dist_out + (int64_t)r * V, s));
    memcpy(h.h_stage, cdist.data(), (size_t)C.n * sizeof(int32_t));
    TG_HIP(hipMemcpyAsync(h.d_stage, h.h_stage, (size_t)C.n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_scatter_stage_i32, dim3(nblk(C.n)), dim3(BLOCK), 0, s, h.d_cpu_g_of_l, h.d_stage, C.n,
                       dist_out + (int64_t)r * V);
    TG_HIP(hipStreamSynchronize(s));
  }
  stats_add("roots", nr);
  add_phase_stats(ph);
  ktimer_emit();
  return TG_OK;
}

// -------------------------------------------------------------- PageRank
int hybrid_pagerank(tg_partition *p, double damping, int32_t iters, int mode, float *rank, hipStream_t s) {
  HybridState &h = *p->hy;
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  CpuPart &C = h.cpu;
  const double N = (double)p->g->n;
  const double base = (1.0 - damping) / N;
  const bool drop = mode == TG_PR_DANGLING_DROP;
  double D = (double)(g.n_dangling + C.n_dangling) / N;
  TG_TRY(gpu_pagerank_setup(p, damping, mode, s, h.d_bdeg, D));
  TG_TRY(fill_f64(h.d_ghost, g.n, 0.0, s));
  std::vector<float> cc((size_t)C.n), cn((size_t)C.n), crank((size_t)C.n);
  std::vector<double> ghost((size_t)C.n, 0.0);
  for (int64_t i = 0; i < C.n; ++i) {
    const int64_t od = C.off[i + 1] - C.off[i] + C.bdeg[i];
    cc[i] = od > 0 ? (float)(1.0 / (N * (double)od)) : 0.0f;
  }
  Phase ph;
  if (iters == 0) {
    TG_TRY(pr_write_initial(g, rank, N, s));
    std::fill(crank.begin(), crank.end(), (float)(1.0 / N));
  }
  for (int32_t k = 0; k < iters; ++k) {
    ++ph.supersteps;
    const bool last = k == iters - 1;
    const auto tg0 = clk::now();
    // outboxes: per remote vertex, the sum of the contributions bound for it
    TG_TRY(launch_outbox(h, s, PrOutbox{{}, h.d_rsrc, ws.cbuf[k & 1], h.d_out_f}, h.d_shub_partials_f));
    if (h.g2c.nslots)
      TG_HIP(hipMemcpyAsync(h.h_out_f, h.d_out_f, h.g2c.nslots * sizeof(double), hipMemcpyDeviceToHost, s));
    const auto tc = clk::now();
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < h.c2g.nslots; ++q) {
      double m = 0.0;
      for (int64_t e = h.c2g.roff[q]; e < h.c2g.roff[q + 1]; ++e) m += (double)cc[h.c2g.rsrc[e]];
      h.h_in_f[q] = m;
    }
    ph.cpu_ms += ms_since(tc);
    if (h.c2g.nslots) {
      TG_HIP(hipMemcpyAsync(h.d_in_f, h.h_in_f, h.c2g.nslots * sizeof(double), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_inbox_pr, dim3(nblk(h.c2g.nslots)), dim3(BLOCK), 0, s, h.d_in_dst, h.d_in_f,
                         h.c2g.nslots, h.d_ghost);
    }
    // GPU gather with the inbox sums; its dangling mass lands in scalars[(k+1)&1]
    TG_TRY(gpu_pagerank_step(p, damping, mode, k, last, rank, s, h.d_ghost, h.d_bdeg));
    double d_gpu = 0.0;
    TG_HIP(hipMemcpyAsync(&ws.h_work[2], ws.scalars + ((k + 1) & 1), sizeof(double), hipMemcpyDeviceToHost, s));
    TG_HIP(hipStreamSynchronize(s));  // GPU messages and dangling mass are on the host
    memcpy(&d_gpu, &ws.h_work[2], sizeof(double));
    ph.gpu_ms += ms_since(tg0);
    ph.bytes += (double)(h.g2c.nslots + h.c2g.nslots) * sizeof(double);
    ph.h2d_bytes += (double)h.c2g.nslots * sizeof(double);
    ph.cpu_edges += (double)(C.m + h.c2g.edges());
    // host gather
    const auto tc2 = clk::now();
    std::fill(ghost.begin(), ghost.end(), 0.0);
    for (int64_t q = 0; q < h.g2c.nslots; ++q) ghost[h.g2c.dst[q]] = h.h_out_f[q];
    const double add = base + (drop ? 0.0 : damping * D / N);
    double d_cpu = 0.0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : d_cpu)
    for (int64_t v = 0; v < C.n; ++v) {
      double sum = ghost[v];
      for (int64_t e = C.ioff[v]; e < C.ioff[v + 1]; ++e) sum += (double)cc[C.icol[e]];
      const double r = add + damping * sum;
      const int64_t od = C.off[v + 1] - C.off[v] + C.bdeg[v];
      if (last) crank[v] = (float)r;
      cn[v] = od > 0 ? (float)(r / (double)od) : 0.0f;
      if (od == 0) d_cpu += r;
    }
    cc.swap(cn);
    ph.cpu_ms += ms_since(tc2);
    D = d_gpu + d_cpu;
    TG_HIP(hipMemcpyAsync(ws.scalars + ((k + 1) & 1), &D, sizeof(double), hipMemcpyHostToDevice, s));
    TG_HIP(hipStreamSynchronize(s));
  }
  // host ranks into the output
  float *hs = reinterpret_cast<float *>(h.h_stage);
  memcpy(hs, crank.data(), (size_t)C.n * sizeof(float));
  TG_HIP(hipMemcpyAsync(h.d_stage, hs, (size_t)C.n * sizeof(float), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_scatter_stage_f32, dim3(nblk(C.n)), dim3(BLOCK), 0, s, h.d_cpu_g_of_l,
                     reinterpret_cast<const float *>(h.d_stage), C.n, rank);
  TG_HIP(hipStreamSynchronize(s));
  add_phase_stats(ph);
  ktimer_emit();
  return TG_OK;
}

}  // namespace tg

// The hybrid split (sections 3-4 and 6.3): building the two partitions and
// the message channels between them.  Partition choice (section 6.3.1): HIGH
// moves the highest-degree vertices to the host until it holds
// cpu_edge_share of the edges, LOW the lowest-degree ones, RAND a seeded
// random subset.
//
// Message reductions are atomic-free: every channel keeps, per slot (one
// distinct remote vertex), the list of its sources (a reverse CSR), and the
// degree-binned gather reduces each slot's list on the GPU, for both
// directions.  Per-source lists of boundary edges name the slot of each
// edge for the sweeps that push from a frontier (the BC backward sweep).
// The supersteps and the exchange are in hybrid_algos.hip.
#include <omp.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "gather.h"
#include "hybrid.h"

using namespace tgk;

namespace tg {

namespace {

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

// The static plan of a device channel: its slot order is a permutation by
// non-increasing source count, and a replay of its virtual blocks (the
// arithmetic of assign_work_rows) covers every source of every slot once.
int check_plan(const Channel &o, const DevChannel &dc, const std::vector<int32_t> &sorder,
               const std::vector<int64_t> &sdeg, const char *name) {
  std::vector<char> seen((size_t)o.nslots, 0);
  for (int64_t i = 0; i < o.nslots; ++i) {
    const int32_t sl = sorder[i];
    if (sl < 0 || sl >= o.nslots || seen[sl]) return set_error(TG_EDEVICE, "hybrid %s: slot order is not a permutation", name);
    seen[sl] = 1;
    if (sdeg[i] != o.roff[sl + 1] - o.roff[sl] || (i > 0 && sdeg[i] > sdeg[i - 1]))
      return set_error(TG_EDEVICE, "hybrid %s: slot order is not by source count", name);
  }
  const Plan &P = dc.h_plan;
  if (P.count != o.nslots || P.pos[0] != 0 || P.pos[NBIN] != o.nslots)
    return set_error(TG_EDEVICE, "hybrid %s: slot plan does not cover the slots", name);
  for (int b = 0; b < NBIN; ++b)
    if (P.pos[b + 1] < P.pos[b] || P.vb[b + 1] < P.vb[b]) return set_error(TG_EDEVICE, "hybrid %s: slot plan not monotone", name);
  const int64_t nh = P.pos[1] - P.pos[0], hc = dc.hub_chunk;
  std::vector<int64_t> hubpref((size_t)nh + 1, 0);
  for (int64_t k = 0; k < nh; ++k) hubpref[k + 1] = hubpref[k] + (sdeg[k] + hc - 1) / hc;
  if (P.vb[1] != hubpref[nh]) return set_error(TG_EDEVICE, "hybrid %s: hub chunks of the slot plan", name);
  std::vector<int64_t> covered((size_t)o.nslots, 0);
  for (int64_t vb = 0; vb < P.vb[NBIN]; ++vb) {
    int b = 0;
    for (int k = 1; k < NBIN; ++k) b += vb >= P.vb[k] ? 1 : 0;
    const int64_t local = vb - P.vb[b];
    if (b == BIN_HUB) {
      const int64_t i = std::upper_bound(hubpref.begin(), hubpref.end(), local) - hubpref.begin() - 1;
      if (i < 0 || i >= nh || local >= hubpref[nh])
        return set_error(TG_EDEVICE, "hybrid %s: hub virtual block %lld", name, (long long)vb);
      const int32_t sl = sorder[P.pos[0] + i];
      const int64_t e0 = o.roff[sl] + (local - hubpref[i]) * hc;
      const int64_t e1 = std::min<int64_t>(e0 + hc, o.roff[sl + 1]);
      if (e0 < o.roff[sl] || e0 >= e1)
        return set_error(TG_EDEVICE, "hybrid %s: hub chunk %lld of slot %d", name, (long long)vb, sl);
      covered[sl] += e1 - e0;
      continue;
    }
    if (b == BIN_ZERO) return set_error(TG_EDEVICE, "hybrid %s: a slot in the empty bin", name);
    for (int t = 0; t < BLOCK; t += lanes_per_vertex(b)) {
      const int64_t qi = P.pos[b] + local * verts_per_vblock(b) + t / lanes_per_vertex(b);
      if (qi >= P.pos[b + 1]) break;
      const int32_t sl = sorder[qi];
      covered[sl] += o.roff[sl + 1] - o.roff[sl];
    }
  }
  for (int64_t sl = 0; sl < o.nslots; ++sl)
    if (covered[sl] != o.roff[sl + 1] - o.roff[sl])
      return set_error(TG_EDEVICE, "hybrid %s: slot plan covers %lld of the %lld sources of slot %lld", name,
                       (long long)covered[sl], (long long)(o.roff[sl + 1] - o.roff[sl]), (long long)sl);
  return TG_OK;
}

int check_hybrid(const tg_partition &p) {
  const HybridState &h = *p.hy;
  const CpuPart &C = h.cpu;
  const int64_t gn = p.gpu.n;
  TG_TRY(check_channel(h.g2c, gn, C.n, p.g->has_w, "GPU-to-host channel"));
  TG_TRY(check_channel(h.c2g, C.n, gn, p.g->has_w, "host-to-GPU channel"));
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

// The per-source boundary lists: every edge names a slot of its channel and
// each slot is named by as many edges as it has sources.
int check_slot_list(const std::vector<int64_t> &off, const std::vector<int32_t> &slot, int64_t nsrc,
                    const Channel &ch, const char *name) {
  if ((int64_t)off.size() != nsrc + 1 || off[0] != 0 || off.back() != (int64_t)slot.size() ||
      (int64_t)slot.size() != ch.edges())
    return set_error(TG_EDEVICE, "hybrid %s: boundary list lengths", name);
  std::vector<int64_t> cnt((size_t)ch.nslots, 0);
  for (int32_t k : slot) {
    if (k < 0 || k >= ch.nslots) return set_error(TG_EDEVICE, "hybrid %s: slot %d out of range", name, k);
    ++cnt[k];
  }
  for (int64_t k = 0; k < ch.nslots; ++k)
    if (cnt[k] != ch.roff[k + 1] - ch.roff[k]) return set_error(TG_EDEVICE, "hybrid %s: slot %lld", name, (long long)k);
  return TG_OK;
}

int check_boundary_lists(const HybridState &h, const std::vector<int32_t> &fb_slot,
                         const std::vector<int64_t> &fb_off, int64_t gn) {
  TG_TRY(check_slot_list(h.hb_off, h.hb_slot, h.cpu.n, h.c2g, "host boundary lists"));
  return check_slot_list(fb_off, fb_slot, gn, h.g2c, "GPU boundary lists");
}

// A channel on the device: reverse CSR, receiver ids, slots ordered by
// decreasing source count (the gather's degree bins) and the static plan
// over them with its hub chunk prefix and partials; checked on the host.
int upload_channel(DevArena &A, const Channel &o, bool weighted, const Tuning &t, DevChannel &dc, const char *name) {
  dc.nslots = o.nslots;
  TG_TRY(up(A, &dc.roff, o.roff.data(), o.roff.size()));
  TG_TRY(up(A, &dc.rsrc, o.rsrc.data(), std::max<size_t>(o.rsrc.size(), 1)));
  if (weighted) TG_TRY(up(A, &dc.rw, o.rw.data(), std::max<size_t>(o.rw.size(), 1)));
  TG_TRY(up(A, &dc.dst, o.dst.data(), std::max<size_t>(o.dst.size(), 1)));
  std::vector<int32_t> sorder((size_t)o.nslots);
  for (int64_t i = 0; i < o.nslots; ++i) sorder[i] = (int32_t)i;
  std::stable_sort(sorder.begin(), sorder.end(), [&](int32_t a, int32_t b) {
    return o.roff[a + 1] - o.roff[a] > o.roff[b + 1] - o.roff[b];
  });
  std::vector<int64_t> sdeg((size_t)o.nslots);
  for (int64_t i = 0; i < o.nslots; ++i) sdeg[i] = o.roff[sorder[i] + 1] - o.roff[sorder[i]];
  TG_TRY(up(A, &dc.order, sorder.data(), std::max<size_t>(sorder.size(), 1)));
  BinBounds bb{};
  int64_t i = 0;
  for (int b = 0; b < NBIN; ++b) {
    while (i < o.nslots && bin_of_degree(sdeg[i], t) < b) ++i;
    bb.bstart[b] = i;
  }
  bb.bstart[NBIN] = o.nslots;
  Plan &P = dc.h_plan;
  memset(&P, 0, sizeof(P));
  P.count = (int32_t)o.nslots;
  for (int b = 0; b <= NBIN; ++b) P.pos[b] = (int32_t)bb.bstart[b];
  const int64_t nh = bb.bstart[1];
  std::vector<int64_t> hubpref((size_t)nh + 1, 0);
  for (int64_t k = 0; k < nh; ++k) hubpref[k + 1] = hubpref[k] + (sdeg[k] + t.hub_chunk - 1) / t.hub_chunk;
  int64_t vb = hubpref[nh];
  P.vb[0] = 0;
  P.vb[1] = vb;
  for (int b = 1; b < NBIN; ++b) {
    if (b != BIN_ZERO) vb += (P.pos[b + 1] - P.pos[b] + verts_per_vblock(b) - 1) / verts_per_vblock(b);
    P.vb[b + 1] = vb;
  }
  dc.hub_chunk = t.hub_chunk;
  TG_TRY(up(A, &dc.hubpref, hubpref.data(), hubpref.size()));
  TG_TRY(up(A, &dc.d_plan, &P, 1));
  TG_TRY(dalloc(A, &dc.partials_f, (size_t)hubpref[nh] + 1));
  TG_TRY(dalloc(A, &dc.partials_i, (size_t)hubpref[nh] + 1));
  return check_plan(o, dc, sorder, sdeg, name);
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
  hy->raw_boundary_edges = (int64_t)gb.dst.size() + (int64_t)cb_dst.size();
  // per-source boundary lists in slot terms: host sources -> host-to-GPU
  // slots, GPU sources -> GPU-to-host slots
  {
    std::vector<int32_t> slot_of((size_t)p->gpu.n, -1);
    for (int64_t k = 0; k < hy->c2g.nslots; ++k) slot_of[hy->c2g.dst[k]] = (int32_t)k;
    hy->hb_off = cb_off;
    hy->hb_slot.resize(cb_dst.size());
    hy->hb_w = std::move(cb_w);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < (int64_t)cb_dst.size(); ++e) hy->hb_slot[e] = slot_of[p->h_l_of_g[cb_dst[e]]];
  }
  std::vector<int32_t> fb_slot(gb.dst.size());
  {
    std::vector<int32_t> slot_of((size_t)C.n, -1);
    for (int64_t k = 0; k < hy->g2c.nslots; ++k) slot_of[hy->g2c.dst[k]] = (int32_t)k;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < (int64_t)gb.dst.size(); ++e) fb_slot[e] = slot_of[c_l_of_g[gb.dst[e]]];
  }
  C.l_of_g = std::move(c_l_of_g);

  TG_TRY(check_hybrid(*p));
  // device side
  GpuPart &g = p->gpu;
  DevArena &A = hy->arena;
  TG_TRY(upload_channel(A, hy->g2c, G.has_w, p->tune, hy->dout, "GPU-to-host channel"));
  TG_TRY(upload_channel(A, hy->c2g, G.has_w, p->tune, hy->din, "host-to-GPU channel"));
  const size_t no = (size_t)std::max<int64_t>(hy->g2c.nslots, 1), nc = (size_t)std::max<int64_t>(C.n, 1);
  TG_TRY(up(A, &hy->d_fb_off, gb.src_off.data(), gb.src_off.size()));
  TG_TRY(up(A, &hy->d_fb_slot, fb_slot.data(), std::max<size_t>(fb_slot.size(), 1)));
  TG_TRY(dalloc(A, &hy->d_osent, no));
  TG_TRY(dalloc(A, &hy->d_oval, no));
  TG_TRY(dalloc(A, &hy->d_ochg, (no + 31) / 32));
  TG_TRY(dalloc(A, &hy->d_hbits, (nc + 31) / 32));
  TG_TRY(dalloc(A, &hy->d_hdist, nc));
  TG_TRY(dalloc(A, &hy->d_hsig, nc));
  std::vector<int32_t> gb_deg((size_t)g.n);
  for (int64_t i = 0; i < g.n; ++i) gb_deg[i] = (int32_t)(gb.src_off[i + 1] - gb.src_off[i]);
  TG_TRY(up(A, &hy->d_bdeg, gb_deg.data(), std::max<size_t>(gb_deg.size(), 1)));
  TG_TRY(dalloc(A, &hy->d_ghost, (size_t)std::max<int64_t>(g.n, 1)));
  TG_TRY(dalloc(A, &hy->d_bdel, (size_t)std::max<int64_t>(g.n, 1)));
  TG_TRY(dalloc(A, &hy->d_gh_lev, no));
  TG_TRY(dalloc(A, &hy->d_gh_sig, no));
  TG_TRY(dalloc(A, &hy->d_gh_del, no));
  TG_TRY(up(A, &hy->d_cpu_g_of_l, C.g_of_l.data(), (size_t)C.n));
  TG_TRY(dalloc(A, &hy->d_stage, (size_t)C.n));
  TG_HIP(hipHostMalloc((void **)&hy->h_stage, (size_t)C.n * sizeof(int32_t), hipHostMallocDefault));
  TG_HIP(hipHostMalloc((void **)&hy->h_scalar, 64, hipHostMallocDefault));
  TG_HIP(hipStreamCreateWithFlags(&hy->cs_d2h, hipStreamNonBlocking));
  TG_HIP(hipStreamCreateWithFlags(&hy->cs_h2d, hipStreamNonBlocking));
  for (int b = 0; b < 2; ++b) {
    TG_HIP(hipEventCreateWithFlags(&hy->ev_ready[b], hipEventDisableTiming));
    for (int k = 0; k < 2; ++k) {
      TG_HIP(hipEventCreate(&hy->ev_d2h[b][k]));
      TG_HIP(hipEventCreate(&hy->ev_h2d[b][k]));
    }
  }
  TG_HIP(hipEventCreateWithFlags(&hy->ev_step, hipEventDisableTiming));
  // the uploads above ran on the null stream; the copy streams do not wait for it
  TG_HIP(hipDeviceSynchronize());
  return check_boundary_lists(*hy, fb_slot, gb.src_off, g.n);
}

HybridState::~HybridState() {
  for (Box *b : {&out, &in})
    for (int k = 0; k < 2; ++k) {
      if (b->d[k]) TG_QUIET(hipFree(b->d[k]));
      if (b->h[k]) TG_QUIET(hipHostFree(b->h[k]));
    }
  if (h_stage) TG_QUIET(hipHostFree(h_stage));
  if (h_scalar) TG_QUIET(hipHostFree(h_scalar));
  if (cs_d2h) TG_QUIET(hipStreamDestroy(cs_d2h));
  if (cs_h2d) TG_QUIET(hipStreamDestroy(cs_h2d));
  for (int b = 0; b < 2; ++b) {
    if (ev_ready[b]) TG_QUIET(hipEventDestroy(ev_ready[b]));
    for (int k = 0; k < 2; ++k) {
      if (ev_d2h[b][k]) TG_QUIET(hipEventDestroy(ev_d2h[b][k]));
      if (ev_h2d[b][k]) TG_QUIET(hipEventDestroy(ev_h2d[b][k]));
    }
  }
  if (ev_step) TG_QUIET(hipEventDestroy(ev_step));
}

int hybrid_boxes(HybridState &h, size_t out_bytes, size_t in_bytes) {
  for (auto [b, want] : {std::pair<Box *, size_t>{&h.out, out_bytes}, {&h.in, in_bytes}}) {
    if (b->cap >= want) continue;
    TG_HIP(hipDeviceSynchronize());  // nothing may still read the old buffers
    for (int k = 0; k < 2; ++k) {
      if (b->d[k]) TG_HIP(hipFree(b->d[k]));
      if (b->h[k]) TG_HIP(hipHostFree(b->h[k]));
      b->d[k] = nullptr;
      b->h[k] = nullptr;
    }
    b->cap = 0;
    const size_t bytes = (want + 255) / 256 * 256;
    for (int k = 0; k < 2; ++k) {
      if (hipMalloc((void **)&b->d[k], bytes) != hipSuccess) return set_error(TG_ENOMEM, "hybrid: message buffers");
      if (hipHostMalloc((void **)&b->h[k], bytes, hipHostMallocDefault) != hipSuccess)
        return set_error(TG_ENOMEM, "hybrid: pinned message buffers");
    }
    b->cap = bytes;
  }
  return TG_OK;
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

}  // namespace tg

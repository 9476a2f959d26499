// The hybrid split (sections 3, 4 and 6): one GPU partition plus one partition
// processed by host threads, exchanging reduced boundary messages over PCIe
// once per superstep.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "tg_internal.h"

namespace tg {

// Edges that leave a partition: per local source (CSR over local ids), the
// global destination ids and weights.
struct BoundaryEdges {
  std::vector<int64_t> src_off;
  std::vector<int32_t> dst;
  std::vector<int32_t> w;
};

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
// vertex, in increasing receiver-local id; per slot, its sender-local sources
// (the outbox of section 4.3.2; the receiver's inbox holds dst).
struct Channel {
  int64_t nslots = 0;
  std::vector<int32_t> dst;   // slot -> receiver-local id (the receiver's inbox)
  std::vector<int64_t> roff;  // slot -> [roff[s], roff[s+1])
  std::vector<int32_t> rsrc;  // sender-local sources
  std::vector<int32_t> rw;    // their edge weights (if weighted)
  int64_t edges() const { return roff.empty() ? 0 : roff.back(); }
};

// A channel's reverse CSR on the device with a static degree-binned plan
// over its slots (slots ordered by decreasing source count), reduced by the
// generic gather: the GPU reduces the GPU-to-host channel from its own
// vertex state (push to the host) and the host-to-GPU channel from the host
// vertex state the host sends (pull, section 4.3.2).
struct DevChannel {
  int64_t nslots = 0;
  int64_t *roff = nullptr;
  int32_t *rsrc = nullptr, *rw = nullptr, *order = nullptr;
  int32_t *dst = nullptr;  // slot -> receiver-local id
  Plan h_plan{};
  Plan *d_plan = nullptr;
  int64_t hub_chunk = 0;  // edges per hub chunk of the plan (fixed at build)
  int64_t *hubpref = nullptr;
  double *partials_f = nullptr;
  int64_t *partials_i = nullptr;
};

// Message buffers of one direction, double-buffered by superstep parity: the
// sender fills buffer (step & 1) while the receiver may still read the other.
struct Box {
  char *d[2] = {nullptr, nullptr};  // device side
  char *h[2] = {nullptr, nullptr};  // pinned host side
  size_t cap = 0;                   // bytes of each buffer
};

struct HybridState {
  CpuPart cpu;
  Channel g2c, c2g;
  int64_t raw_boundary_edges = 0;  // boundary edges before reduction (both directions)
  // host boundary edges per host source: the host-to-GPU slot of each edge
  // and its weight (the host's part of the BC backward sweep)
  std::vector<int64_t> hb_off;
  std::vector<int32_t> hb_slot, hb_w;
  DevArena arena;
  DevChannel dout, din;  // GPU-to-host and host-to-GPU channels on the device
  // GPU boundary edges per GPU source: the GPU-to-host slot of each edge
  int64_t *d_fb_off = nullptr;
  int32_t *d_fb_slot = nullptr;
  // per GPU-to-host slot: what was last sent (BFS/BC: a flag, SSSP: the
  // distance), the value of this superstep and the changed-slot bitmap
  int32_t *d_osent = nullptr;
  int64_t *d_oval = nullptr;
  uint32_t *d_ochg = nullptr;
  // host vertex state the host sends for the host-to-GPU reduction: a
  // membership bitmap (frontier, active set), distances, path counts
  uint32_t *d_hbits = nullptr;
  int32_t *d_hdist = nullptr;
  double *d_hsig = nullptr;
  int32_t *d_bdeg = nullptr;    // GPU vertices' boundary out-degree
  double *d_ghost = nullptr;    // PageRank: inbox sums per GPU vertex
  double *d_bdel = nullptr;     // BC: boundary part of delta per GPU vertex
  int32_t *d_gh_lev = nullptr;  // BC: level, sigma and delta of each
  double *d_gh_sig = nullptr;   //     GPU-to-host slot's host vertex
  float *d_gh_del = nullptr;
  int32_t *d_cpu_g_of_l = nullptr;
  int32_t *d_stage = nullptr;   // host-partition results on their way to the output
  int32_t *h_stage = nullptr;
  double *h_scalar = nullptr;   // pinned: dangling mass on its way to the GPU
  Box out, in;                  // GPU-to-host and host-to-GPU messages
  hipStream_t cs_d2h = nullptr, cs_h2d = nullptr;  // copy streams (default priority)
  hipEvent_t ev_ready[2] = {}, ev_d2h[2][2] = {}, ev_h2d[2][2] = {}, ev_step = nullptr;
  ~HybridState();
};

// Stable counting sort of `ids` by decreasing key[id] (keys >= 0).
void sort_desc_by_key(const std::vector<int64_t> &key, std::vector<int32_t> &ids);
void transpose_csr(int64_t n, const std::vector<int64_t> &off, const std::vector<int32_t> &col,
                   std::vector<int64_t> &ioff, std::vector<int32_t> &icol);
int build_gpu_part(tg_partition *p, const std::vector<int32_t> &verts, BoundaryEdges *boundary);
int build_hybrid(tg_partition *p, uint64_t seed);
void hybrid_free(tg_partition *p);
std::string hybrid_info_json(const tg_partition *p);
// Grows both boxes to at least `bytes` per buffer (no messages in flight).
int hybrid_boxes(HybridState &h, size_t out_bytes, size_t in_bytes);
int hybrid_bfs(tg_partition *p, const int32_t *roots, int32_t nr, int32_t *levels, int32_t *parents,
               hipStream_t s);
int hybrid_sssp(tg_partition *p, const int32_t *roots, int32_t nr, int32_t *dist, hipStream_t s);
int hybrid_pagerank(tg_partition *p, double damping, int32_t iters, int mode, float *rank, hipStream_t s);
// Brandes BC over both partitions; scores (global ids, fp32) are written once
// for all sources.  Returns TG_ERANGE if a path count reaches 2^53.
int hybrid_bc(tg_partition *p, const int32_t *sources, int32_t ns, float *scores, hipStream_t s);

}  // namespace tg

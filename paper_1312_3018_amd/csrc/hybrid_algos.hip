// Supersteps of the hybrid split (section 4.1): in each superstep both
// partitions compute, each reduces the messages bound for every remote vertex
// into one value at the source (section 3.4), the messages cross PCIe and
// each receiver folds its inbox into its vertex state.
//
// Reductions.  The GPU reduces both channels, over their reverse CSRs on
// the device (atomic-free and deterministic, the degree-binned gather): the
// GPU-to-host channel from its own vertex state (the sender reduces,
// section 3.4), the host-to-GPU channel from the state of the host's
// boundary sources, which the host sends (the receiver pulls its remote
// in-neighbours' state, section 4.3.2).  The host threads only expand their
// own frontier over local edges and apply the GPU's messages; the boundary
// edges, nearly all of them hub edges under HIGH, are scanned on the GPU.
//
// Exchange.  The GPU sends one bit per slot (BFS: reached for the first
// time), or (slot, value) lists of the slots whose value improved (SSSP: a
// 4-byte distance; BC: an 8-byte path count, a 4-byte delta), or 4 bytes
// per slot (PageRank).  The host sends its frontier as a bitmap (BFS), its
// active set or frontier with values (SSSP, BC), or one 4-byte contribution
// per vertex (PageRank).  Copies run on two copy streams of their own, one
// per direction, into buffers double-buffered by superstep parity and
// ordered by events (section 4.3.4 (iv)); sending only what changed is the
// compression that section 4.4 points to.  The host's part of a superstep
// is sent before it computes, so the GPU's reduction never waits for the
// host's expansion, and PageRank's host gather runs beside the GPU step.

#include <omp.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "gather.h"
#include "hybrid.h"

using namespace tgk;

namespace tg {
namespace {

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t) { return std::chrono::duration<double, std::milli>(clk::now() - t).count(); }

constexpr int64_t I64_INF = INT64_MAX;
constexpr int32_t OVF_MSG = -1;          // SSSP message: a candidate distance >= INT32_MAX
constexpr size_t LIST_HDR = 16;          // list header: the entry count (uint32)
constexpr int64_t LIST_PREFIX = 16384;   // entries copied with the header

// One entry of an (id, value) list: a slot of the GPU-to-host channel, or a
// host vertex whose state the host sends.
template <typename T>
struct Msg {
  int32_t id;
  T val;
};

template <typename T>
size_t list_bytes(int64_t n) {
  return LIST_HDR + (size_t)std::max<int64_t>(n, 1) * sizeof(Msg<T>);
}
template <typename T>
Msg<T> *entries(char *box) {
  return reinterpret_cast<Msg<T> *>(box + LIST_HDR);
}

// ------------------------------------------------------------- GPU kernels
// Outbox reductions over the GPU-to-host channel (k_gather over its slots).

// BFS: a slot not sent before gets a bit if any of its sources is on
// frontier L.
struct BfsOut {
  using T = int32_t;
  const int32_t *rsrc;
  const int32_t *level;
  int32_t L;
  int32_t *sent;
  uint32_t *bits;
  __device__ static int32_t identity() { return 0; }
  __device__ static int32_t combine(int32_t a, int32_t b) { return a | b; }
  __device__ int32_t vstate(int32_t slot) const { return sent[slot]; }
  __device__ static bool live(int32_t was_sent) { return was_sent == 0; }
  __device__ int32_t term(int32_t, int64_t e) const { return level[rsrc[e]] == L ? 1 : 0; }
  __device__ void finish(int32_t slot, int32_t r) const {
    if (!r) return;
    sent[slot] = 1;
    atomicOr(bits + (slot >> 5), 1u << (slot & 31));
  }
};

// SSSP: least dist(src) + w over the sources that relaxed this superstep;
// sent when below the last value sent (or, once, as an overflow mark).
struct SsspOut {
  using T = int64_t;
  const int32_t *rsrc;
  const int32_t *rw;
  const int32_t *dist;
  const uint32_t *cur;
  int32_t *sent;
  int64_t *val;
  uint32_t *chg;
  __device__ static int64_t identity() { return I64_INF; }
  __device__ static int64_t combine(int64_t a, int64_t b) { return a < b ? a : b; }
  __device__ int32_t vstate(int32_t) const { return 0; }
  __device__ static bool live(int32_t) { return true; }
  __device__ int64_t term(int32_t, int64_t e) const {
    const int32_t u = rsrc[e];
    return ((cur[u >> 5] >> (u & 31)) & 1u) ? (int64_t)dist[u] + (int64_t)rw[e] : I64_INF;
  }
  __device__ void finish(int32_t slot, int64_t r) const {
    if (r == I64_INF) return;
    const int32_t last = sent[slot];
    int32_t m;
    if (r >= (int64_t)TG_INF) {
      if (last != TG_INF) return;  // a finite distance was sent: the mark changes nothing
      m = OVF_MSG;
    } else {
      if (r >= (int64_t)last) return;
      m = (int32_t)r;
      sent[slot] = m;
    }
    val[slot] = m;
    atomicOr(chg + (slot >> 5), 1u << (slot & 31));
  }
};

// PageRank: the sum of the contributions c(src) bound for one host vertex.
struct PrOut : SumF64 {
  const int32_t *rsrc;
  const float *c;
  float *msg;
  __device__ int32_t vstate(int32_t) const { return 0; }
  __device__ double term(int32_t, int64_t e) const { return (double)c[rsrc[e]]; }
  __device__ void finish(int32_t slot, double r) const { msg[slot] = (float)r; }
};

// BC forward: sum of sigma(src) over the sources on frontier L, sent the
// first time a slot has any (the receiver is then at level <= L + 1; a
// later message could only reach a vertex already placed).
struct SigmaOut : SumF64 {
  const int32_t *rsrc;
  const int32_t *level;
  const double *sigma;
  int32_t L;
  int32_t *sent;
  int64_t *val;
  uint32_t *chg;
  __device__ int32_t vstate(int32_t slot) const { return sent[slot]; }
  __device__ static bool live(int32_t was_sent) { return was_sent == 0; }
  __device__ double term(int32_t, int64_t e) const {
    const int32_t u = rsrc[e];
    return level[u] == L ? sigma[u] : 0.0;
  }
  __device__ void finish(int32_t slot, double r) const {
    if (r == 0.0) return;
    sent[slot] = 1;
    val[slot] = __double_as_longlong(r);
    atomicOr(chg + (slot >> 5), 1u << (slot & 31));
  }
};

// BC forward on the GPU: a new vertex adds the pull over its local in-edges
// to what its inbox gave it (the host in-neighbours' sigma).
struct SigmaPullHy : SumF64 {
  const int32_t *col;
  const int32_t *level;
  double *sigma;
  uint32_t *flags;
  int32_t parent_level;
  __device__ double vstate(int32_t) const { return 0.0; }
  __device__ double term(double, int64_t e) const {
    const int32_t u = col[e];
    return level[u] == parent_level ? sigma[u] : 0.0;
  }
  __device__ void finish(int32_t v, double s) const {
    const double t = sigma[v] + s;
    sigma[v] = t;
    if (t >= 9007199254740992.0) flags[2] = 1u;  // 2^53: fp64 counts stop being exact
  }
};

// Brandes' term sigma(v)/sigma(w) * (1 + delta(w)), ratio in fp32 as on the
// GPU-only path.
__device__ __forceinline__ double brandes_term(double sv, double sw, float dw) {
  const float ratio = (float)(sv / sw);
  return (double)(ratio * (1.0f + dw));
}

// BC backward on the GPU, boundary part: children on the host (ghost level,
// sigma and delta per GPU-to-host slot).  A vertex without local out-edges
// finishes here; the others keep the sum for DeltaAccumHy.
struct DeltaBoundary : SumF64 {
  const int32_t *fb_slot;
  const int32_t *gh_lev;
  const double *gh_sig;
  const float *gh_del;
  const double *sigma;
  const int64_t *out_off;
  float *delta;
  double *score;
  double *bdel;
  int32_t child_level;
  __device__ double vstate(int32_t v) const { return sigma[v]; }
  __device__ double term(double sv, int64_t e) const {
    const int32_t k = fb_slot[e];
    return gh_lev[k] == child_level ? brandes_term(sv, gh_sig[k], gh_del[k]) : 0.0;
  }
  __device__ void finish(int32_t v, double r) const {
    if (out_off[v + 1] == out_off[v]) {
      const float d = (float)r;
      delta[v] = d;
      score[v] += (double)d;
    } else {
      bdel[v] = r;
    }
  }
};

// BC backward on the GPU, local part plus the boundary sum.
struct DeltaAccumHy : SumF64 {
  const int32_t *col;
  const int32_t *level;
  const double *sigma;
  const double *bdel;
  float *delta;
  double *score;
  int32_t child_level;
  __device__ double vstate(int32_t v) const { return sigma[v]; }
  __device__ double term(double sv, int64_t e) const {
    const int32_t w = col[e];
    return level[w] == child_level ? brandes_term(sv, sigma[w], delta[w]) : 0.0;
  }
  __device__ void finish(int32_t v, double s) const {
    const float d = (float)(s + bdel[v]);
    delta[v] = d;
    score[v] += (double)d;
  }
};

// Changed slots of the GPU outbox, with their values.
struct SelChangedI32 {
  const uint32_t *chg;
  const int64_t *val;
  __device__ bool take(int64_t k, int32_t &v) const {
    if (!((chg[k >> 5] >> (k & 31)) & 1u)) return false;
    v = (int32_t)val[k];
    return true;
  }
};
struct SelChangedF64 {
  const uint32_t *chg;
  const int64_t *val;
  __device__ bool take(int64_t k, double &v) const {
    if (!((chg[k >> 5] >> (k & 31)) & 1u)) return false;
    v = __longlong_as_double(val[k]);
    return true;
  }
};
// BC backward: delta of the GPU's host-to-GPU receivers at level lv.
struct SelLevelDelta {
  const int32_t *dst;
  const int32_t *level;
  const float *delta;
  int32_t lv;
  __device__ bool take(int64_t k, float &v) const {
    const int32_t x = dst[k];
    if (level[x] != lv) return false;
    v = delta[x];
    return true;
  }
};

// Compacts the slots k < n that `sel` takes into the list box: one atomic
// per wave on the header's count, entries in slot order within a wave.
template <typename T, class Sel>
__global__ __launch_bounds__(BLOCK) void k_select(Sel sel, int64_t n, char *box) {
  uint32_t *cnt = reinterpret_cast<uint32_t *>(box);
  Msg<T> *ent = reinterpret_cast<Msg<T> *>(box + LIST_HDR);
  const int lane = threadIdx.x & 63;
  for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < n; base += (int64_t)gridDim.x * BLOCK) {
    const int64_t k = base + threadIdx.x;
    T v{};
    const bool take = k < n && sel.take(k, v);
    const unsigned long long m = __ballot(take);
    if (m == 0ull) continue;  // the same for the whole wave
    const int first = __builtin_ctzll(m);
    uint32_t pos = 0;
    if (lane == first) pos = atomicAdd(cnt, (uint32_t)__popcll(m));
    pos = __shfl(pos, first, 64);
    if (take) {
      const uint32_t r = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      ent[pos + r] = Msg<T>{(int32_t)k, v};
    }
  }
}

// Host-to-GPU reductions over the device copy of that channel, from the
// host vertex state the host sent (its frontier, active set, distances,
// contributions, path counts): the GPU pulls its remote in-neighbours'
// state (section 4.3.2) and folds the result straight into its own.

// BFS: an unvisited GPU vertex is reached, at level `lv`, if a host
// in-neighbour is on the host frontier (skipped once visited: the bottom-up
// test over remote in-edges).
struct BfsIn {
  using T = int32_t;
  const int32_t *rsrc;
  const uint32_t *hfront;
  const int32_t *dst;
  uint32_t *visited;
  int32_t *level;
  int32_t lv;
  __device__ static int32_t identity() { return 0; }
  __device__ static int32_t combine(int32_t a, int32_t b) { return a | b; }
  __device__ int32_t vstate(int32_t slot) const {
    const int32_t v = dst[slot];
    return (int32_t)((visited[v >> 5] >> (v & 31)) & 1u);
  }
  __device__ static bool live(int32_t was_visited) { return was_visited == 0; }
  __device__ int32_t term(int32_t, int64_t e) const {
    const int32_t u = rsrc[e];
    return (int32_t)((hfront[u >> 5] >> (u & 31)) & 1u);
  }
  __device__ void finish(int32_t slot, int32_t r) const {
    if (!r) return;
    const int32_t v = dst[slot];
    atomicOr(visited + (v >> 5), 1u << (v & 31));
    level[v] = lv;
  }
};

// SSSP: least hdist(u) + w over the host in-neighbours active this
// superstep; a GPU vertex that improves joins the active set.  Slots are
// distinct vertices, so no two finishers write one distance.
struct SsspIn {
  using T = int64_t;
  const int32_t *rsrc;
  const int32_t *rw;
  const int32_t *hdist;
  const uint32_t *hact;
  const int32_t *dst;
  int32_t *dist;
  uint32_t *active, *ovf, *flags;
  __device__ static int64_t identity() { return I64_INF; }
  __device__ static int64_t combine(int64_t a, int64_t b) { return a < b ? a : b; }
  __device__ int32_t vstate(int32_t) const { return 0; }
  __device__ static bool live(int32_t) { return true; }
  __device__ int64_t term(int32_t, int64_t e) const {
    const int32_t u = rsrc[e];
    return ((hact[u >> 5] >> (u & 31)) & 1u) ? (int64_t)hdist[u] + (int64_t)rw[e] : I64_INF;
  }
  __device__ void finish(int32_t slot, int64_t r) const {
    if (r == I64_INF) return;
    const int32_t v = dst[slot];
    if (r >= (int64_t)TG_INF) {
      if (dist[v] == TG_INF) {
        atomicOr(ovf + (v >> 5), 1u << (v & 31));
        flags[0] = 1u;
      }
    } else if (r < (int64_t)dist[v]) {
      dist[v] = (int32_t)r;
      atomicOr(active + (v >> 5), 1u << (v & 31));
    }
  }
};

// PageRank: ghost(v) = sum of the host in-neighbours' contributions.
struct PrIn : SumF64 {
  const int32_t *rsrc;
  const float *hc;
  const int32_t *dst;
  double *ghost;
  __device__ int32_t vstate(int32_t) const { return 0; }
  __device__ double term(int32_t, int64_t e) const { return (double)hc[rsrc[e]]; }
  __device__ void finish(int32_t slot, double r) const { ghost[dst[slot]] = r; }
};

// BC forward: a GPU vertex not yet placed (level unset) takes the sum of
// sigma over its host in-neighbours on frontier L and is reached at L + 1.
struct SigmaIn : SumF64 {
  const int32_t *rsrc;
  const uint32_t *hfront;
  const double *hsig;
  const int32_t *dst;
  const int32_t *level;
  double *sigma;
  uint32_t *visited;
  __device__ int32_t vstate(int32_t slot) const { return level[dst[slot]]; }
  __device__ static bool live(int32_t lv) { return lv == TG_INF; }
  __device__ double term(int32_t, int64_t e) const {
    const int32_t u = rsrc[e];
    return ((hfront[u >> 5] >> (u & 31)) & 1u) ? hsig[u] : 0.0;
  }
  __device__ void finish(int32_t slot, double r) const {
    if (r == 0.0) return;
    const int32_t v = dst[slot];
    if (level[v] != TG_INF) return;
    sigma[v] = r;
    atomicOr(visited + (v >> 5), 1u << (v & 31));
  }
};

// The host's (vertex, value) list into the dense host-state arrays and the
// membership bitmap (cleared before; ids are distinct).
template <typename T>
__global__ void k_host_state(const Msg<T> *__restrict__ ent, int64_t n, T *val, uint32_t *bits) {
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k >= n) return;
  const Msg<T> m = ent[k];
  val[m.id] = m.val;
  atomicOr(bits + (m.id >> 5), 1u << (m.id & 31));
}

// BC backward: deltas of host vertices (by GPU-to-host slot).
__global__ void k_inbox_delta(const Msg<float> *__restrict__ ent, int64_t n, float *gh_del) {
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k < n) gh_del[ent[k].id] = ent[k].val;
}

// BC: level and sigma of the GPU's host-to-GPU receivers, for the host.
__global__ void k_ghost_out(const int32_t *__restrict__ dst, int64_t n, const int32_t *__restrict__ level,
                            const double *__restrict__ sigma, double *sig_out, int32_t *lev_out) {
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k >= n) return;
  const int32_t x = dst[k];
  sig_out[k] = sigma[x];
  lev_out[k] = level[x];
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

__global__ void k_set_f64h(double *p, int64_t i, double v) {
  if (threadIdx.x == 0) p[i] = v;
}

inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>((n + BLOCK - 1) / BLOCK, 1); }
inline unsigned select_grid(int64_t n) { return (unsigned)std::min<int64_t>(nblk(n), 8192); }

// Reduces a device channel's slots with `op`.  The slot plan, its hub chunk
// prefix and the partials were sized at partition time with dc.hub_chunk; a
// later retune does not change the chunking they were built for.
template <class Op>
int launch_gather(const DevChannel &dc, hipStream_t s, Op op, typename Op::T *partials) {
  if (dc.nslots == 0) return TG_OK;
  hipLaunchKernelGGL(k_gather<Op>, dim3(launch_grid(dc.h_plan.vb[NBIN])), dim3(BLOCK), 0, s, dc.d_plan, dc.order,
                     dc.hubpref, dc.roff, dc.hub_chunk, partials, op);
  if (dc.h_plan.pos[1] > dc.h_plan.pos[0])
    hipLaunchKernelGGL(k_gather_hubs<Op>, dim3(64), dim3(BLOCK), 0, s, dc.d_plan, dc.order, dc.hubpref, partials, op);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

template <typename T, class Sel>
int launch_select(Sel sel, int64_t n, char *box, hipStream_t s) {
  TG_HIP(hipMemsetAsync(box, 0, sizeof(uint32_t), s));
  if (n > 0) hipLaunchKernelGGL((k_select<T, Sel>), dim3(select_grid(n)), dim3(BLOCK), 0, s, sel, n, box);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int clear_words(uint32_t *w, int64_t n, hipStream_t s) {
  if (n > 0) TG_HIP(hipMemsetAsync(w, 0, (size_t)n * sizeof(uint32_t), s));
  return TG_OK;
}

// ---------------------------------------------------------------- exchange
// Every superstep waits for the GPU stream before the next one starts (the
// frontier plan is read back), so a buffer of parity b is free again when
// superstep b + 2 fills it.

// GPU -> host: once the GPU stream has produced box b, copy `bytes` of it.
int post_d2h(HybridState &h, int b, size_t bytes, hipStream_t s) {
  TG_HIP(hipEventRecord(h.ev_ready[b], s));
  TG_HIP(hipStreamWaitEvent(h.cs_d2h, h.ev_ready[b], 0));
  TG_HIP(hipEventRecord(h.ev_d2h[b][0], h.cs_d2h));
  if (bytes) TG_HIP(hipMemcpyAsync(h.out.h[b], h.out.d[b], bytes, hipMemcpyDeviceToHost, h.cs_d2h));
  TG_HIP(hipEventRecord(h.ev_d2h[b][1], h.cs_d2h));
  return TG_OK;
}

// Waits for it; adds the copy's time.
int wait_d2h(HybridState &h, int b, double *ms) {
  TG_HIP(hipEventSynchronize(h.ev_d2h[b][1]));
  float t = 0.0f;
  TG_QUIET(hipEventElapsedTime(&t, h.ev_d2h[b][0], h.ev_d2h[b][1]));
  *ms += t;
  return TG_OK;
}

// A list from the GPU in box b: the header and the first LIST_PREFIX entries
// came with the first copy, the rest (if any) is fetched now.  Returns the
// entry count; `bytes` gets what crossed.
template <typename T>
int fetch_list(HybridState &h, int b, int64_t *count, double *bytes, double *ms) {
  TG_TRY(wait_d2h(h, b, ms));
  const int64_t n = *reinterpret_cast<const uint32_t *>(h.out.h[b]);
  *bytes += (double)(LIST_HDR + std::min<int64_t>(n, LIST_PREFIX) * sizeof(Msg<T>));
  if (n > LIST_PREFIX) {
    const auto t0 = clk::now();
    const size_t off = LIST_HDR + (size_t)LIST_PREFIX * sizeof(Msg<T>);
    const size_t rest = (size_t)(n - LIST_PREFIX) * sizeof(Msg<T>);
    TG_HIP(hipMemcpyAsync(h.out.h[b] + off, h.out.d[b] + off, rest, hipMemcpyDeviceToHost, h.cs_d2h));
    TG_HIP(hipStreamSynchronize(h.cs_d2h));
    *bytes += (double)rest;
    *ms += ms_since(t0);
  }
  *count = n;
  return TG_OK;
}

template <typename T>
size_t list_prefix_bytes(int64_t nslots) {
  return LIST_HDR + (size_t)std::min<int64_t>(nslots, LIST_PREFIX) * sizeof(Msg<T>);
}

// host -> GPU: copy `bytes` from offset `off` of host box b to the same
// offset of the device box; the GPU stream waits for it.
int post_h2d(HybridState &h, int b, size_t off, size_t bytes, hipStream_t s) {
  TG_HIP(hipEventRecord(h.ev_h2d[b][0], h.cs_h2d));
  if (bytes) TG_HIP(hipMemcpyAsync(h.in.d[b] + off, h.in.h[b] + off, bytes, hipMemcpyHostToDevice, h.cs_h2d));
  TG_HIP(hipEventRecord(h.ev_h2d[b][1], h.cs_h2d));
  TG_HIP(hipStreamWaitEvent(s, h.ev_h2d[b][1], 0));
  return TG_OK;
}

// Time of the last host-to-GPU copy of parity b (complete once the GPU
// stream has passed it).
double h2d_ms(HybridState &h, int b) {
  float t = 0.0f;
  TG_QUIET(hipEventElapsedTime(&t, h.ev_h2d[b][0], h.ev_h2d[b][1]));
  return t;
}

// ------------------------------------------------------------- host side
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

// Per-call accounting.  cpu_edges: the local out-edges the host threads
// processed; exchange_ms: time of the copies in both directions (copy
// stream events); exchange_bytes: what they moved, of which h2d_bytes went
// to the GPU.
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

// Local out-edges of a host frontier: the edges the host threads process
// (its boundary edges are reduced on the GPU).
double frontier_edges(const CpuPart &C, const std::vector<int32_t> &front) {
  double s = 0;
  for (int32_t v : front) s += (double)(C.off[v + 1] - C.off[v]);
  return s;
}

double elapsed(hipEvent_t a, hipEvent_t b) {
  float t = 0.0f;
  TG_QUIET(hipEventElapsedTime(&t, a, b));
  return t;
}

struct Events {
  hipEvent_t e[4] = {};
  int init() {
    for (auto &x : e) TG_HIP(hipEventCreate(&x));
    return TG_OK;
  }
  ~Events() {
    for (auto x : e)
      if (x) TG_QUIET(hipEventDestroy(x));
  }
};

// Host results (levels, distances) into the output row.
int stage_host_i32(HybridState &h, const std::vector<int32_t> &vals, int32_t *out, hipStream_t s) {
  const int64_t n = h.cpu.n;
  memcpy(h.h_stage, vals.data(), (size_t)n * sizeof(int32_t));
  TG_HIP(hipMemcpyAsync(h.d_stage, h.h_stage, (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_scatter_stage_i32, dim3(nblk(n)), dim3(BLOCK), 0, s, h.d_cpu_g_of_l, h.d_stage, n, out);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

int stage_host_f32(HybridState &h, const std::vector<float> &vals, float *out, hipStream_t s) {
  const int64_t n = h.cpu.n;
  float *hs = reinterpret_cast<float *>(h.h_stage);
  memcpy(hs, vals.data(), (size_t)n * sizeof(float));
  TG_HIP(hipMemcpyAsync(h.d_stage, hs, (size_t)n * sizeof(float), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_scatter_stage_f32, dim3(nblk(n)), dim3(BLOCK), 0, s, h.d_cpu_g_of_l,
                     reinterpret_cast<const float *>(h.d_stage), n, out);
  TG_HIP(hipGetLastError());
  return TG_OK;
}

}  // namespace

// ------------------------------------------------------------------- BFS
// The GPU side runs the device-resident superstep of the GPU-only path
// (top-down or bottom-up over local edges, Beamer's switch on the device);
// the host reads the frontier size back every superstep.  GPU to host: a
// bitmap over the GPU-to-host slots, bit k set when slot k's host vertex is
// reached for the first time through the channel (each slot at most once
// per search: a receiver's level is final when first reached).  Host to
// GPU: the host frontier as a bitmap over host vertices, sent at the start
// of the superstep; the GPU reduces the host-to-GPU channel itself.
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
  const int64_t no = h.g2c.nslots;
  const int64_t nwo = (no + 31) / 32, nwc = (C.n + 31) / 32;
  TG_TRY(hybrid_boxes(h, (size_t)nwo * 4, (size_t)nwc * 4));
  std::vector<uint8_t> cvis((size_t)C.n);
  std::vector<int32_t> clev((size_t)C.n);
  std::vector<int32_t> cfront, cnext;
  std::vector<std::vector<int32_t>> tl((size_t)omp_get_max_threads());
  Phase ph;
  Events ev;
  TG_TRY(ev.init());
  for (int32_t r = 0; r < nr; ++r) {
    const int32_t root = roots[r];
    const int32_t gl = p->h_l_of_g[root];
    uint32_t *visited = ws.bits_a;
    TG_HIP(hipMemsetAsync(visited, 0, ws.nwords * sizeof(uint32_t), s));
    TG_HIP(hipMemsetAsync(ws.bits_b, 0, ws.nwords * sizeof(uint32_t), s));
    TG_TRY(fill_i32(ws.state, g.n, TG_INF, s));
    if (no) TG_TRY(fill_i32(h.d_osent, no, 0, s));
    std::fill(cvis.begin(), cvis.end(), 0);
    std::fill(clev.begin(), clev.end(), TG_INF);
    cfront.clear();
    if (gl < 0) {
      const int32_t cl = C.l_of_g[root];
      if (cl < 0) return set_error(TG_EDEVICE, "hybrid bfs: root %d is on neither side", root);
      cvis[cl] = 1;
      clev[cl] = 0;
      cfront.push_back(cl);
    }
    TG_TRY(bfs_dev_start(g, ws, gl, s));  // gl < 0: no GPU root
    TG_TRY(frontier_compact_bfs_dev(g, ws, t, s));
    TG_HIP(hipMemcpyAsync(ws.h_plan, ws.plan, sizeof(Plan), hipMemcpyDeviceToHost, s));
    TG_HIP(hipStreamSynchronize(s));
    for (int32_t L = 0;; ++L) {
      const bool gpu_front = ws.h_plan->count > 0, host_front = !cfront.empty();
      if (!gpu_front && !host_front) break;
      if (L > V) return set_error(TG_EDEVICE, "hybrid bfs: more supersteps than vertices");
      ++ph.supersteps;
      const int b = L & 1;
      TG_HIP(hipEventRecord(ev.e[0], s));
      // GPU: direction and plan, the expansion, the GPU-to-host reduction
      TG_TRY(frontier_plan_bfs_dev(g, ws, t, s));
      if (gpu_front) {
        TG_TRY(clear_words(reinterpret_cast<uint32_t *>(h.out.d[b]), nwo, s));
        TG_TRY(bfs_dev_step(g, ws, t, s, true));
        TG_TRY(launch_gather(h.dout, s,
                             BfsOut{h.dout.rsrc, ws.state, L, h.d_osent, reinterpret_cast<uint32_t *>(h.out.d[b])},
                             reinterpret_cast<int32_t *>(h.dout.partials_i)));
        TG_TRY(post_d2h(h, b, (size_t)nwo * 4, s));
      }
      // the host frontier to the GPU, which reduces the host-to-GPU channel
      if (host_front) {
        const auto tc = clk::now();
        uint32_t *hb = reinterpret_cast<uint32_t *>(h.in.h[b]);
        memset(hb, 0, (size_t)nwc * 4);
        for (int32_t v : cfront) hb[v >> 5] |= 1u << (v & 31);
        ph.cpu_ms += ms_since(tc);
        TG_TRY(post_h2d(h, b, 0, (size_t)nwc * 4, s));
        TG_TRY(launch_gather(h.din, s,
                             BfsIn{h.din.rsrc, reinterpret_cast<const uint32_t *>(h.in.d[b]), h.din.dst, visited,
                                   ws.state, L + 1},
                             reinterpret_cast<int32_t *>(h.din.partials_i)));
        ph.bytes += (double)nwc * 4;
        ph.h2d_bytes += (double)nwc * 4;
      }
      TG_TRY(bfs_dev_resume(ws, L, s));
      TG_TRY(frontier_compact_bfs_dev(g, ws, t, s));
      TG_HIP(hipEventRecord(ev.e[1], s));
      TG_HIP(hipMemcpyAsync(ws.h_plan, ws.plan, sizeof(Plan), hipMemcpyDeviceToHost, s));
      // host: expand its frontier over its local edges while the GPU runs
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
      }
      concat(tl, cnext);
      ph.cpu_ms += ms_since(tc);
      ph.cpu_edges += frontier_edges(C, cfront);
      TG_HIP(hipStreamSynchronize(s));  // the GPU's next frontier size is on the host
      ph.gpu_ms += elapsed(ev.e[0], ev.e[1]);
      if (host_front) ph.exchange_ms += h2d_ms(h, b);
      // the GPU's bits: its frontier's first reach of host vertices
      if (gpu_front) {
        TG_TRY(wait_d2h(h, b, &ph.exchange_ms));
        ph.bytes += (double)nwo * 4;
        const auto tc2 = clk::now();
        const uint32_t *ob = reinterpret_cast<const uint32_t *>(h.out.h[b]);
        for (int64_t w = 0; w < nwo; ++w)
          for (uint32_t bits = ob[w]; bits; bits &= bits - 1u) {
            const int32_t x = h.g2c.dst[w * 32 + __builtin_ctz(bits)];
            if (!cvis[x]) {
              cvis[x] = 1;
              clev[x] = L + 1;
              cnext.push_back(x);
            }
          }
        ph.cpu_ms += ms_since(tc2);
      }
      cfront.swap(cnext);
    }
    TG_TRY(collect_levels(g, ws.bits_a, ws.state, levels + (int64_t)r * V, s));
    TG_TRY(stage_host_i32(h, clev, levels + (int64_t)r * V, s));
    TG_HIP(hipStreamSynchronize(s));
  }
  stats_add("roots", nr);
  add_phase_stats(ph);
  ktimer_emit();
  return TG_OK;
}

// ------------------------------------------------------------------ SSSP
// GPU to host: (slot, distance) lists of the slots whose candidate improved
// on the last value sent.  Host to GPU: (vertex, distance) of the host's
// active set, sent at the start of the superstep; the GPU reduces the
// host-to-GPU channel over it.
int hybrid_sssp(tg_partition *p, const int32_t *roots, int32_t nr, int32_t *dist_out, hipStream_t s) {
  HybridState &h = *p->hy;
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  CpuPart &C = h.cpu;
  const Tuning &t = p->tune;
  TG_TRY(ws.ensure(g, 0));
  const int64_t V = p->g->n;
  const int64_t no = h.g2c.nslots;
  const int64_t nwo = (no + 31) / 32, nwc = (C.n + 31) / 32;
  TG_TRY(hybrid_boxes(h, list_bytes<int32_t>(no), list_bytes<int32_t>(C.n)));
  std::vector<int32_t> cdist((size_t)C.n);
  std::vector<uint8_t> cin_next((size_t)C.n), covf((size_t)C.n);
  std::vector<int32_t> cfront, cnext;
  std::vector<std::vector<int32_t>> tl((size_t)omp_get_max_threads());
  Phase ph;
  Events ev;
  TG_TRY(ev.init());
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
    if (no) TG_TRY(fill_i32(h.d_osent, no, TG_INF, s));
    TG_TRY(clear_words(h.d_ochg, nwo, s));
    std::fill(cdist.begin(), cdist.end(), TG_INF);
    std::fill(cin_next.begin(), cin_next.end(), 0);
    std::fill(covf.begin(), covf.end(), 0);
    cfront.clear();
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
      const bool gpu_front = ws.h_plan->count > 0, host_front = !cfront.empty();
      if (!gpu_front && !host_front) break;
      if (step > V) return set_error(TG_EDEVICE, "hybrid sssp: no convergence");
      ++ph.supersteps;
      const int b = (int)(step & 1);
      TG_HIP(hipEventRecord(ev.e[0], s));
      if (gpu_front) {
        TG_TRY(sssp_relax_launch(g, ws, ws.queue, ws.h_plan->vb[NBIN], t, s));
        TG_TRY(launch_gather(h.dout, s, SsspOut{h.dout.rsrc, h.dout.rw, dist, cur, h.d_osent, h.d_oval, h.d_ochg},
                             h.dout.partials_i));
        TG_TRY(launch_select<int32_t>(SelChangedI32{h.d_ochg, h.d_oval}, no, h.out.d[b], s));
        TG_TRY(clear_words(h.d_ochg, nwo, s));
        TG_TRY(post_d2h(h, b, list_prefix_bytes<int32_t>(no), s));
      }
      // the host's active set with its distances to the GPU, which reduces
      // the host-to-GPU channel over it
      if (host_front) {
        Msg<int32_t> *ie = entries<int32_t>(h.in.h[b]);
        const int64_t n_in = (int64_t)cfront.size();
        for (int64_t i = 0; i < n_in; ++i) ie[i] = Msg<int32_t>{cfront[i], cdist[cfront[i]]};
        const size_t bytes = (size_t)n_in * sizeof(Msg<int32_t>);
        TG_TRY(post_h2d(h, b, LIST_HDR, bytes, s));
        TG_TRY(clear_words(h.d_hbits, nwc, s));
        hipLaunchKernelGGL(k_host_state<int32_t>, dim3(nblk(n_in)), dim3(BLOCK), 0, s, entries<int32_t>(h.in.d[b]),
                           n_in, h.d_hdist, h.d_hbits);
        TG_HIP(hipGetLastError());
        TG_TRY(launch_gather(h.din, s,
                             SsspIn{h.din.rsrc, h.din.rw, h.d_hdist, h.d_hbits, h.din.dst, dist, active, ovf,
                                    ws.counters},
                             h.din.partials_i));
        ph.bytes += (double)bytes;
        ph.h2d_bytes += (double)bytes;
      }
      TG_HIP(hipEventRecord(ev.e[1], s));
      TG_TRY(frontier_compact(g, ws, 2, active, cur, ws.queue, nullptr, 0, s));
      // host: relax its frontier over its local edges while the GPU runs
      const auto tc = clk::now();
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
      }
      concat(tl, cnext);
      ph.cpu_ms += ms_since(tc);
      ph.cpu_edges += frontier_edges(C, cfront);
      TG_TRY(frontier_plan(g, ws, ws.queue, t, s, true));
      ph.gpu_ms += elapsed(ev.e[0], ev.e[1]);
      if (host_front) ph.exchange_ms += h2d_ms(h, b);
      if (gpu_front) {
        int64_t n_out = 0;
        TG_TRY(fetch_list<int32_t>(h, b, &n_out, &ph.bytes, &ph.exchange_ms));
        const auto tc2 = clk::now();
        const Msg<int32_t> *oe = entries<int32_t>(h.out.h[b]);
        for (int64_t i = 0; i < n_out; ++i) {
          const int32_t x = h.g2c.dst[oe[i].id];
          const int32_t m = oe[i].val;
          if (m == OVF_MSG) {
            if (cdist[x] == TG_INF) covf[x] = 1;
            continue;
          }
          if (m < cdist[x]) {
            cdist[x] = m;
            if (!cin_next[x]) {
              cin_next[x] = 1;
              cnext.push_back(x);
            }
          }
        }
        ph.cpu_ms += ms_since(tc2);
      }
      for (int32_t x : cnext) cin_next[x] = 0;
      cfront.swap(cnext);
    }
    bool cpu_overflow = false;
    for (int64_t i = 0; i < C.n; ++i)
      if (covf[i] && cdist[i] == TG_INF) cpu_overflow = true;
    TG_TRY(sssp_overflow_check(g, ws, s));
    if (ws.h_flags[1] || cpu_overflow)
      return set_error(TG_ERANGE, "sssp: a shortest-path distance does not fit below INT32_MAX");
    TG_TRY(collect_i32(g, dist, dist_out + (int64_t)r * V, s));
    TG_TRY(stage_host_i32(h, cdist, dist_out + (int64_t)r * V, s));
    TG_HIP(hipStreamSynchronize(s));
  }
  stats_add("roots", nr);
  add_phase_stats(ph);
  ktimer_emit();
  return TG_OK;
}

// -------------------------------------------------------------- PageRank
// Iteration k: the GPU reduces the GPU-to-host channel from its
// contributions and sends the sums; the host sends its contributions (one
// fp32 per host vertex, kept in the pinned box: the gather of iteration k
// writes those of k+1 into the other buffer) and the GPU reduces the
// host-to-GPU channel over them before its step.  The host's gather needs
// only the GPU's sums, so it runs beside the GPU's step.  The dangling mass
// of both sides is combined before the next iteration.
int hybrid_pagerank(tg_partition *p, double damping, int32_t iters, int mode, float *rank, hipStream_t s) {
  HybridState &h = *p->hy;
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  CpuPart &C = h.cpu;
  const int64_t no = h.g2c.nslots;
  const double N = (double)p->g->n;
  const double base = (1.0 - damping) / N;
  const bool drop = mode == TG_PR_DANGLING_DROP;
  double D = (double)(g.n_dangling + C.n_dangling) / N;
  TG_TRY(hybrid_boxes(h, (size_t)no * sizeof(float), (size_t)C.n * sizeof(float)));
  TG_TRY(gpu_pagerank_setup(p, damping, mode, s, h.d_bdeg, D));
  TG_TRY(fill_f64(h.d_ghost, g.n, 0.0, s));
  std::vector<float> crank((size_t)C.n);
  std::vector<double> ghost((size_t)C.n, 0.0);
  float *cc0 = reinterpret_cast<float *>(h.in.h[0]);
  for (int64_t i = 0; i < C.n; ++i) {
    const int64_t od = C.off[i + 1] - C.off[i] + C.bdeg[i];
    cc0[i] = od > 0 ? (float)(1.0 / (N * (double)od)) : 0.0f;
  }
  Phase ph;
  Events ev;
  TG_TRY(ev.init());
  if (iters == 0) {
    TG_TRY(pr_write_initial(g, rank, N, s));
    std::fill(crank.begin(), crank.end(), (float)(1.0 / N));
  }
  for (int32_t k = 0; k < iters; ++k) {
    ++ph.supersteps;
    const bool last = k == iters - 1;
    const int b = k & 1;
    const float *cc = reinterpret_cast<const float *>(h.in.h[b]);
    float *cn = reinterpret_cast<float *>(h.in.h[b ^ 1]);
    // GPU-to-host sums, then the host's contributions and the GPU step
    TG_HIP(hipEventRecord(ev.e[0], s));
    TG_TRY(launch_gather(h.dout, s,
                         PrOut{{}, h.dout.rsrc, ws.cbuf[k & 1], reinterpret_cast<float *>(h.out.d[b])},
                         h.dout.partials_f));
    TG_HIP(hipEventRecord(ev.e[1], s));
    TG_TRY(post_d2h(h, b, (size_t)no * sizeof(float), s));
    TG_TRY(post_h2d(h, b, 0, (size_t)C.n * sizeof(float), s));
    TG_HIP(hipEventRecord(ev.e[2], s));
    TG_TRY(launch_gather(h.din, s, PrIn{{}, h.din.rsrc, reinterpret_cast<const float *>(h.in.d[b]), h.din.dst, h.d_ghost},
                         h.din.partials_f));
    // GPU gather with the ghost sums; its dangling mass lands in scalars[(k+1)&1]
    TG_TRY(gpu_pagerank_step(p, damping, mode, k, last, rank, s, h.d_ghost, h.d_bdeg));
    TG_HIP(hipMemcpyAsync(&ws.h_work[2], ws.scalars + ((k + 1) & 1), sizeof(double), hipMemcpyDeviceToHost, s));
    TG_HIP(hipEventRecord(ev.e[3], s));
    // host gather, beside the GPU step
    TG_TRY(wait_d2h(h, b, &ph.exchange_ms));
    const auto tc = clk::now();
    const float *hout = reinterpret_cast<const float *>(h.out.h[b]);
    for (int64_t q = 0; q < no; ++q) ghost[h.g2c.dst[q]] = (double)hout[q];
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
    ph.cpu_ms += ms_since(tc);
    TG_HIP(hipEventSynchronize(ev.e[3]));
    double d_gpu = 0.0;
    memcpy(&d_gpu, &ws.h_work[2], sizeof(double));
    ph.gpu_ms += elapsed(ev.e[0], ev.e[1]) + elapsed(ev.e[2], ev.e[3]);
    ph.exchange_ms += h2d_ms(h, b);
    ph.bytes += (double)(no + C.n) * sizeof(float);
    ph.h2d_bytes += (double)C.n * sizeof(float);
    ph.cpu_edges += (double)C.m;
    D = d_gpu + d_cpu;
    h.h_scalar[0] = D;
    TG_HIP(hipMemcpyAsync(ws.scalars + ((k + 1) & 1), h.h_scalar, sizeof(double), hipMemcpyHostToDevice, s));
  }
  TG_TRY(stage_host_f32(h, crank, rank, s));
  TG_HIP(hipStreamSynchronize(s));
  add_phase_stats(ph);
  ktimer_emit();
  return TG_OK;
}

// -------------------------------------------------------------------- BC
namespace {

// Host-side state of one BC source.
struct HostBc {
  std::vector<uint8_t> vis;
  std::vector<int32_t> lev, hg_lev, slot_of;  // slot_of: host vertex -> GPU-to-host slot
  std::vector<double> sig, del, hg_sig;
  std::vector<float> hg_del;
};

// Brandes for one source (section 7.2, Figure 18) over both partitions.
// Forward: a BFS superstep on each side; each new vertex's sigma is the sum
// over its in-neighbours one level up, local ones pulled, remote ones from
// the sigma messages.  Then each side learns the level and sigma of the
// other side's vertices that its boundary edges reach (once), and the
// backward sweep exchanges, per level, the deltas of those vertices.
int hybrid_bc_source(tg_partition *p, int32_t src, hipStream_t s, std::vector<double> &cscore, HostBc &H,
                     Phase &ph, bool *host_overflow) {
  HybridState &h = *p->hy;
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  CpuPart &C = h.cpu;
  const Tuning &t = p->tune;
  const int64_t V = p->g->n;
  const int64_t no = h.g2c.nslots, ni = h.c2g.nslots;
  const int64_t nwo = (no + 31) / 32, nwc = (C.n + 31) / 32;
  uint32_t *visited = ws.bits_a, *prev = ws.bits_b;
  int32_t *level = ws.state;
  TG_HIP(hipMemsetAsync(visited, 0, ws.nwords * sizeof(uint32_t), s));
  TG_HIP(hipMemsetAsync(prev, 0, ws.nwords * sizeof(uint32_t), s));
  TG_TRY(fill_i32(level, g.n, TG_INF, s));
  TG_TRY(fill_f64(ws.sigma, g.n, 0.0, s));
  TG_TRY(fill_f32(ws.delta, g.n, 0.0f, s));
  if (no) {
    TG_TRY(fill_i32(h.d_osent, no, 0, s));
    TG_TRY(fill_f32(h.d_gh_del, no, 0.0f, s));
  }
  TG_TRY(clear_words(h.d_ochg, nwo, s));
  std::fill(H.vis.begin(), H.vis.end(), 0);
  std::fill(H.lev.begin(), H.lev.end(), TG_INF);
  std::fill(H.sig.begin(), H.sig.end(), 0.0);
  std::fill(H.del.begin(), H.del.end(), 0.0);
  std::fill(H.hg_del.begin(), H.hg_del.end(), 0.0f);
  std::vector<int32_t> cfront, cnext;
  std::vector<std::vector<int32_t>> tl((size_t)omp_get_max_threads());
  const int32_t gl = p->h_l_of_g[src];
  if (gl >= 0) {
    hipLaunchKernelGGL(k_set_f64h, dim3(1), dim3(64), 0, s, ws.sigma, (int64_t)gl, 1.0);
    TG_TRY(set_bit(visited, gl, s));
  } else {
    const int32_t cl = C.l_of_g[src];
    if (cl < 0) return set_error(TG_EDEVICE, "hybrid bc: source %d is on neither side", src);
    H.vis[cl] = 1;
    H.lev[cl] = 0;
    H.sig[cl] = 1.0;
    cfront.push_back(cl);
  }
  TG_TRY(frontier_compact(g, ws, 0, visited, prev, ws.queue, level, 0, s));
  TG_TRY(frontier_plan_off(g, ws, ws.queue, g.out.off, t, s, true));

  std::vector<Plan> plans;
  std::vector<int64_t> segoff;
  std::vector<std::vector<int32_t>> hfront;
  int64_t off = 0;
  int32_t L = 0;
  for (;;) {
    const Plan cur = *ws.h_plan;
    const bool gpu_front = cur.count > 0;
    if (!gpu_front && cfront.empty()) break;
    if (L > V) return set_error(TG_EDEVICE, "hybrid bc: more supersteps than vertices");
    ++ph.supersteps;
    plans.push_back(cur);
    segoff.push_back(off);
    const int b = L & 1;
    if (gpu_front) {
      TG_TRY(bfs_expand_launch(g, ws, ws.queue + off, cur.vb[NBIN], t, s));
      TG_TRY(launch_gather(h.dout, s, SigmaOut{{}, h.dout.rsrc, level, ws.sigma, L, h.d_osent, h.d_oval, h.d_ochg},
                           h.dout.partials_f));
      TG_TRY(launch_select<double>(SelChangedF64{h.d_ochg, h.d_oval}, no, h.out.d[b], s));
      TG_TRY(clear_words(h.d_ochg, nwo, s));
      TG_TRY(post_d2h(h, b, list_prefix_bytes<double>(no), s));
    }
    // the host frontier with its sigma to the GPU, which reduces the
    // host-to-GPU channel over it
    int64_t n_in = 0;
    if (!cfront.empty()) {
      Msg<double> *ie = entries<double>(h.in.h[b]);
      n_in = (int64_t)cfront.size();
      for (int64_t i = 0; i < n_in; ++i) ie[i] = Msg<double>{cfront[i], H.sig[cfront[i]]};
      const size_t bytes = (size_t)n_in * sizeof(Msg<double>);
      TG_TRY(post_h2d(h, b, LIST_HDR, bytes, s));
      TG_TRY(clear_words(h.d_hbits, nwc, s));
      hipLaunchKernelGGL(k_host_state<double>, dim3(nblk(n_in)), dim3(BLOCK), 0, s, entries<double>(h.in.d[b]), n_in,
                         h.d_hsig, h.d_hbits);
      TG_HIP(hipGetLastError());
      TG_TRY(launch_gather(h.din, s, SigmaIn{{}, h.din.rsrc, h.d_hbits, h.d_hsig, h.din.dst, level, ws.sigma, visited},
                           h.din.partials_f));
      ph.bytes += (double)bytes;
      ph.h2d_bytes += (double)bytes;
    }
    // host: expand over its local edges, sigma of its new vertices (pull
    // over local in-edges)
    const auto tc = clk::now();
#pragma omp parallel
    {
      auto &mine = tl[omp_get_thread_num()];
#pragma omp for schedule(dynamic, 64)
      for (size_t i = 0; i < cfront.size(); ++i) {
        const int32_t v = cfront[i];
        for (int64_t e = C.off[v]; e < C.off[v + 1]; ++e) {
          const int32_t x = C.col[e];
          if (!H.vis[x] && !test_and_set(&H.vis[x])) {
            H.lev[x] = L + 1;
            mine.push_back(x);
          }
        }
      }
    }
    concat(tl, cnext);
#pragma omp parallel for schedule(dynamic, 64)
    for (size_t i = 0; i < cnext.size(); ++i) {
      const int32_t x = cnext[i];
      double sg = 0.0;
      for (int64_t e = C.ioff[x]; e < C.ioff[x + 1]; ++e)
        if (H.lev[C.icol[e]] == L) sg += H.sig[C.icol[e]];
      H.sig[x] = sg;
    }
    ph.cpu_ms += ms_since(tc);
    ph.cpu_edges += frontier_edges(C, cfront);
    // GPU: the next frontier and its sigma
    const int64_t noff = off + cur.count;
    TG_TRY(frontier_compact(g, ws, 0, visited, prev, ws.queue + noff, level, L + 1, s));
    TG_TRY(frontier_plan_off(g, ws, ws.queue + noff, g.out.off, t, s, true));
    if (n_in) ph.exchange_ms += h2d_ms(h, b);
    if (ws.h_plan->count > 0) {
      int64_t vbs = ws.h_plan->vb[NBIN];
      if (!g.in_alias) {
        TG_TRY(frontier_plan_off(g, ws, ws.queue + noff, g.in.off, t, s, true, true));
        vbs = ws.h_plan->vb[NBIN];
      }
      SigmaPullHy op{{}, g.in.col, level, ws.sigma, ws.counters, L};
      hipLaunchKernelGGL(k_gather<SigmaPullHy>, dim3(launch_grid(vbs)), dim3(BLOCK), 0, s, ws.plan, ws.queue + noff,
                         ws.hubpref, g.in.off, t.hub_chunk, ws.hub_partials, op);
      hipLaunchKernelGGL(k_gather_hubs<SigmaPullHy>, dim3(64), dim3(BLOCK), 0, s, ws.plan, ws.queue + noff,
                         ws.hubpref, ws.hub_partials, op);
      TG_HIP(hipGetLastError());
      if (!g.in_alias) TG_TRY(frontier_plan_off(g, ws, ws.queue + noff, g.out.off, t, s, true));
    }
    // host: sigma sums from the GPU; a host vertex reached only through them
    // has no local in-neighbour on frontier L
    if (gpu_front) {
      int64_t n_out = 0;
      TG_TRY(fetch_list<double>(h, b, &n_out, &ph.bytes, &ph.exchange_ms));
      const Msg<double> *oe = entries<double>(h.out.h[b]);
      for (int64_t i = 0; i < n_out; ++i) {
        const int32_t x = h.g2c.dst[oe[i].id];
        if (H.lev[x] == TG_INF) {
          H.vis[x] = 1;
          H.lev[x] = L + 1;
          H.sig[x] = oe[i].val;
          cnext.push_back(x);
        } else if (H.lev[x] == L + 1) {
          H.sig[x] += oe[i].val;
        }
      }
    }
    for (int32_t x : cnext)
      if (H.sig[x] >= 9007199254740992.0) *host_overflow = true;
    hfront.push_back(std::move(cfront));
    cfront.swap(cnext);
    cnext.clear();
    off = noff;
    ++L;
  }

  // levels and sigma of the vertices across the boundary: the GPU's
  // host-to-GPU receivers for the host, the host's GPU-to-host receivers
  // for the GPU
  if (ni) {
    double *sig_o = reinterpret_cast<double *>(h.out.d[0]);
    int32_t *lev_o = reinterpret_cast<int32_t *>(h.out.d[0] + (size_t)ni * sizeof(double));
    hipLaunchKernelGGL(k_ghost_out, dim3(nblk(ni)), dim3(BLOCK), 0, s, h.din.dst, ni, level, ws.sigma, sig_o, lev_o);
    TG_HIP(hipGetLastError());
    TG_TRY(post_d2h(h, 0, (size_t)ni * 12, s));
  }
  if (no) {
    double *sig_i = reinterpret_cast<double *>(h.in.h[0]);
    int32_t *lev_i = reinterpret_cast<int32_t *>(h.in.h[0] + (size_t)no * sizeof(double));
    for (int64_t k = 0; k < no; ++k) {
      sig_i[k] = H.sig[h.g2c.dst[k]];
      lev_i[k] = H.lev[h.g2c.dst[k]];
    }
    TG_HIP(hipEventRecord(h.ev_h2d[0][0], h.cs_h2d));
    TG_HIP(hipMemcpyAsync(h.d_gh_sig, sig_i, (size_t)no * sizeof(double), hipMemcpyHostToDevice, h.cs_h2d));
    TG_HIP(hipMemcpyAsync(h.d_gh_lev, lev_i, (size_t)no * sizeof(int32_t), hipMemcpyHostToDevice, h.cs_h2d));
    TG_HIP(hipEventRecord(h.ev_h2d[0][1], h.cs_h2d));
    TG_HIP(hipStreamWaitEvent(s, h.ev_h2d[0][1], 0));
    ph.bytes += (double)no * 12;
    ph.h2d_bytes += (double)no * 12;
  }
  if (ni) {
    TG_TRY(wait_d2h(h, 0, &ph.exchange_ms));
    memcpy(H.hg_sig.data(), h.out.h[0], (size_t)ni * sizeof(double));
    memcpy(H.hg_lev.data(), h.out.h[0] + (size_t)ni * sizeof(double), (size_t)ni * sizeof(int32_t));
    ph.bytes += (double)ni * 12;
  }
  TG_HIP(hipStreamSynchronize(s));
  if (no) ph.exchange_ms += h2d_ms(h, 0);

  // backward: the deepest level keeps delta = 0; levels L-2 .. 1
  for (int32_t lv = L - 2; lv >= 1; --lv) {
    const int b = lv & 1;
    // deltas at level lv+1 of the receivers on the other side
    if (ni) {
      TG_TRY(launch_select<float>(SelLevelDelta{h.din.dst, level, ws.delta, lv + 1}, ni, h.out.d[b], s));
      TG_TRY(post_d2h(h, b, list_prefix_bytes<float>(ni), s));
    }
    int64_t n_in = 0;
    Msg<float> *ie = entries<float>(h.in.h[b]);
    for (int32_t x : hfront[lv + 1])
      if (H.slot_of[x] >= 0) ie[n_in++] = Msg<float>{H.slot_of[x], (float)H.del[x]};
    if (n_in) {
      const size_t bytes = (size_t)n_in * sizeof(Msg<float>);
      TG_TRY(post_h2d(h, b, LIST_HDR, bytes, s));
      hipLaunchKernelGGL(k_inbox_delta, dim3(nblk(n_in)), dim3(BLOCK), 0, s, entries<float>(h.in.d[b]), n_in,
                         h.d_gh_del);
      TG_HIP(hipGetLastError());
      ph.bytes += (double)bytes;
      ph.h2d_bytes += (double)bytes;
    }
    if (ni) {
      int64_t n_out = 0;
      TG_TRY(fetch_list<float>(h, b, &n_out, &ph.bytes, &ph.exchange_ms));
      const Msg<float> *oe = entries<float>(h.out.h[b]);
      for (int64_t i = 0; i < n_out; ++i) H.hg_del[oe[i].id] = oe[i].val;
    }
    // GPU: delta of level lv, boundary children first
    const Plan &P = plans[lv];
    if (P.count > 0) {
      TG_HIP(hipMemcpyAsync(ws.plan, &P, sizeof(Plan), hipMemcpyHostToDevice, s));
      TG_TRY(frontier_plan_off(g, ws, ws.queue + segoff[lv], h.d_fb_off, t, s, true, true));
      DeltaBoundary ob{{}, h.d_fb_slot, h.d_gh_lev, h.d_gh_sig, h.d_gh_del, ws.sigma, g.out.off,
                       ws.delta, ws.bc_acc, h.d_bdel, lv + 1};
      hipLaunchKernelGGL(k_gather<DeltaBoundary>, dim3(launch_grid(ws.h_plan->vb[NBIN])), dim3(BLOCK), 0, s, ws.plan,
                         ws.queue + segoff[lv], ws.hubpref, h.d_fb_off, t.hub_chunk, ws.hub_partials, ob);
      hipLaunchKernelGGL(k_gather_hubs<DeltaBoundary>, dim3(64), dim3(BLOCK), 0, s, ws.plan, ws.queue + segoff[lv],
                         ws.hubpref, ws.hub_partials, ob);
      TG_HIP(hipGetLastError());
      TG_HIP(hipMemcpyAsync(ws.plan, &P, sizeof(Plan), hipMemcpyHostToDevice, s));
      TG_TRY(frontier_plan_off(g, ws, ws.queue + segoff[lv], g.out.off, t, s, false));
      DeltaAccumHy oa{{}, g.out.col, level, ws.sigma, h.d_bdel, ws.delta, ws.bc_acc, lv + 1};
      hipLaunchKernelGGL(k_gather<DeltaAccumHy>, dim3(launch_grid(P.vb[NBIN])), dim3(BLOCK), 0, s, ws.plan,
                         ws.queue + segoff[lv], ws.hubpref, g.out.off, t.hub_chunk, ws.hub_partials, oa);
      hipLaunchKernelGGL(k_gather_hubs<DeltaAccumHy>, dim3(64), dim3(BLOCK), 0, s, ws.plan, ws.queue + segoff[lv],
                         ws.hubpref, ws.hub_partials, oa);
      TG_HIP(hipGetLastError());
    }
    // host: delta of level lv
    const auto tc = clk::now();
    const std::vector<int32_t> &fr = hfront[lv];
#pragma omp parallel for schedule(dynamic, 64)
    for (size_t i = 0; i < fr.size(); ++i) {
      const int32_t v = fr[i];
      const double sv = H.sig[v];
      double d = 0.0;
      for (int64_t e = C.off[v]; e < C.off[v + 1]; ++e) {
        const int32_t w = C.col[e];
        if (H.lev[w] == lv + 1) d += sv / H.sig[w] * (1.0 + H.del[w]);
      }
      for (int64_t e = h.hb_off[v]; e < h.hb_off[v + 1]; ++e) {
        const int32_t k = h.hb_slot[e];
        if (H.hg_lev[k] == lv + 1) d += sv / H.hg_sig[k] * (1.0 + (double)H.hg_del[k]);
      }
      H.del[v] = d;
      cscore[v] += d;
    }
    ph.cpu_ms += ms_since(tc);
    TG_HIP(hipStreamSynchronize(s));  // the GPU's deltas of level lv are final
    if (n_in) ph.exchange_ms += h2d_ms(h, b);
  }
  return TG_OK;
}

}  // namespace

int hybrid_bc(tg_partition *p, const int32_t *sources, int32_t ns, float *scores, hipStream_t s) {
  HybridState &h = *p->hy;
  GpuPart &g = p->gpu;
  Workspace &ws = p->ws;
  CpuPart &C = h.cpu;
  // the boundary delta gather chunks hubs by their boundary degree
  TG_TRY(ws.ensure(g, h.g2c.edges() / p->tune.hub_chunk + g.max_out_hubs + 1));
  const int64_t no = h.g2c.nslots, ni = h.c2g.nslots;
  // GPU -> host: sigma lists over GPU-to-host slots, delta lists and the
  // (sigma, level) arrays over host-to-GPU slots; host -> GPU: sigma lists
  // over host vertices, delta lists and the (sigma, level) arrays over
  // GPU-to-host slots
  const size_t ob = std::max({list_bytes<double>(no), list_bytes<float>(ni), (size_t)ni * 12 + 16});
  const size_t ib = std::max({list_bytes<double>(C.n), list_bytes<float>(no), (size_t)no * 12 + 16});
  TG_TRY(hybrid_boxes(h, ob, ib));
  HostBc H;
  H.vis.resize((size_t)C.n);
  H.lev.resize((size_t)C.n);
  H.sig.resize((size_t)C.n);
  H.del.resize((size_t)C.n);
  H.hg_lev.resize((size_t)ni);
  H.hg_sig.resize((size_t)ni);
  H.hg_del.resize((size_t)ni);
  H.slot_of.assign((size_t)C.n, -1);
  for (int64_t k = 0; k < no; ++k) H.slot_of[h.g2c.dst[k]] = (int32_t)k;
  std::vector<double> cscore((size_t)C.n, 0.0);
  TG_TRY(fill_f64(ws.bc_acc, g.n, 0.0, s));
  TG_HIP(hipMemsetAsync(ws.counters, 0, 64 * sizeof(uint32_t), s));
  Phase ph;
  bool host_overflow = false;
  for (int32_t i = 0; i < ns; ++i) TG_TRY(hybrid_bc_source(p, sources[i], s, cscore, H, ph, &host_overflow));
  TG_TRY(collect_f64_to_f32(g, ws.bc_acc, scores, s));
  std::vector<float> cs((size_t)C.n);
  for (int64_t i = 0; i < C.n; ++i) cs[i] = (float)cscore[i];
  TG_TRY(stage_host_f32(h, cs, scores, s));
  TG_HIP(hipMemcpyAsync(ws.h_flags, ws.counters, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  TG_HIP(hipStreamSynchronize(s));
  if (ws.h_flags[2] || host_overflow) return set_error(TG_ERANGE, "bc: a shortest-path count reached 2^53");
  stats_add("sources", ns);
  add_phase_stats(ph);
  ktimer_emit();
  return TG_OK;
}

}  // namespace tg

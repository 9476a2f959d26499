// Device-side building blocks shared by the superstep kernels: degree bins,
// the frontier plan, and the mapping of a virtual block to (vertex, lanes).
//
// Vertices of a GPU partition are relabelled in order of decreasing degree
// (partition by degree centrality, section 6.2), so each degree bin is a
// contiguous id range and a frontier queue sorted by id is also sorted by
// degree: its bins are contiguous queue segments.
//
// Bin -> lanes per vertex (wave64, 256-thread blocks):
//   HUB   : several blocks per vertex, each taking `hub_chunk` edges
//   BLOCK : one 256-thread block per vertex
//   WAVE  : one 64-lane wavefront per vertex (4 per block)
//   G16   : 16 lanes per vertex (16 per block)
//   G4    : 4 lanes per vertex (64 per block)
//   G1    : one lane per vertex (256 per block)
//   ZERO  : degree 0, no edge work
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tgk {

constexpr int NBIN = 7;
enum { BIN_HUB = 0, BIN_BLOCK = 1, BIN_WAVE = 2, BIN_G16 = 3, BIN_G4 = 4, BIN_G1 = 5, BIN_ZERO = 6 };
constexpr int BLOCK = 256;
// vertices handled by one virtual block, per bin (HUB: per chunk)
// (ZERO is laid out like G1 so that kernels which must touch every vertex,
// such as the last PageRank step, can walk it.)
__host__ __device__ constexpr int verts_per_vblock(int b) {
  return b == BIN_WAVE ? 4 : b == BIN_G16 ? 16 : b == BIN_G4 ? 64 : (b == BIN_G1 || b == BIN_ZERO) ? 256 : 1;
}
__host__ __device__ constexpr int lanes_per_vertex(int b) {
  return b == BIN_WAVE ? 64 : b == BIN_G16 ? 16 : b == BIN_G4 ? 4 : (b == BIN_G1 || b == BIN_ZERO) ? 1 : 256;
}

// First vertex id of each bin (bstart[NBIN] = n).  Passed by value.
struct BinBounds {
  int64_t bstart[NBIN + 1];
};

// Frontier plan: queue segments per bin and virtual-block offsets.
struct Plan {
  int32_t count;           // frontier length
  int32_t queue_skipped;  // device-resident BFS: 1 if the last compaction wrote no queue
  int32_t pos[NBIN + 1];   // queue index where bin b starts; pos[NBIN] = count
  int64_t vb[NBIN + 1];    // virtual blocks of bin b: [vb[b], vb[b+1])
};

// Device-resident control block of one BFS (the superstep loop of section
// 4.1 run without the host): the one-block plan kernel advances it after
// each compaction, and every other kernel of a superstep reads it to decide
// whether it has work.  Once the frontier is empty the search is over and
// the remaining supersteps of a chunk are no-ops.
struct BfsCtl {
  int64_t m_u;        // out-edges of vertices not yet in any frontier
  int32_t L;          // level of the current frontier (-1 before the root's compaction)
  int32_t bottom_up;  // 1: the current superstep runs bottom-up
  int32_t active;     // 0 once a compaction produced an empty frontier
  int32_t steps;      // non-empty frontiers expanded so far
};

// Copy the plan into LDS (it is indexed by the block's bin, so a register
// copy would be spilled to scratch).  Every thread must call this.
__device__ __forceinline__ const Plan &load_plan(const Plan *__restrict__ Pp) {
  __shared__ Plan sP;
  constexpr int words = (int)(sizeof(Plan) / sizeof(uint32_t));
  if (threadIdx.x < words)
    reinterpret_cast<uint32_t *>(&sP)[threadIdx.x] = reinterpret_cast<const uint32_t *>(Pp)[threadIdx.x];
  __syncthreads();
  return sP;
}

// Streaming read of edge data: bypass-friendly, so that the edge stream does
// not evict the randomly accessed vertex state from the caches.
template <typename T>
__device__ __forceinline__ T stream_load(const T *p) {
  return __builtin_nontemporal_load(p);
}

// Work of one thread inside a virtual block.
struct Assign {
  int32_t v;        // vertex (local id), valid only if ok
  int32_t qi;       // queue index of v
  int64_t e_begin;  // first edge this group handles
  int64_t e_end;    // one past its last edge
  int lane;         // lane within the group
  int stride;       // group size
  int bin;          // bin of this virtual block (block-uniform)
  int64_t chunk;    // HUB only: global chunk index
  bool ok;
};

__device__ __forceinline__ int segment_of(int64_t vb, const Plan &P) {
  int b = 0;
#pragma unroll
  for (int k = 1; k < NBIN; ++k) b += (vb >= P.vb[k]) ? 1 : 0;
  // a bin with no virtual blocks has vb[k] == vb[k+1]; the count above
  // already skips over it because vb is non-decreasing
  return b;
}

// As assign_work_rows, with vertex v's edges [first(v), last(v)); a hub's
// chunks start at first(v).
template <typename FirstF, typename LastF>
__device__ __forceinline__ Assign assign_work_range(int64_t vb, const Plan &P, const int32_t *queue,
                                                    const int32_t *order, const int64_t *hubpref, FirstF first,
                                                    LastF last, int64_t hub_chunk);

// Map virtual block `vb` to this thread's work.  `queue == nullptr` means the
// identity frontier (every vertex, in id order) optionally through `order`.
// `row(i)` returns the offset of row i (rows v and v+1 bound vertex v's edges).
template <typename RowF>
__device__ __forceinline__ Assign assign_work_rows(int64_t vb, const Plan &P, const int32_t *queue,
                                                   const int32_t *order, const int64_t *hubpref, RowF row,
                                                   int64_t hub_chunk) {
  return assign_work_range(vb, P, queue, order, hubpref, [row](int32_t v) { return row(v); },
                           [row](int32_t v) { return row((int64_t)v + 1); }, hub_chunk);
}

template <typename FirstF, typename LastF>
__device__ __forceinline__ Assign assign_work_range(int64_t vb, const Plan &P, const int32_t *queue,
                                                    const int32_t *order, const int64_t *hubpref, FirstF first,
                                                    LastF last, int64_t hub_chunk) {
  Assign a;
  a.ok = false;
  a.chunk = -1;
  const int t = threadIdx.x;
  const int b = segment_of(vb, P);
  a.bin = b;
  int64_t local = vb - P.vb[b];
  int32_t qi;
  if (b == BIN_HUB) {
    // find hub i with hubpref[i] <= local < hubpref[i+1]
    int lo = 0, hi = P.pos[1] - P.pos[0];
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (hubpref[mid] <= local) lo = mid; else hi = mid;
    }
    qi = P.pos[0] + lo;
    int32_t v = queue ? queue[qi] : (order ? order[qi] : qi);
    int64_t k = local - hubpref[lo];
    a.e_begin = first(v) + k * hub_chunk;
    int64_t end = last(v);
    a.e_end = (a.e_begin + hub_chunk < end) ? a.e_begin + hub_chunk : end;
    a.v = v;
    a.qi = qi;
    a.lane = t;
    a.stride = BLOCK;
    a.chunk = local;
    a.ok = true;
    return a;
  }
  const int vpb = verts_per_vblock(b);
  const int lpv = lanes_per_vertex(b);
  qi = P.pos[b] + (int32_t)(local * vpb) + t / lpv;
  a.lane = t % lpv;
  a.stride = lpv;
  a.qi = qi;
  if (qi < P.pos[b + 1]) {
    int32_t v = queue ? stream_load(queue + qi) : (order ? stream_load(order + qi) : qi);
    a.v = v;
    a.e_begin = first(v);
    a.e_end = last(v);
    a.ok = true;
  }
  return a;
}

__device__ __forceinline__ Assign assign_work(int64_t vb, const Plan &P, const int32_t *queue,
                                              const int32_t *order, const int64_t *hubpref,
                                              const int64_t *off, int64_t hub_chunk) {
  return assign_work_rows(vb, P, queue, order, hubpref, [off](int64_t i) { return stream_load(off + i); },
                          hub_chunk);
}

// ------------------------------------------------------------ reductions

template <typename T>
__device__ __forceinline__ T group_sum(T x, int width) {
  // butterfly within groups of `width` lanes (power of two <= 64)
  for (int o = width >> 1; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Per-call counters that every block of a large grid adds to.  Atomics from
// thousands of blocks on one address serialize (device-scope atomics are
// resolved beyond the L2): a counter is STAT_SLOTS slots on separate
// 128-byte lines, block b adds into slot b mod STAT_SLOTS, and the host sums
// the slots.  Counter k starts at stat_counter(base, k).
constexpr int STAT_SLOTS = 64;
constexpr int STAT_STRIDE = 16;  // unsigned long longs between slots (128 bytes)
constexpr int STAT_SPAN = STAT_SLOTS * STAT_STRIDE;
constexpr int STAT_COUNTERS = 8;

__host__ __device__ __forceinline__ unsigned long long *stat_counter(unsigned long long *base, int k) {
  return base + (size_t)k * STAT_SPAN;
}

__device__ __forceinline__ void stat_add(unsigned long long *counter, unsigned long long x) {
  atomicAdd(counter + (size_t)(blockIdx.x & (STAT_SLOTS - 1)) * STAT_STRIDE, x);
}

// Sum over the 256-thread block; every thread gets the result.
template <typename T>
__device__ __forceinline__ T block_sum(T x) {
  __shared__ T red[BLOCK / 64];
  x = wave_sum(x);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = x;
  __syncthreads();
  T s = red[0];
#pragma unroll
  for (int k = 1; k < BLOCK / 64; ++k) s += red[k];
  return s;
}

// Exclusive prefix sum over the 256-thread block; `total` gets the sum.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t &total) {
  __shared__ uint32_t wsum[BLOCK / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = x;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  __syncthreads();
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t before = 0;
  total = 0;
#pragma unroll
  for (int k = 0; k < BLOCK / 64; ++k) {
    if (k < w) before += wsum[k];
    total += wsum[k];
  }
  return before + inc - x;
}

}  // namespace tgk

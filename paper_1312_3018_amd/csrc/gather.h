// Generic degree-binned gather-reduce over a queue of rows: for each row v,
// r(v) = reduce over edges e of v of op.term(vs, e), then op.finish(v, r(v))
// once, where vs = op.vstate(v) is loaded once per row; a row whose state
// fails op.live(vs) skips its edges and reduces to the identity.  The
// reduction is op.combine (associative, commutative) with identity
// op.identity().
//
// Hub rows are split into chunks of `hub_chunk` edges, one block each; a chunk
// block stores its partial and a second launch (k_gather_hubs, one wave per
// hub) combines each hub's partials with a fixed reduction tree, so the
// result does not depend on scheduling.  (A "last block to finish combines"
// scheme would need device-scope fences, which write back and invalidate the
// XCD's L2 on this part.)  Used for the BC sigma pull and delta accumulation
// and for the atomic-free outbox reductions of the hybrid split.
#pragma once
#include "kcommon.h"

namespace tgk {

template <typename T, class Op>
__device__ __forceinline__ T group_reduce(T x, int width, const Op &op) {
  for (int o = width >> 1; o > 0; o >>= 1) x = op.combine(x, __shfl_xor(x, o, 64));
  return x;
}

template <typename T, class Op>
__device__ __forceinline__ T block_reduce(T x, const Op &op) {
  __shared__ T red[BLOCK / 64];
  x = group_reduce(x, 64, op);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = x;
  __syncthreads();
  T s = red[0];
#pragma unroll
  for (int k = 1; k < BLOCK / 64; ++k) s = op.combine(s, red[k]);
  return s;
}

// Sum in fp64: the default reduction.
struct SumF64 {
  using T = double;
  __device__ static double identity() { return 0.0; }
  __device__ static double combine(double a, double b) { return a + b; }
  template <typename V>
  __device__ static bool live(V) { return true; }
};

template <class Op>
__global__ __launch_bounds__(BLOCK) void k_gather(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                  const int64_t *__restrict__ hubpref,
                                                  const int64_t *__restrict__ off, int64_t hub_chunk,
                                                  typename Op::T *hub_partials, Op op) {
  using T = typename Op::T;
  const Plan &P = load_plan(Pp);
  const int64_t total = P.vb[NBIN];
  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const Assign a = assign_work(vb, P, queue, nullptr, hubpref, off, hub_chunk);
    T s = op.identity();
    if (a.ok) {
      const auto vs = op.vstate(a.v);
      if (op.live(vs))
        for (int64_t e = a.e_begin + a.lane; e < a.e_end; e += a.stride) s = op.combine(s, op.term(vs, e));
    }
    if (a.bin == BIN_HUB) {
      s = block_reduce(s, op);
      if (threadIdx.x == 0) hub_partials[a.chunk] = s;  // finished by k_gather_hubs
      continue;
    }
    if (a.bin == BIN_BLOCK) s = block_reduce(s, op);
    else s = group_reduce(s, a.stride, op);
    if (a.ok && a.lane == 0) op.finish(a.v, s);
  }
}

// One wave per hub of the plan: combine its chunk partials (lane-strided,
// then a fixed butterfly) and finish the row.
template <class Op>
__global__ __launch_bounds__(BLOCK) void k_gather_hubs(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                       const int64_t *__restrict__ hubpref,
                                                       const typename Op::T *__restrict__ hub_partials, Op op) {
  using T = typename Op::T;
  const int32_t p0 = Pp->pos[0], nh = Pp->pos[1] - p0;
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * BLOCK) >> 6;
  for (int64_t i = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6; i < nh; i += nw) {
    T s = op.identity();
    for (int64_t c = hubpref[i] + lane; c < hubpref[i + 1]; c += 64) s = op.combine(s, hub_partials[c]);
    s = group_reduce(s, 64, op);
    if (lane == 0) op.finish(queue ? queue[p0 + i] : p0 + (int32_t)i, s);
  }
}

}  // namespace tgk

// Generic degree-binned gather-reduce over a frontier queue: for each
// frontier vertex v, s(v) = sum over edges e of v of op.term(vs, e) (fp64),
// then op.finish(v, s(v)) once.  `vs` is op.vstate(v), loaded once per
// vertex.  Hub vertices are split into chunks of `hub_chunk` edges; the last
// chunk block of a hub to finish sums the chunk partials in chunk order, so
// the result does not depend on scheduling.
#pragma once
#include "kcommon.h"

namespace tgk {

template <class Op>
__global__ __launch_bounds__(BLOCK) void k_gather(const Plan *__restrict__ Pp, const int32_t *__restrict__ queue,
                                                  const int64_t *__restrict__ hubpref,
                                                  const int64_t *__restrict__ off, int64_t hub_chunk,
                                                  double *hub_partials, uint32_t *hub_counters, Op op) {
  __shared__ int s_last;
  const Plan P = *Pp;
  const int64_t total = P.vb[NBIN];
  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const Assign a = assign_work(vb, P, queue, nullptr, hubpref, off, hub_chunk);
    double s = 0.0;
    if (a.ok) {
      const double vs = op.vstate(a.v);
      for (int64_t e = a.e_begin + a.lane; e < a.e_end; e += a.stride) s += op.term(vs, e);
    }
    if (a.bin == BIN_HUB) {
      s = block_sum(s);
      const int32_t hi = a.qi - P.pos[0];
      if (threadIdx.x == 0) {
        hub_partials[a.chunk] = s;
        __threadfence();
        const uint32_t nchunks = (uint32_t)(hubpref[hi + 1] - hubpref[hi]);
        const uint32_t prev = atomicAdd(hub_counters + hi, 1u);
        s_last = (prev == nchunks - 1) ? 1 : 0;
      }
      __syncthreads();
      if (s_last && threadIdx.x == 0) {
        __threadfence();
        double tot = 0.0;
        for (int64_t k = hubpref[hi]; k < hubpref[hi + 1]; ++k)
          tot += __hip_atomic_load(hub_partials + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        op.finish(a.v, tot);
        hub_counters[hi] = 0u;
      }
      __syncthreads();
      continue;
    }
    if (a.bin == BIN_BLOCK) s = block_sum(s);
    else s = group_sum(s, a.stride);
    if (a.ok && a.lane == 0) op.finish(a.v, s);
  }
}

}  // namespace tgk

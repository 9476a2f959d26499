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

struct HybridState;

// Stable counting sort of `ids` by decreasing key[id] (keys >= 0).
void sort_desc_by_key(const std::vector<int64_t> &key, std::vector<int32_t> &ids);
void transpose_csr(int64_t n, const std::vector<int64_t> &off, const std::vector<int32_t> &col,
                   std::vector<int64_t> &ioff, std::vector<int32_t> &icol);
int build_gpu_part(tg_partition *p, const std::vector<int32_t> &verts, BoundaryEdges *boundary);
int build_hybrid(tg_partition *p, uint64_t seed);
void hybrid_free(tg_partition *p);
std::string hybrid_info_json(const tg_partition *p);
int hybrid_bfs(tg_partition *p, const int32_t *roots, int32_t nr, int32_t *levels, int32_t *parents,
               hipStream_t s);
int hybrid_sssp(tg_partition *p, const int32_t *roots, int32_t nr, int32_t *dist, hipStream_t s);
int hybrid_pagerank(tg_partition *p, double damping, int32_t iters, int mode, float *rank, hipStream_t s);

}  // namespace tg

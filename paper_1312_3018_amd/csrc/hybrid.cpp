#include "hybrid.h"

namespace tg {

int build_hybrid(tg_partition *, uint64_t) {
  return set_error(TG_EUNSUPPORTED, "partition_by_degree: cpu_edge_share > 0 is not available yet");
}
void hybrid_free(tg_partition *) {}
std::string hybrid_info_json(const tg_partition *) { return ""; }
int hybrid_bfs(tg_partition *, const int32_t *, int32_t, int32_t *, int32_t *, hipStream_t) {
  return set_error(TG_EUNSUPPORTED, "hybrid bfs unavailable");
}
int hybrid_sssp(tg_partition *, const int32_t *, int32_t, int32_t *, hipStream_t) {
  return set_error(TG_EUNSUPPORTED, "hybrid sssp unavailable");
}
int hybrid_pagerank(tg_partition *, double, int32_t, int, float *, hipStream_t) {
  return set_error(TG_EUNSUPPORTED, "hybrid pagerank unavailable");
}

}  // namespace tg

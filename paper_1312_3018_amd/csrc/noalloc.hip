// Breadth-first search for callers that cannot allocate device memory (code
// under stream capture, serving loops with a fixed memory budget): the
// search's workspace lives in a file-scope device array instead of the
// partition's allocated workspace.  The array is part of the library's code
// object, so each GPU the library is loaded on holds it until the process
// ends.
#include <mutex>

#include "tg_internal.h"

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
// Per device: the array's device address (found once, with that device
// current) and a lock that serializes the calls using it.
struct DeviceScratch {
  std::mutex mu;
  void *ptr = nullptr;
  tgk::BfsCtl host_ctl{};  // read-back of the control block (pageable host memory)
};
DeviceScratch g_dev[MAX_DEVICES];

}  // namespace

extern "C" int bfs_noalloc(const tg_partition *pc, const int32_t *roots, int32_t num_roots, int32_t *levels,
                           void *stream) {
  using namespace tg;
  clear_error();
  if (!pc) return set_error(TG_EINVAL, "bfs_noalloc: partition is NULL");
  if (!levels) return set_error(TG_EINVAL, "bfs_noalloc: levels is NULL");
  if (num_roots < 0 || (num_roots > 0 && !roots)) return set_error(TG_EINVAL, "bfs_noalloc: bad roots");
  for (int32_t r = 0; r < num_roots; ++r)
    if (roots[r] < 0 || roots[r] >= pc->g->n)
      return set_error(TG_EINVAL, "bfs_noalloc: root %d out of range [0, %lld)", roots[r], (long long)pc->g->n);
  if (pc->alpha > 0.0) return set_error(TG_EUNSUPPORTED, "bfs_noalloc: GPU-only partitions (cpu_edge_share 0)");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
    return set_error(TG_EDEVICE, "bfs_noalloc: no usable current device");
  if (dev != pc->device)
    return set_error(TG_EINVAL, "bfs_noalloc: the partition lives on device %d, device %d is current", pc->device,
                     dev);
  DeviceScratch &D = g_dev[dev];
  std::lock_guard<std::mutex> lock(D.mu);
  if (!D.ptr) {
    // the array's address on this device (host code may not use its name)
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_error(TG_EDEVICE, "bfs_noalloc: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
    D.ptr = ptr;
  }
  tg_partition *p = const_cast<tg_partition *>(pc);
  Workspace ws;
  TG_TRY(ws.bind_bfs(p->gpu, D.ptr, SCRATCH_BYTES));
  stats_reset("bfs");
  return gpu_bfs_roots_bound(p, ws, roots, num_roots, levels, (hipStream_t)stream, &D.host_ctl);
}

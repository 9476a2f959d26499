// Multi-source (slot) engine: up to 64 BFS or SSSP queries advancing together
// over one GPU partition, joining and retiring at superstep boundaries.
#pragma once
#include <stdint.h>

#include "tg_internal.h"

namespace tg {

constexpr int kSlots = 64;
enum { kSlotBfs = 0, kSlotSssp = 1 };

// Per-slot output pointer (BFS levels are written as they settle) and the
// superstep at which the slot's root had level 0.  Passed by value.
struct SlotTable {
  int32_t *out[kSlots];
  int32_t join[kSlots];
};

struct SlotEngine {
  tg_partition *p = nullptr;
  int kind = kSlotBfs;
  hipStream_t s = nullptr;
  Workspace ws;       // frontier queue, plan, touched bitmap (bits_a), flags
  DevArena arena;
  unsigned long long *visited = nullptr, *frontier = nullptr, *next = nullptr, *alive = nullptr;
  int32_t *dist = nullptr;  // SSSP: [n][kSlots]
  // SSSP overflow: per vertex, the slots whose candidate for it did not fit
  // in int32; ovf_slots[0] = the slots with any such mark, [1] = scratch
  unsigned long long *ovf = nullptr, *ovf_slots = nullptr;
  unsigned long long *h_alive = nullptr, *h_ovf = nullptr;
  SlotTable tab{};
  unsigned long long busy = 0;  // slots in use
  int64_t step = 0;             // superstep counter (levels are step - join)
  int64_t supersteps = 0;
  bool have_queue = false;
  ~SlotEngine();
  int init(tg_partition *part, int kind, hipStream_t stream);
  int free_slot() const;
  // Slot `slot` starts at local root; BFS levels go to out_global (original
  // ids, filled with TG_INF first).  Takes effect at the next superstep.
  int join(int slot, int32_t root_local, int32_t *out_global);
  // One superstep; `finished` gets the slots whose frontier became empty.
  // launch_step() only enqueues (so several engines can overlap on the
  // device); finish_step() waits for it.
  int superstep(unsigned long long *finished);
  int launch_step();
  int finish_step(unsigned long long *finished);
  // Release finished slots (SSSP: write their distances to tab.out first,
  // and set in *overflow the slots among them whose true distances do not
  // all fit below INT32_MAX, the exact verdict of sssp()).
  int retire(unsigned long long mask, unsigned long long *overflow);
};

int slots_run_batch(tg_partition *p, int kind, const int32_t *roots, int32_t nr, int32_t *out, hipStream_t s,
                    int64_t *supersteps_out);

}  // namespace tg

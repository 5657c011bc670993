// batch_core.hpp -- device helpers shared by the persistent batch scans
// (batch.hip, and the NaN-aware one in nan.hip): the wave-uniform scan
// parameters of a task and the task that owns a work item.
#pragma once

#include "common.hpp"
#include "internal.hpp"

namespace tsds {

// A task's scan parameters, every field read from the task table made
// wave-uniform.
__device__ inline ScanParams task_scan_params_uniform(char *ws, const BatchTask *__restrict__ t, int32_t small) {
  ScanParams sp;
  sp.y = uniform(t->y);
  sp.n = uniform(t->n);
  sp.shift = uniform(t->shift);
  sp.chunk = uniform(t->chunk);
  sp.nchunks = uniform(t->nchunks);
  const void *x = uniform(t->x);
  sp.edges = x ? (const int64_t *)(ws + uniform(t->o_edges)) : nullptr;
  sp.nb = uniform(t->nb);
  sp.binres = (int64_t *)(ws + uniform(t->o_binres));
  sp.partL = (Partial *)(ws + uniform(t->o_partL));
  sp.partR = (Partial *)(ws + uniform(t->o_partR));
  sp.small = small;
  sp.variant = 3;
  sp.stage = uniform(t->stage);
  sp.x = nullptr;
  sp.xedges = nullptr;
  sp.xclass = 0;
  return sp;
}

// Task (index into the task table) of a group's work item: the last task of
// the group's list whose first item is <= item (tasks without items share
// their successor's start).  A 64-wide probe of the list narrows the range
// 64-fold per round; in the last round (step 1) the probe is exact, and the
// lanes load the task indices beside the starts, so the answer comes from a
// lane of that same round trip (one dependent load per round, none after).
__device__ inline int32_t group_task_of_item(const int64_t *__restrict__ cb, const int32_t *__restrict__ tix,
                                             int64_t ntasks, int64_t item, int lane) {
  if (ntasks <= 1) return uniform(tix[0]);
  int64_t lo = 0, hi = ntasks;  // cb[lo] <= item < cb[hi]
  for (;;) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t q = lo + (int64_t)lane * step;
    const bool le = q < hi && cb[q] <= item;
    int32_t tq = 0;
    if (step == 1 && q < hi) tq = tix[q];
    const int cnt = __builtin_popcountll(ballot(le));  // >= 1: lane 0 probes lo
    if (step == 1) return uniform(__builtin_amdgcn_readlane(tq, cnt - 1));
    const int64_t nlo = lo + (int64_t)(cnt - 1) * step;
    const int64_t nhi = lo + (int64_t)cnt * step;
    lo = nlo;
    hi = nhi < hi ? nhi : hi;
  }
}

}  // namespace tsds

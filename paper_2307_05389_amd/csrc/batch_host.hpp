// batch_host.hpp -- host-side batch planning shared by the batched C ABI
// (api_batch.cpp) and the serving engine (serve.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "internal.hpp"
#include "tsds.h"

// Work-list groups: g = dtype + 11 * staged for the plain scan, 22 + dtype
// for NaN-aware tasks (floating-point y only), 33 + dtype for tasks reduced
// one wavefront per bin (work items are bins, not chunks).
constexpr int kBatchGroups = 44;
constexpr int kBatchDirectGroup = 33;

struct ts_plan {
  std::vector<ts_task> in;
  std::vector<tsds::BatchTask> tasks;
  std::vector<int32_t> slot_task, lttb_tasks;
  int64_t total_chunks = 0, total_slots = 0;
  int64_t wave_slots = 0;   // slots of tasks merged a wavefront per bin come first
  // per group (see kBatchGroups): task list and first work items
  std::vector<int64_t> group_cb[kBatchGroups];
  std::vector<int32_t> group_tix[kBatchGroups];
  int64_t group_total[kBatchGroups] = {0};
  double group_bytes[kBatchGroups] = {0};  // bytes of y the group reads
  size_t group_off_cb[kBatchGroups] = {0}, group_off_tix[kBatchGroups] = {0};
  size_t ws_bytes = 0;      // for the largest chunk count in the tuning space
  int64_t out_needed = 0;   // max(out_offset + n_out)
  bool any_x = false;
  int64_t max_m = 0;        // largest MinMaxLTTB candidate capacity
  // tuning
  int64_t chunk_bytes = 65536;
  int32_t small = 128;
  int64_t grid_blocks = 0;
  // device table
  void *d_table = nullptr;
  size_t table_bytes = 0;
  int device = 0;
  // side streams (default priority) on which the scans of different element
  // types overlap, joined back before the merge; created on first use
  static constexpr int kSide = 3;
  hipStream_t side[kSide] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kSide] = {nullptr, nullptr, nullptr};
  // graph
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void *g_out = nullptr, *g_counts = nullptr, *g_ws = nullptr;
};

namespace tsds {

// Lays out every task of p->in for chunk size chunk_bytes (tables, offsets,
// workspace regions); returns the workspace bytes.
size_t batch_layout(ts_plan *p, int64_t chunk_bytes);
// Size of the device table for the current layout (sets its internal offsets).
size_t batch_table_bytes(ts_plan *p);
// Writes the device table image (batch_table_bytes bytes) to dst.
void batch_pack_table(const ts_plan *p, char *dst);
// Enqueues the batch kernels using a device table already holding the image.
// With fan set and the plan's side streams created, the scans of different
// element types run on up to 1 + kSide streams (forked from and joined back
// to st, so the caller sees one ordered sequence on st).
int batch_enqueue(const ts_plan *p, const void *d_table, int64_t *out, int64_t *counts, void *ws, hipStream_t st,
                  bool fan = false);
// Validation of one task (same rules as the single-series calls).
int batch_check_task(const ts_task &t);

}  // namespace tsds

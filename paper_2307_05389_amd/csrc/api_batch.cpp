// api_batch.cpp -- batched downsampling: plan (per-series offset tables and
// workspace layout), eager or hipGraph launch, and an autotuner over the
// chunk size, the one-lane-per-bin threshold and the persistent grid size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"
#include "batch_host.hpp"
#include "internal.hpp"
#include "tsds.h"

namespace tsds {

size_t lttb_group_count(int64_t n_out);

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace tsds

using namespace tsds;


namespace {

const int64_t kMinChunk = 4096;
const int64_t kStageBin = 4096, kStageChunk = 8192;
// Tasks without x whose bins hold 4..512 KB of y: one wavefront per bin (the
// single-series rule, also for bins of fewer than kStageBin elements), no
// chunks and no merge.
const int64_t kDirectMinBinBytes = 4096, kDirectMaxBinBytes = 512 << 10;

size_t esize(int dt) { return elem_size(dt); }

}  // namespace

namespace tsds {

size_t batch_layout(ts_plan *p, int64_t chunk_bytes) {
  p->tasks.clear();
  p->slot_task.clear();
  p->lttb_tasks.clear();
  p->total_chunks = 0;
  p->total_slots = 0;
  p->any_x = false;
  p->max_m = 0;
  for (int g = 0; g < kBatchGroups; g++) {
    p->group_cb[g].clear();
    p->group_tix[g].clear();
    p->group_total[g] = 0;
    p->group_bytes[g] = 0;
  }
  size_t o = 0;
  int64_t ti = 0;
  for (const ts_task &in : p->in) {
    BatchTask t;
    memset(&t, 0, sizeof t);
    const ts_series &s = in.series;
    // NaN-aware calls on integer y are the plain ones (no NaN to skip)
    const bool fy = s.y_dtype == TS_F16 || s.y_dtype == TS_F32 || s.y_dtype == TS_F64;
    t.algo = fy ? in.algo : in.algo == TS_NAN_MINMAX ? TS_MINMAX : in.algo == TS_NAN_M4 ? TS_M4 : in.algo;
    const bool nan_task = t.algo == TS_NAN_MINMAX || t.algo == TS_NAN_M4;
    t.ydt = s.y_dtype;
    t.xdt = s.x ? s.x_dtype : TS_NONE;
    t.n_out = in.n_out;
    t.out_offset = in.out_offset;
    t.yf = s.y;
    t.xf = s.x;
    t.nf = s.n;
    t.y = s.y;
    t.x = s.x;
    t.n = s.n;
    t.mode = 0;
    if (s.n <= in.n_out) {
      t.mode = 1;
    } else if (in.algo == TS_MINMAXLTTB) {
      const int64_t npre = in.n_out * in.minmax_ratio;
      if (s.n - 2 <= npre) {
        t.mode = 2;
      } else {
        t.y = (const char *)s.y + esize(s.y_dtype);
        t.x = s.x ? (const char *)s.x + esize(s.x_dtype) : nullptr;
        t.n = s.n - 2;
      }
    }
    int grp = 0;
    if (t.mode == 0) {
      const int64_t es = (int64_t)esize(t.ydt);
      t.nb = in.algo == TS_MINMAX || in.algo == TS_NAN_MINMAX ? in.n_out / 2
             : in.algo == TS_M4 || in.algo == TS_NAN_M4     ? in.n_out / 4
                                                             : in.n_out * in.minmax_ratio / 2;
      // bins averaging fewer than kStageBin elements: LDS-staged chunks
      // (the NaN-aware scan has no staged form)
      t.stage = !nan_task && t.n / t.nb < kStageBin ? 1 : 0;
      const int64_t bin_bytes = t.n / t.nb * es;
      if (!nan_task && !t.x && bin_bytes >= kDirectMinBinBytes && bin_bytes <= kDirectMaxBinBytes) t.stage = 2;
      t.chunk = (t.stage == 1 ? kStageChunk : chunk_bytes) / es;
      grp = nan_task ? 22 + t.ydt : t.stage == 2 ? kBatchDirectGroup + t.ydt : t.ydt + 11 * t.stage;
      t.chunk_begin = p->group_total[grp];
      t.shift = (int64_t)(((uintptr_t)t.y & 15) / (uintptr_t)es);
      t.nchunks = (t.n + t.shift + t.chunk - 1) / t.chunk;
      // workspace regions (sized for the smallest chunk of the tuning space)
      const int64_t nch_max = (t.n + 16 + kMinChunk / es - 1) / (kMinChunk / es);
      if (t.x) {
        t.o_edges = (int64_t)o;
        o = al256(o + 8 * (size_t)(t.nb + 1));
        p->any_x = true;
      }
      t.o_binres = (int64_t)o;
      o = al256(o + 16 * (size_t)t.nb);
      t.o_partL = (int64_t)o;
      o = al256(o + sizeof(Partial) * (size_t)nch_max);
      t.o_partR = (int64_t)o;
      o = al256(o + sizeof(Partial) * (size_t)nch_max);
      t.o_sel = (int64_t)o;
      o = al256(o + 32 * (size_t)t.nb);
      t.o_cnt = (int64_t)o;
      o = al256(o + 8 * (size_t)t.nb);
      p->group_cb[grp].push_back(p->group_total[grp]);
      p->group_tix[grp].push_back((int32_t)ti);
      // a direct task's work items are its bins
      p->group_total[grp] += t.stage == 2 ? t.nb : t.nchunks;
      p->group_bytes[grp] += (double)t.n * (double)es;
      p->total_chunks += t.nchunks;
      p->total_slots += t.nb + 1;
    }
    if (in.algo == TS_MINMAXLTTB && t.mode != 1) {
      t.m_max = t.mode == 0 ? in.n_out * in.minmax_ratio + 2 : s.n;
      if (t.mode == 0) {
        t.o_cand = (int64_t)o;
        o = al256(o + 8 * (size_t)t.m_max);
        t.o_m = (int64_t)o;
        o = al256(o + 8);
      }
      t.o_cx = (int64_t)o;
      o = al256(o + 8 * (size_t)(in.n_out - 2));
      t.o_cy = (int64_t)o;
      o = al256(o + 8 * (size_t)(in.n_out - 2));
      t.o_next = (int64_t)o;
      o = al256(o + 8 * (size_t)t.m_max);
      t.o_entry = (int64_t)o;
      o = al256(o + 4 * (lttb_group_count(in.n_out) + 1));
      if (t.mode == 0) {  // gathered candidate coordinates
        t.o_gx = (int64_t)o;
        o = al256(o + 8 * (size_t)t.m_max);
        t.o_gy = (int64_t)o;
        o = al256(o + 8 * (size_t)t.m_max);
      }
      p->max_m = std::max(p->max_m, t.m_max);
    }
    if (in.algo == TS_MINMAXLTTB) p->lttb_tasks.push_back((int32_t)ti);
    p->tasks.push_back(t);
    ti++;
  }
  // Per-bin groups: longest bins first.  A wavefront reduces a whole bin, so
  // the wavefronts of the longest bins set the group's time; started first,
  // they overlap with the short ones instead of trailing after them.
  for (int g = kBatchDirectGroup; g < kBatchGroups; g++) {
    std::vector<int32_t> &tix = p->group_tix[g];
    if (tix.size() < 2) continue;
    const auto bin_len = [&](int32_t k) { return p->tasks[k].n / p->tasks[k].nb; };
    std::stable_sort(tix.begin(), tix.end(), [&](int32_t a, int32_t b) { return bin_len(a) > bin_len(b); });
    int64_t pos = 0;
    for (size_t i = 0; i < tix.size(); i++) {
      p->group_cb[g][i] = pos;
      p->tasks[tix[i]].chunk_begin = pos;
      pos += p->tasks[tix[i]].nb;
    }
  }
  // Bin slots: tasks whose bins span many chunks first (a wavefront merges
  // each of their bins), then the rest (a thread per bin).
  p->wave_slots = 0;
  int64_t next = 0;
  for (int pass = 0; pass < 2; pass++) {
    for (size_t k = 0; k < p->tasks.size(); k++) {
      BatchTask &t = p->tasks[k];
      if (t.mode != 0) continue;
      const bool lanes = t.stage || t.n / t.nb <= kLaneMergeChunks * t.chunk;
      if (lanes != (pass == 1)) continue;
      t.slot_begin = next;
      next += t.nb + 1;
      for (int64_t b = 0; b < t.nb + 1; b++) p->slot_task.push_back((int32_t)k);
    }
    if (pass == 0) p->wave_slots = next;
  }
  return o;
}

size_t batch_table_bytes(ts_plan *p) {
  const size_t a = al256(sizeof(BatchTask) * p->tasks.size());
  const size_t b = al256(sizeof(int32_t) * p->slot_task.size());
  const size_t c = al256(sizeof(int32_t) * p->lttb_tasks.size());
  size_t need = a + b + c;
  for (int g = 0; g < kBatchGroups; g++) {
    p->group_off_cb[g] = need;
    need += al256(sizeof(int64_t) * p->group_cb[g].size());
    p->group_off_tix[g] = need;
    need += al256(sizeof(int32_t) * p->group_tix[g].size());
  }
  return std::max<size_t>(need, 256);
}

void batch_pack_table(const ts_plan *p, char *h) {
  const size_t a = al256(sizeof(BatchTask) * p->tasks.size());
  const size_t b = al256(sizeof(int32_t) * p->slot_task.size());
  memcpy(h, p->tasks.data(), sizeof(BatchTask) * p->tasks.size());
  memcpy(h + a, p->slot_task.data(), sizeof(int32_t) * p->slot_task.size());
  memcpy(h + a + b, p->lttb_tasks.data(), sizeof(int32_t) * p->lttb_tasks.size());
  for (int g = 0; g < kBatchGroups; g++) {
    memcpy(h + p->group_off_cb[g], p->group_cb[g].data(), sizeof(int64_t) * p->group_cb[g].size());
    memcpy(h + p->group_off_tix[g], p->group_tix[g].data(), sizeof(int32_t) * p->group_tix[g].size());
  }
}

}  // namespace tsds

namespace {

int upload(ts_plan *p) {
  const size_t need = batch_table_bytes(p);
  hipError_t e;
  if (need > p->table_bytes) {
    if (p->d_table) (void)hipFree(p->d_table);
    p->d_table = nullptr;
    if ((e = hipMalloc(&p->d_table, need)) != hipSuccess) return api_fail(TS_ERR_HIP, "plan table allocation failed");
    p->table_bytes = need;
  }
  std::vector<char> h(need, 0);
  batch_pack_table(p, h.data());
  if ((e = hipMemcpy(p->d_table, h.data(), need, hipMemcpyHostToDevice)) != hipSuccess)
    return api_fail(TS_ERR_HIP, "plan table upload failed");
  return TS_OK;
}

BatchArgs args(const ts_plan *p, const void *d_table, int64_t *out, int64_t *counts, void *ws) {
  BatchArgs a;
  const size_t ta = al256(sizeof(BatchTask) * p->tasks.size());
  const size_t tb = al256(sizeof(int32_t) * p->slot_task.size());
  a.tasks = (const BatchTask *)d_table;
  a.slot_task = (const int32_t *)((const char *)d_table + ta);
  a.lttb_tasks = (const int32_t *)((const char *)d_table + ta + tb);
  a.ntasks = (int64_t)p->tasks.size();
  a.total_chunks = p->total_chunks;
  a.total_slots = p->total_slots;
  a.wave_slots = p->wave_slots;
  a.n_lttb = (int64_t)p->lttb_tasks.size();
  a.ws = (char *)ws;
  a.out = out;
  a.counts = counts;
  a.small = p->small;
  a.max_m = p->max_m;
  a.lds_m = kWalkMapLds / 8;
  a.lds_ok = p->max_m <= a.lds_m ? 1 : 0;
  if (a.lds_ok) a.lds_m = std::max<int64_t>(p->max_m, 1);
  return a;
}

}  // namespace

int tsds::batch_enqueue(const ts_plan *p, const void *d_table, int64_t *out, int64_t *counts, void *ws,
                        hipStream_t st, bool fan) {
  const BatchArgs a = args(p, d_table, out, counts, ws);
  hipError_t e;
  if (p->any_x && (e = launch_batch_edges(a, st)) != hipSuccess) return api_fail(TS_ERR_HIP, "batch edges launch failed");
  // Groups by estimated cost, largest first, each onto the stream with the
  // least cost so far (longest-processing-time first).  Cost = the group's
  // bytes weighted by how slowly its kernel moves them: staged groups (many
  // small bins, latency-bound) x4; chunked scans of bytes x3, of 16-bit
  // types x1.5 (measured on the 512-series mix: 0.687 -> 0.640 ms against
  // bytes-only ordering); groups reduced a wavefront per bin by their rates
  // alone on the GPU: bytes x2, 16-bit types x1.15, else x1 (bytes ~2.8,
  // 16-bit ~5.1, wider ~5.9 TB/s).
  auto cost = [p](int g) {
    const bool staged = g < 22 && g / 11 == 1, direct = g >= kBatchDirectGroup;
    const size_t es = esize(g % 11);
    if (direct) return p->group_bytes[g] * (es == 1 ? 2.0 : es == 2 ? 1.15 : 1.0);
    return p->group_bytes[g] * (staged ? 4.0 : es == 1 ? 3.0 : es == 2 ? 1.5 : 1.0);
  };
  std::vector<int> order;
  for (int g = 0; g < kBatchGroups; g++)
    if (p->group_total[g] > 0) order.push_back(g);
  std::stable_sort(order.begin(), order.end(), [&](int u, int v) { return cost(u) > cost(v); });
  const bool use_side = fan && p->side[0] && order.size() > 1;
  int used = 0;
  if (use_side) {
    if ((e = hipEventRecord(p->ev_fork, st)) != hipSuccess) return api_fail(TS_ERR_HIP, "fork event failed");
    used = std::min<int>((int)order.size() - 1, ts_plan::kSide);
    for (int k = 0; k < used; k++)
      if ((e = hipStreamWaitEvent(p->side[k], p->ev_fork, 0)) != hipSuccess)
        return api_fail(TS_ERR_HIP, "fork wait failed");
  }
  std::vector<int> queue_of(order.size(), 0);  // 0: st, q > 0: side[q - 1]
  if (use_side) {
    // LDS-staged groups (many short bins: latency-bound, a fraction of the
    // bandwidth) are enqueued first, one after another on the plan's stream,
    // and run beside the bandwidth-bound groups, which go longest-first onto
    // the side streams (512-series mix: 0.599 -> 0.577 ms against placing
    // every group by cost on all four streams).
    const auto staged = [](int g) { return g < 22 && g / 11 == 1; };
    std::stable_partition(order.begin(), order.end(), staged);
    const bool any_staged = staged(order.front());
    const bool any_other = !staged(order.back());
    const int first = any_staged && any_other ? 1 : 0;
    std::vector<double> load(1 + used, 0.0);
    for (size_t k = 0; k < order.size(); k++) {
      int best = first;
      if (!(first && staged(order[k])))
        for (int q = first + 1; q <= used; q++)
          if (load[q] < load[best]) best = q;
      if (first && staged(order[k])) best = 0;
      queue_of[k] = best;
      load[best] += cost(order[k]);
    }
  }
  // The per-bin byte group is enqueued first on whichever stream it shares:
  // its many short dependent tile chains overlap best with everything else
  // from the start.  512-series mix, two best tunings: these weights with the
  // byte group first 0.551-0.555 ms; the same with it behind the f16 group
  // 0.571-0.578 ms; bytes x4 and 16-bit x1 (the byte group alone on a stream,
  // the two 16-bit groups one after the other) 0.557-0.560 ms.
  {
    std::vector<size_t> li(order.size());
    for (size_t k = 0; k < li.size(); k++) li[k] = k;
    std::stable_partition(li.begin(), li.end(),
                          [&](size_t k) { return order[k] >= kBatchDirectGroup && esize(order[k] % 11) == 1; });
    std::vector<int> o2(order.size()), q2(order.size());
    for (size_t k = 0; k < li.size(); k++) {
      o2[k] = order[li[k]];
      q2[k] = queue_of[li[k]];
    }
    order.swap(o2);
    queue_of.swap(q2);
  }
  for (size_t k = 0; k < order.size(); k++) {
    const int g = order[k];
    BatchGroup bg;
    bg.cb = (const int64_t *)((const char *)d_table + p->group_off_cb[g]);
    bg.tix = (const int32_t *)((const char *)d_table + p->group_off_tix[g]);
    bg.ntasks = (int64_t)p->group_cb[g].size();
    bg.total = p->group_total[g];
    bg.ydt = g % 11;
    bg.nan = g >= 22 && g < kBatchDirectGroup ? 1 : 0;
    bg.stage = g >= kBatchDirectGroup ? 2 : g >= 22 ? 0 : g / 11;
    const hipStream_t s = queue_of[k] > 0 ? p->side[queue_of[k] - 1] : st;
    if ((e = launch_batch_scan(a, bg, p->grid_blocks, s)) != hipSuccess)
      return api_fail(TS_ERR_HIP, "batch scan launch failed");
  }
  for (int k = 0; k < used; k++) {
    if ((e = hipEventRecord(p->ev_join[k], p->side[k])) != hipSuccess) return api_fail(TS_ERR_HIP, "join event failed");
    if ((e = hipStreamWaitEvent(st, p->ev_join[k], 0)) != hipSuccess) return api_fail(TS_ERR_HIP, "join wait failed");
  }
  if ((e = launch_batch_merge(a, st)) != hipSuccess) return api_fail(TS_ERR_HIP, "batch merge launch failed");
  if ((e = launch_batch_compact(a, st)) != hipSuccess) return api_fail(TS_ERR_HIP, "batch compact launch failed");
  if ((e = launch_batch_lttb(a, st)) != hipSuccess) return api_fail(TS_ERR_HIP, "batch lttb launch failed");
  return TS_OK;
}

namespace {

// Side streams and fork/join events of a plan, on the plan's device.
int ensure_side(ts_plan *p) {
  if (p->side[0]) return TS_OK;
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return api_fail(TS_ERR_HIP, "no HIP device");
  if (cur != p->device && hipSetDevice(p->device) != hipSuccess) return api_fail(TS_ERR_HIP, "cannot select the plan's device");
  bool ok = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) == hipSuccess;
  for (int k = 0; ok && k < ts_plan::kSide; k++)
    ok = hipStreamCreateWithFlags(&p->side[k], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&p->ev_join[k], hipEventDisableTiming) == hipSuccess;
  if (cur != p->device) (void)hipSetDevice(cur);
  if (!ok) return api_fail(TS_ERR_HIP, "side stream creation failed");
  return TS_OK;
}

void free_side(ts_plan *p) {
  for (int k = 0; k < ts_plan::kSide; k++) {
    if (p->side[k]) (void)hipStreamDestroy(p->side[k]);
    if (p->ev_join[k]) (void)hipEventDestroy(p->ev_join[k]);
    p->side[k] = nullptr;
    p->ev_join[k] = nullptr;
  }
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  p->ev_fork = nullptr;
}

int enqueue(ts_plan *p, int64_t *out, int64_t *counts, void *ws, hipStream_t st) {
  int rc = ensure_side(p);
  if (rc) return rc;
  return batch_enqueue(p, p->d_table, out, counts, ws, st, true);
}

void drop_graph(ts_plan *p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  p->g_out = p->g_counts = p->g_ws = nullptr;
}

int check_run(const ts_plan *p, const int64_t *out, const int64_t *counts, const void *ws, size_t ws_bytes) {
  if (!p) return api_fail(TS_ERR_NULL, "plan is NULL");
  if (!counts || (!out && p->out_needed > 0)) return api_fail(TS_ERR_NULL, "out_idx / counts is NULL");
  if (p->ws_bytes > 0) {
    if (!ws) return api_fail(TS_ERR_WORKSPACE, "workspace is NULL");
    if ((uintptr_t)ws % 256) return api_fail(TS_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    if (ws_bytes < p->ws_bytes) return api_fail(TS_ERR_WORKSPACE, "workspace smaller than ts_batch_workspace_bytes");
  }
  return TS_OK;
}

std::string signature(const ts_plan *p) {
  // dtype / algo / size-class histogram of the batch
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    h ^= v;
    h *= 1099511628211ull;
  };
  for (const ts_task &t : p->in) {
    int64_t lg = 0;
    while ((1ll << lg) < t.series.n) lg++;
    mix((uint64_t)t.algo);
    mix((uint64_t)(t.series.y_dtype + 16));
    mix((uint64_t)lg);
    mix((uint64_t)(t.series.x != nullptr));
  }
  char buf[64];
  snprintf(buf, sizeof buf, "%016llx-%zu", (unsigned long long)h, p->in.size());
  return buf;
}

}  // namespace

int tsds::batch_check_task(const ts_task &t) {
  int rc;
  if (t.algo != TS_MINMAX && t.algo != TS_M4 && t.algo != TS_MINMAXLTTB && t.algo != TS_NAN_MINMAX &&
      t.algo != TS_NAN_M4)
    return api_fail(TS_ERR_ARG, "batched tasks are MinMax, M4, MinMaxLTTB or their NaN-aware MinMax / M4");
  if ((rc = api_check_series(&t.series)) || (rc = api_check_nout(t.algo, t.n_out, t.minmax_ratio))) return rc;
  if (t.algo == TS_MINMAXLTTB && t.minmax_ratio > 30)
    return api_fail(TS_ERR_ARG, "batched MinMaxLTTB needs minmax_ratio <= 30");
  if (t.out_offset < 0) return api_fail(TS_ERR_ARG, "out_offset < 0");
  return TS_OK;
}

extern "C" {

int ts_batch_plan(const ts_task *tasks, int64_t n_tasks, ts_plan **out_plan) {
  if (!out_plan) return api_fail(TS_ERR_NULL, "out_plan is NULL");
  *out_plan = nullptr;
  if (n_tasks < 0 || n_tasks > (1 << 24)) return api_fail(TS_ERR_ARG, "n_tasks out of range");
  if (n_tasks > 0 && !tasks) return api_fail(TS_ERR_NULL, "tasks is NULL");
  ts_plan *p = new ts_plan();
  for (int64_t i = 0; i < n_tasks; i++) {
    const ts_task &t = tasks[i];
    int rc;
    if ((rc = batch_check_task(t))) {
      delete p;
      return rc;
    }
    p->out_needed = std::max(p->out_needed, t.out_offset + t.n_out);
    p->in.push_back(t);
  }
  int cus = 256;
  if (hipGetDevice(&p->device) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess) {
    delete p;
    return api_fail(TS_ERR_HIP, "no HIP device");
  }
  p->grid_blocks = (int64_t)cus * 16;
  p->ws_bytes = batch_layout(p, kMinChunk);        // largest chunk count of the tuning space
  batch_layout(p, p->chunk_bytes);
  int rc = upload(p);
  if (rc) {
    if (p->d_table) (void)hipFree(p->d_table);
    delete p;
    return rc;
  }
  *out_plan = p;
  return TS_OK;
}

size_t ts_batch_workspace_bytes(const ts_plan *p) { return p ? p->ws_bytes : 0; }

int64_t ts_batch_out_size(const ts_plan *p) { return p ? p->out_needed : 0; }

int ts_batch_set_tuning(ts_plan *p, int64_t chunk_bytes, int32_t small_bin, int64_t grid_blocks) {
  if (!p) return api_fail(TS_ERR_NULL, "plan is NULL");
  if (chunk_bytes < kMinChunk || chunk_bytes > (1 << 22) || (chunk_bytes & (chunk_bytes - 1)))
    return api_fail(TS_ERR_ARG, "chunk_bytes must be a power of two in [4096, 4 MiB]");
  if (small_bin < 1) return api_fail(TS_ERR_ARG, "small_bin must be >= 1");
  if (grid_blocks < 1) return api_fail(TS_ERR_ARG, "grid_blocks must be >= 1");
  p->chunk_bytes = chunk_bytes;
  p->small = small_bin;
  p->grid_blocks = grid_blocks;
  batch_layout(p, chunk_bytes);
  drop_graph(p);
  return upload(p);
}

int ts_batch_get_tuning(const ts_plan *p, int64_t *chunk_bytes, int32_t *small_bin, int64_t *grid_blocks) {
  if (!p || !chunk_bytes || !small_bin || !grid_blocks) return api_fail(TS_ERR_NULL, "NULL argument");
  *chunk_bytes = p->chunk_bytes;
  *small_bin = p->small;
  *grid_blocks = p->grid_blocks;
  return TS_OK;
}

int ts_batch_run(ts_plan *p, int64_t *out_idx, int64_t *counts, void *ws, size_t ws_bytes, void *stream,
                 int use_graph) {
  int rc;
  if ((rc = check_run(p, out_idx, counts, ws, ws_bytes))) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (!use_graph) return enqueue(p, out_idx, counts, ws, st);
  if (!p->exec || p->g_out != out_idx || p->g_counts != counts || p->g_ws != ws) {
    drop_graph(p);
    hipError_t e;
    if (!p->cap_stream && (e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking)) != hipSuccess)
      return api_fail(TS_ERR_HIP, "capture stream creation failed");
    if ((rc = ensure_side(p))) return rc;  // streams and events exist before the capture starts
    if ((e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return api_fail(TS_ERR_HIP, "graph capture failed to start");
    rc = enqueue(p, out_idx, counts, ws, p->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->cap_stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return api_fail(TS_ERR_HIP, "graph capture failed");
    p->graph = g;
    if ((e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
      drop_graph(p);
      return api_fail(TS_ERR_HIP, "graph instantiation failed");
    }
    p->g_out = out_idx;
    p->g_counts = counts;
    p->g_ws = ws;
  }
  hipError_t e = hipGraphLaunch(p->exec, st);
  if (e != hipSuccess) return api_fail(TS_ERR_HIP, "graph launch failed");
  return TS_OK;
}

// Times each (chunk, small-bin threshold, grid) candidate on the caller's
// buffers and keeps the fastest.  With a cache path, results are stored per
// batch signature (dtype / algorithm / size-class mix) and reused.
int ts_batch_autotune(ts_plan *p, int64_t *out_idx, int64_t *counts, void *ws, size_t ws_bytes, void *stream,
                      const char *cache_path) {
  int rc;
  if ((rc = check_run(p, out_idx, counts, ws, ws_bytes))) return rc;
  const std::string sig = signature(p);
  if (cache_path) {
    FILE *f = fopen(cache_path, "r");
    if (f) {
      char key[128];
      long long cb, gb;
      int sm;
      while (fscanf(f, "%127s %lld %d %lld", key, &cb, &sm, &gb) == 4) {
        if (sig == key) {
          fclose(f);
          return ts_batch_set_tuning(p, cb, sm, gb);
        }
      }
      fclose(f);
    }
  }
  hipStream_t st = (hipStream_t)stream;
  int cus = 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess)
    return api_fail(TS_ERR_HIP, "device query failed");
  const int64_t chunks[] = {16384, 32768, 65536};
  const int32_t smalls[] = {32, 128, 512};
  const int64_t grids[] = {(int64_t)cus * 4, (int64_t)cus * 8, (int64_t)cus * 16};
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return api_fail(TS_ERR_HIP, "event creation failed");
  float best = 1e30f;
  int64_t bc = p->chunk_bytes, bg = p->grid_blocks;
  int32_t bs = p->small;
  for (int64_t cb : chunks)
    for (int32_t sm : smalls)
      for (int64_t gb : grids) {
        if ((rc = ts_batch_set_tuning(p, cb, sm, gb))) break;
        if ((rc = enqueue(p, out_idx, counts, ws, st))) break;  // warm-up
        if (hipEventRecord(a, st) != hipSuccess) { rc = api_fail(TS_ERR_HIP, "event record failed"); break; }
        for (int r = 0; r < 3 && !rc; r++) rc = enqueue(p, out_idx, counts, ws, st);
        if (rc) break;
        float ms = 0;
        if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
            hipEventElapsedTime(&ms, a, b) != hipSuccess) {
          rc = api_fail(TS_ERR_HIP, "event timing failed");
          break;
        }
        if (ms < best) {
          best = ms;
          bc = cb;
          bs = sm;
          bg = gb;
        }
      }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc) return rc;
  if ((rc = ts_batch_set_tuning(p, bc, bs, bg))) return rc;
  if (cache_path) {
    FILE *f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "%s %lld %d %lld\n", sig.c_str(), (long long)bc, bs, (long long)bg);
      fclose(f);
    }
  }
  return TS_OK;
}

void ts_plan_free(ts_plan *p) {
  if (!p) return;
  drop_graph(p);
  free_side(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->d_table) (void)hipFree(p->d_table);
  delete p;
}

}  // extern "C"

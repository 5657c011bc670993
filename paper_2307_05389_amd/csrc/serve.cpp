// serve.cpp -- serving engine for zoom/pan downsampling requests over series
// kept resident in HBM (the interactive use the paper motivates in Sec. 1:
// downsampling on every zoom or pan of a large chart).
//
// One scheduler thread drives S slots, each with its own HIP stream, device
// arena (workspace, outputs, task table) and pinned host buffers:
//   FREE       -> take the oldest pending requests that fit the slot (at most
//                 max_batch, and their worst-case workspace within the arena),
//                 resolve their x-windows on the device (one search kernel),
//                 copy the [i0, i1) pairs back            -> RESOLVING
//   RESOLVING  -> when the ranges have arrived: one MinMaxLTTB task per
//                 request on its window, laid out as one batch (persistent
//                 scan, merge, candidates, LTTB), results copied back
//                                                          -> RUNNING
//   RUNNING    -> when done: results handed to poll()      -> FREE
// Requests that arrive while other batches are on the GPU are admitted as soon
// as a slot is free, so several batches overlap on the device (continuous
// batching).  Every request's arithmetic is the same as a single
// ts_minmaxlttb call on its window, whatever batch it lands in.
// A batch of one request runs the single-series kernels (ts_minmaxlttb on its
// window), which take fewer launches than the batched chain; larger batches
// run as one batch.
// Plain mode (cfg.plain = 1) runs each request alone, in arrival order, with
// the single-series ts_window + ts_minmaxlttb calls: the comparison baseline.
// Requests still pending can be cancelled (ts_server_cancel) and expire after
// cfg.timeout_s; both come back from poll() with an error status and no
// indices.  The scheduler's phases are marked as roctx ranges for profilers.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "batch_host.hpp"
#include "internal.hpp"
#include "tsds.h"

using namespace tsds;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
  int64_t id;
  int32_t series;
  int64_t xa, xb, n_out;
  double t_submit;
};

struct Res {
  int64_t id;
  int32_t series;
  int32_t status;
  int64_t i0, i1;
  double t_submit, t_done, t_admit, t_run;
  int32_t batch;
  std::vector<int64_t> idx;
};

enum { FREE = 0, RESOLVING = 1, RUNNING = 2 };

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev_ranges = nullptr, ev_done = nullptr;
  int64_t *d_ranges = nullptr, *d_out = nullptr, *d_counts = nullptr;
  void *d_table = nullptr, *ws = nullptr;
  size_t table_cap = 0, ws_cap = 0;
  int64_t *h_ranges = nullptr, *h_out = nullptr, *h_counts = nullptr;
  char *h_table = nullptr;
  // device-side addresses of the host buffers
  int64_t *m_ranges = nullptr, *m_out = nullptr, *m_counts = nullptr;
  char *m_table = nullptr;
  ts_plan plan;
  std::vector<Req> batch;
  int state = FREE;
  double t_admit = 0.0, t_run = 0.0;
};

}  // namespace

struct ts_server {
  std::vector<ts_series> series;
  ts_server_config cfg;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req> pending;
  std::deque<Res> done;
  std::thread worker;
  bool stop = false;
  int64_t next_id = 0;
  int64_t batches = 0, max_batch_seen = 0, requests_done = 0, requests_dropped = 0;
  int device = 0;
  int error = 0;
  size_t ws_per_request_max = 0;
  std::vector<size_t> ws_series;  // worst-case workspace of one request per series
  int64_t grid_blocks = 1536;
};

namespace {

// Worst-case workspace of one MinMaxLTTB request on a window of up to n points.
size_t request_ws(ts_series s, int64_t n_out, int64_t ratio) {
  ts_plan p;
  ts_task t;
  memset(&t, 0, sizeof t);
  t.algo = TS_MINMAXLTTB;
  t.series = s;
  t.n_out = n_out;
  t.minmax_ratio = ratio;
  p.in.push_back(t);
  return batch_layout(&p, 4096);
}

int alloc_slot(ts_server *sv, Slot &sl) {
  const int64_t mb = sv->cfg.max_batch;
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t r) {
    if (r != hipSuccess && e == hipSuccess) e = r;
  };
  ok(hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking));
  ok(hipEventCreateWithFlags(&sl.ev_ranges, hipEventDisableTiming));
  ok(hipEventCreateWithFlags(&sl.ev_done, hipEventDisableTiming));
  ok(hipMalloc((void **)&sl.d_ranges, sizeof(int64_t) * 2 * mb));
  ok(hipMalloc((void **)&sl.d_out, sizeof(int64_t) * mb * sv->cfg.max_nout));
  ok(hipMalloc((void **)&sl.d_counts, sizeof(int64_t) * mb));
  // table: tasks + bin slots + lists, for max_batch worst-case requests
  const int64_t nb = sv->cfg.max_nout * sv->cfg.minmax_ratio / 2 + 1;
  sl.table_cap = 256 * 40 + sizeof(BatchTask) * mb + sizeof(int32_t) * mb * nb + 16 * mb;
  ok(hipMalloc(&sl.d_table, sl.table_cap));
  sl.ws_cap = std::max<size_t>(sv->cfg.arena_bytes, 256);
  ok(hipMalloc(&sl.ws, sl.ws_cap));
  // host buffers: pinned, mapped and coherent; kernels read and write them
  // directly (see launch_copy_bytes)
  ok(hipHostMalloc((void **)&sl.h_ranges, sizeof(int64_t) * 2 * mb, hipHostMallocCoherent));
  ok(hipHostMalloc((void **)&sl.h_out, sizeof(int64_t) * mb * sv->cfg.max_nout, hipHostMallocCoherent));
  ok(hipHostMalloc((void **)&sl.h_counts, sizeof(int64_t) * mb, hipHostMallocCoherent));
  ok(hipHostMalloc((void **)&sl.h_table, sl.table_cap, hipHostMallocCoherent));
  if (e == hipSuccess) {
    ok(hipHostGetDevicePointer((void **)&sl.m_ranges, sl.h_ranges, 0));
    ok(hipHostGetDevicePointer((void **)&sl.m_out, sl.h_out, 0));
    ok(hipHostGetDevicePointer((void **)&sl.m_counts, sl.h_counts, 0));
    ok(hipHostGetDevicePointer((void **)&sl.m_table, sl.h_table, 0));
  }
  return e == hipSuccess ? TS_OK : api_fail(TS_ERR_HIP, "server slot allocation failed");
}

void free_slot(Slot &sl) {
  if (sl.st) (void)hipStreamSynchronize(sl.st);
  if (sl.ev_ranges) (void)hipEventDestroy(sl.ev_ranges);
  if (sl.ev_done) (void)hipEventDestroy(sl.ev_done);
  for (void *p : {(void *)sl.d_ranges, (void *)sl.d_out, (void *)sl.d_counts, sl.d_table, sl.ws})
    if (p) (void)hipFree(p);
  for (void *p : {(void *)sl.h_ranges, (void *)sl.h_out, (void *)sl.h_counts, (void *)sl.h_table})
    if (p) (void)hipHostFree(p);
  if (sl.st) (void)hipStreamDestroy(sl.st);
}

// FREE -> RESOLVING: window search for the slot's batch.
int start_batch(ts_server *sv, Slot &sl) {
  sl.t_admit = now_s();
  WindowBatch wb;
  memset(&wb, 0, sizeof wb);
  wb.count = (int32_t)sl.batch.size();
  wb.ranges = sl.d_ranges;
  wb.host_ranges = sl.m_ranges;
  for (int i = 0; i < wb.count; i++) {
    const ts_series &s = sv->series[sl.batch[i].series];
    wb.x[i] = s.x;
    wb.n[i] = s.n;
    wb.xa[i] = sl.batch[i].xa;
    wb.xb[i] = sl.batch[i].xb;
    wb.xdt[i] = s.x_dtype;
  }
  if (launch_windows(wb, sl.st) != hipSuccess) return TS_ERR_HIP;
  if (hipEventRecord(sl.ev_ranges, sl.st) != hipSuccess) return TS_ERR_HIP;
  sl.state = RESOLVING;
  return TS_OK;
}

// Sub-series of request i on its resolved window.
ts_series window_series(const ts_server *sv, const Slot &sl, int i) {
  ts_series s = sv->series[sl.batch[i].series];
  const int64_t i0 = sl.h_ranges[2 * i], i1 = std::max(sl.h_ranges[2 * i + 1], i0);
  const size_t ex = elem_size(s.x_dtype), ey = elem_size(s.y_dtype);
  s.x = (const char *)s.x + ex * (size_t)i0;
  s.y = (const char *)s.y + ey * (size_t)i0;
  s.n = i1 - i0;
  if (s.n == 0) {
    s.x = nullptr;
    s.x_dtype = TS_NONE;
    s.y = nullptr;
  }
  return s;
}

// RESOLVING -> RUNNING: downsampling of every request on its window.
int run_batch(ts_server *sv, Slot &sl) {
  sl.t_run = now_s();
  const int nb = (int)sl.batch.size();
  const int64_t mo = sv->cfg.max_nout;
  if (sv->cfg.plain || nb == 1) {
    for (int i = 0; i < nb; i++) {
      const ts_series s = window_series(sv, sl, i);
      int rc = ts_minmaxlttb(&s, sl.batch[i].n_out, sv->cfg.minmax_ratio, sl.d_out + i * mo, sl.d_counts + i, sl.ws,
                             sl.ws_cap, sl.st);
      if (rc) return rc;
    }
  } else {
    sl.plan.in.clear();
    for (int i = 0; i < nb; i++) {
      ts_task t;
      memset(&t, 0, sizeof t);
      t.algo = TS_MINMAXLTTB;
      t.series = window_series(sv, sl, i);
      t.n_out = sl.batch[i].n_out;
      t.minmax_ratio = sv->cfg.minmax_ratio;
      t.out_offset = i * mo;
      sl.plan.in.push_back(t);
    }
    const size_t need = batch_layout(&sl.plan, sl.plan.chunk_bytes);
    const size_t tb = batch_table_bytes(&sl.plan);
    if (need > sl.ws_cap || tb > sl.table_cap) return api_fail(TS_ERR_WORKSPACE, "batch exceeds the slot arena");
    batch_pack_table(&sl.plan, sl.h_table);
    if (launch_copy_bytes(sl.d_table, sl.m_table, tb, sl.st) != hipSuccess) return TS_ERR_HIP;
    int rc = batch_enqueue(&sl.plan, sl.d_table, sl.d_out, sl.d_counts, sl.ws, sl.st);
    if (rc) return rc;
  }
  if (launch_export_rows(sl.d_counts, sl.d_out, mo, nb, sl.m_counts, sl.m_out, sl.st) != hipSuccess ||
      hipEventRecord(sl.ev_done, sl.st) != hipSuccess)
    return TS_ERR_HIP;
  sl.state = RUNNING;
  return TS_OK;
}

// RUNNING -> FREE: results (indices into the full series) to the done queue.
void finish_batch(ts_server *sv, Slot &sl) {
  const double t = now_s();
  const int nb = (int)sl.batch.size();
  std::vector<Res> out;
  for (int i = 0; i < nb; i++) {
    Res r;
    r.id = sl.batch[i].id;
    r.series = sl.batch[i].series;
    r.status = 0;
    r.i0 = sl.h_ranges[2 * i];
    r.i1 = std::max(sl.h_ranges[2 * i + 1], r.i0);
    r.t_submit = sl.batch[i].t_submit;
    r.t_done = t;
    r.t_admit = sl.t_admit;
    r.t_run = sl.t_run;
    r.batch = nb;
    const int64_t c = sl.h_counts[i];
    const int64_t *src = sl.h_out + i * sv->cfg.max_nout;
    r.idx.resize((size_t)std::max<int64_t>(c, 0));
    for (int64_t k = 0; k < c; k++) r.idx[k] = src[k] + r.i0;
    out.push_back(std::move(r));
  }
  std::lock_guard<std::mutex> g(sv->mu);
  for (auto &r : out) sv->done.push_back(std::move(r));
  sv->batches++;
  sv->max_batch_seen = std::max<int64_t>(sv->max_batch_seen, nb);
  sv->requests_done += nb;
  sl.batch.clear();
  sl.state = FREE;
}

void fail_batch(ts_server *sv, Slot &sl, int rc) {
  (void)hipStreamSynchronize(sl.st);
  std::lock_guard<std::mutex> g(sv->mu);
  for (const Req &q : sl.batch) {
    Res r;
    r.id = q.id;
    r.series = q.series;
    r.status = rc;
    r.i0 = r.i1 = 0;
    r.t_submit = q.t_submit;
    r.t_done = now_s();
    r.t_admit = sl.t_admit;
    r.t_run = sl.t_run;
    r.batch = (int32_t)sl.batch.size();
    sv->done.push_back(std::move(r));
  }
  sv->error = rc;
  sl.batch.clear();
  sl.state = FREE;
}

// A request that never ran: its result carries `status` and no indices.
// Caller holds sv->mu.
void drop_request(ts_server *sv, const Req &q, int status) {
  Res r;
  r.id = q.id;
  r.series = q.series;
  r.status = status;
  r.i0 = r.i1 = 0;
  r.t_submit = q.t_submit;
  r.t_done = now_s();
  r.t_admit = r.t_run = 0.0;
  r.batch = 0;
  sv->done.push_back(std::move(r));
  sv->requests_dropped++;
}

void worker(ts_server *sv) {
  (void)hipSetDevice(sv->device);
  for (;;) {
    bool progressed = false;
    for (Slot &sl : sv->slots) {
      if (sl.state == RESOLVING && hipEventQuery(sl.ev_ranges) == hipSuccess) {
        roctxRangePushA("tsds.serve.run");
        int rc = run_batch(sv, sl);
        if (rc) fail_batch(sv, sl, rc);
        roctxRangePop();
        progressed = true;
      } else if (sl.state == RUNNING && hipEventQuery(sl.ev_done) == hipSuccess) {
        roctxRangePushA("tsds.serve.finish");
        finish_batch(sv, sl);
        roctxRangePop();
        progressed = true;
      }
    }
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      // expiry: pending requests are in submission order, so the expired
      // ones are at the front
      if (sv->cfg.timeout_s > 0.0) {
        const double t = now_s();
        while (!sv->pending.empty() && t - sv->pending.front().t_submit > sv->cfg.timeout_s) {
          drop_request(sv, sv->pending.front(), TS_ERR_TIMEOUT);
          sv->pending.pop_front();
          progressed = true;
        }
      }
      bool busy = false;
      for (Slot &sl : sv->slots) busy |= sl.state != FREE;
      if (sv->stop && sv->pending.empty() && !busy) break;
      for (Slot &sl : sv->slots) {
        if (sl.state != FREE || sv->pending.empty()) continue;
        // admission: oldest first, at most max_batch, worst-case workspace
        // of the admitted requests within the slot arena
        size_t mem = 0;
        while (!sv->pending.empty() && (int64_t)sl.batch.size() < sv->cfg.max_batch) {
          const Req &q = sv->pending.front();
          const size_t need = sv->ws_series[q.series];
          if (!sl.batch.empty() && mem + need > sl.ws_cap) break;
          mem += need;
          sl.batch.push_back(q);
          sv->pending.pop_front();
          if (sv->cfg.plain) break;
        }
        lk.unlock();
        roctxRangePushA("tsds.serve.admit");
        int rc = start_batch(sv, sl);
        if (rc) fail_batch(sv, sl, rc);
        roctxRangePop();
        lk.lock();
        progressed = true;
      }
      if (!progressed) {
        bool any_busy = false;
        for (Slot &sl : sv->slots) any_busy |= sl.state != FREE;
        if (any_busy) {
          lk.unlock();
          std::this_thread::yield();
        } else {
          sv->cv.wait_for(lk, std::chrono::microseconds(200));
        }
      }
    }
  }
}

}  // namespace

extern "C" {

double ts_server_now(void) { return now_s(); }

int ts_server_create(const ts_series *series, int32_t n_series, const ts_server_config *cfg, ts_server **out) {
  if (!out || !cfg) return api_fail(TS_ERR_NULL, "NULL argument");
  *out = nullptr;
  if (n_series < 1 || !series) return api_fail(TS_ERR_ARG, "need at least one series");
  if (cfg->n_streams < 1 || cfg->n_streams > 16) return api_fail(TS_ERR_ARG, "n_streams must be 1..16");
  if (cfg->max_batch < 1 || cfg->max_batch > kMaxWindows) return api_fail(TS_ERR_ARG, "max_batch must be 1..32");
  if (cfg->max_nout < 3 || cfg->minmax_ratio < 1 || cfg->minmax_ratio > 30)
    return api_fail(TS_ERR_ARG, "bad max_nout / minmax_ratio");
  if (!(cfg->timeout_s >= 0.0)) return api_fail(TS_ERR_ARG, "timeout_s must be >= 0");
  ts_server *sv = new ts_server();
  sv->cfg = *cfg;
  if (sv->cfg.plain) {
    sv->cfg.n_streams = 1;
    sv->cfg.max_batch = 1;
  }
  for (int i = 0; i < n_series; i++) {
    int rc = api_check_series(&series[i]);
    if (!rc && (!series[i].x || series[i].x_dtype == TS_F32 || series[i].x_dtype == TS_F64))
      rc = api_fail(TS_ERR_DTYPE, "served series need integer x");
    if (rc) {
      delete sv;
      return rc;
    }
    sv->series.push_back(series[i]);
    // worst case over windows: the whole series at the largest n_out, for the
    // batched layout and for the single-series call of plain mode
    size_t w = request_ws(series[i], sv->cfg.max_nout, sv->cfg.minmax_ratio);
    w = std::max(w, ts_workspace_bytes(TS_MINMAXLTTB, &series[i], sv->cfg.max_nout, sv->cfg.minmax_ratio));
    sv->ws_series.push_back(w);
    sv->ws_per_request_max = std::max(sv->ws_per_request_max, w);
  }
  // default arena: max_batch worst-case requests; never below one
  if (sv->cfg.arena_bytes == 0) sv->cfg.arena_bytes = sv->ws_per_request_max * (size_t)sv->cfg.max_batch;
  if (sv->cfg.arena_bytes < sv->ws_per_request_max) sv->cfg.arena_bytes = sv->ws_per_request_max;
  int cus = 256;
  if (hipGetDevice(&sv->device) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, sv->device) != hipSuccess) {
    delete sv;
    return api_fail(TS_ERR_HIP, "no HIP device");
  }
  sv->grid_blocks = (int64_t)cus * 6;
  sv->slots.resize(sv->cfg.n_streams);
  // latency over throughput: short chunks (more wavefronts on small windows)
  // and a grid that leaves room for the other slots' kernels
  for (Slot &sl : sv->slots) {
    sl.plan.grid_blocks = sv->grid_blocks;
    sl.plan.chunk_bytes = 16384;
  }
  for (Slot &sl : sv->slots) {
    int rc = alloc_slot(sv, sl);
    if (rc) {
      for (Slot &s2 : sv->slots) free_slot(s2);
      delete sv;
      return rc;
    }
  }
  sv->worker = std::thread(worker, sv);
  *out = sv;
  return TS_OK;
}

int ts_server_submit(ts_server *sv, int32_t series, int64_t xa, int64_t xb, int64_t n_out, int64_t *req_id) {
  if (!sv) return api_fail(TS_ERR_NULL, "server is NULL");
  if (series < 0 || series >= (int32_t)sv->series.size()) return api_fail(TS_ERR_ARG, "no such series");
  if (n_out < 3 || n_out > sv->cfg.max_nout || (n_out * sv->cfg.minmax_ratio) % 2)
    return api_fail(TS_ERR_ARG, "n_out out of range for this server");
  Req q;
  q.series = series;
  q.xa = xa;
  q.xb = xb;
  q.n_out = n_out;
  q.t_submit = now_s();
  {
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->stop) return api_fail(TS_ERR_ARG, "server is stopping");
    q.id = sv->next_id++;
    sv->pending.push_back(q);
  }
  sv->cv.notify_one();
  if (req_id) *req_id = q.id;
  return TS_OK;
}

int ts_server_cancel(ts_server *sv, int64_t req_id) {
  if (!sv) return api_fail(TS_ERR_NULL, "server is NULL");
  std::lock_guard<std::mutex> g(sv->mu);
  for (auto it = sv->pending.begin(); it != sv->pending.end(); ++it) {
    if (it->id != req_id) continue;
    drop_request(sv, *it, TS_ERR_CANCELLED);
    sv->pending.erase(it);
    return TS_OK;
  }
  return api_fail(TS_ERR_ARG, "request is not pending (unknown, already admitted, or finished)");
}

int ts_server_poll(ts_server *sv, ts_result *res, int32_t max_results, int64_t *idx, int64_t idx_cap,
                   int32_t *n_results) {
  if (!sv || !res || !n_results || (!idx && idx_cap > 0)) return api_fail(TS_ERR_NULL, "NULL argument");
  std::lock_guard<std::mutex> g(sv->mu);
  int32_t k = 0;
  int64_t used = 0;
  while (k < max_results && !sv->done.empty()) {
    Res &r = sv->done.front();
    if (used + (int64_t)r.idx.size() > idx_cap) break;
    ts_result &o = res[k];
    o.id = r.id;
    o.series = r.series;
    o.status = r.status;
    o.count = (int64_t)r.idx.size();
    o.offset = used;
    o.i0 = r.i0;
    o.i1 = r.i1;
    o.t_submit = r.t_submit;
    o.t_done = r.t_done;
    o.batch_size = r.batch;
    o.t_admit = r.t_admit;
    o.t_run = r.t_run;
    if (!r.idx.empty()) memcpy(idx + used, r.idx.data(), sizeof(int64_t) * r.idx.size());
    used += (int64_t)r.idx.size();
    sv->done.pop_front();
    k++;
  }
  *n_results = k;
  return TS_OK;
}

int ts_server_stats(ts_server *sv, int64_t *batches, int64_t *max_batch, int64_t *requests_done, int64_t *pending) {
  if (!sv) return api_fail(TS_ERR_NULL, "server is NULL");
  std::lock_guard<std::mutex> g(sv->mu);
  if (batches) *batches = sv->batches;
  if (max_batch) *max_batch = sv->max_batch_seen;
  if (requests_done) *requests_done = sv->requests_done;
  if (pending) *pending = (int64_t)sv->pending.size();
  return sv->error;
}

void ts_server_free(ts_server *sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_one();
  if (sv->worker.joinable()) sv->worker.join();
  for (Slot &sl : sv->slots) free_slot(sl);
  delete sv;
}

}  // extern "C"

// batch.hip -- batched MinMax / M4 / MinMaxLTTB-preselection over hundreds
// of series of uneven length, dtype and n_out in one pass.
//
// The host plan (api_batch.cpp) lays every series out as a run of equal-byte
// chunks in one global work list (per-task offset table `chunk_begin`) and
// one global list of bin slots (`slot_begin`, nb + 1 slots per task).
//   k_batch_edges   one wavefront per bin slot of every task with x.
//   k_batch_scan    persistent: a fixed grid of wavefronts, each taking one
//                   contiguous range of the global work list and walking the
//                   task table as it crosses series boundaries; each item is
//                   the same per-chunk reduction as the single-series scan.
//   k_batch_merge   one wavefront per bin slot: merge + per-bin selection.
//   k_batch_compact one workgroup per task: scan of the per-bin counts and
//                   the compacted output (or MinMaxLTTB candidates).
// Results are identical to one plain call per series: every per-bin merge is
// order-independent and the per-task arithmetic is the same code.
#include "common.hpp"
#include "internal.hpp"
#include "scan_core.hpp"

namespace tsds {

__device__ inline ScanParams task_scan_params(const BatchArgs &a, const BatchTask &t, int32_t small) {
  ScanParams sp;
  sp.y = t.y;
  sp.n = t.n;
  sp.shift = t.shift;
  sp.chunk = t.chunk;
  sp.nchunks = t.nchunks;
  sp.edges = t.x ? (const int64_t *)(a.ws + t.o_edges) : nullptr;
  sp.nb = t.nb;
  sp.binres = (int64_t *)(a.ws + t.o_binres);
  sp.partL = (Partial *)(a.ws + t.o_partL);
  sp.partR = (Partial *)(a.ws + t.o_partR);
  sp.small = small;
  sp.variant = 3;
  return sp;
}

template <typename X>
__device__ inline int64_t task_edge(const BatchTask &t, int64_t b, int lane) {
  return edge_start<X>((const X *)t.x, t.n, t.nb, b, lane);
}

__global__ __launch_bounds__(256) void k_batch_edges(BatchArgs a) {
  const int lane = lane_id();
  const int64_t slot = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (slot >= a.total_slots) return;
  const BatchTask &t = a.tasks[a.slot_task[slot]];
  if (!t.x || t.mode != 0) return;
  const int64_t b = slot - t.slot_begin;
  int64_t s = 0;
  switch (t.xdt) {
    case TS_I32: s = task_edge<int32_t>(t, b, lane); break;
    case TS_I64: s = task_edge<int64_t>(t, b, lane); break;
    case TS_U32: s = task_edge<uint32_t>(t, b, lane); break;
    case TS_U64: s = task_edge<uint64_t>(t, b, lane); break;
    case TS_F32: s = task_edge<float>(t, b, lane); break;
    case TS_F64: s = task_edge<double>(t, b, lane); break;
  }
  if (lane == 0) ((int64_t *)(a.ws + t.o_edges))[b] = s;
}

hipError_t launch_batch_edges(const BatchArgs &a, hipStream_t st) {
  if (a.total_slots == 0) return hipSuccess;
  k_batch_edges<<<dim3((unsigned)((a.total_slots + 3) / 4)), dim3(256), 0, st>>>(a);
  return hipGetLastError();
}

// Last task whose chunk_begin <= item (tasks without chunks share starts).
__device__ int64_t task_of_item(const BatchArgs &a, int64_t item, int lane) {
  int64_t lo = 0, hi = a.ntasks;  // tasks[lo].chunk_begin <= item < tasks[hi].chunk_begin
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t q = lo + (int64_t)lane * step;
    const bool le = q < hi && a.tasks[q].chunk_begin <= item;
    const int cnt = __builtin_popcountll(ballot(le));
    const int64_t nlo = lo + (int64_t)(cnt - 1) * step;
    const int64_t nhi = lo + (int64_t)cnt * step;
    lo = nlo;
    hi = nhi < hi ? nhi : hi;
  }
  while (lo + 1 < a.ntasks && a.tasks[lo + 1].chunk_begin <= item) lo++;
  return lo;
}

__global__ __launch_bounds__(256) void k_batch_scan(BatchArgs a) {
  const int lane = lane_id();
  const int64_t W = (int64_t)gridDim.x * 4;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t i0 = a.total_chunks * w / W, i1 = a.total_chunks * (w + 1) / W;
  if (i0 >= i1) return;
  int64_t t = task_of_item(a, i0, lane);
  for (int64_t item = i0; item < i1; item++) {
    while (t + 1 < a.ntasks && a.tasks[t + 1].chunk_begin <= item) t++;
    const BatchTask &tk = a.tasks[t];
    const ScanParams sp = task_scan_params(a, tk, a.small);
    const int64_t c = item - tk.chunk_begin;
    switch (tk.ydt) {
      case TS_I8: scan_chunk<int8_t, 2, 2>(sp, c, lane); break;
      case TS_I16: scan_chunk<int16_t, 2, 2>(sp, c, lane); break;
      case TS_I32: scan_chunk<int32_t, 2, 2>(sp, c, lane); break;
      case TS_I64: scan_chunk<int64_t, 2, 2>(sp, c, lane); break;
      case TS_U8: scan_chunk<uint8_t, 2, 2>(sp, c, lane); break;
      case TS_U16: scan_chunk<uint16_t, 2, 2>(sp, c, lane); break;
      case TS_U32: scan_chunk<uint32_t, 2, 2>(sp, c, lane); break;
      case TS_U64: scan_chunk<uint64_t, 2, 2>(sp, c, lane); break;
      case TS_F16: scan_chunk<half_t, 2, 2>(sp, c, lane); break;
      case TS_F32: scan_chunk<float, 2, 2>(sp, c, lane); break;
      case TS_F64: scan_chunk<double, 2, 2>(sp, c, lane); break;
    }
  }
}

hipError_t launch_batch_scan(const BatchArgs &a, int64_t grid_blocks, hipStream_t st) {
  if (a.total_chunks == 0) return hipSuccess;
  int64_t g = grid_blocks;
  if (g > (a.total_chunks + 3) / 4) g = (a.total_chunks + 3) / 4;
  if (g < 1) g = 1;
  k_batch_scan<<<dim3((unsigned)g), dim3(256), 0, st>>>(a);
  return hipGetLastError();
}

__device__ inline MergeParams task_merge_params(const BatchArgs &a, const BatchTask &t) {
  MergeParams mp;
  mp.n = t.n;
  mp.shift = t.shift;
  mp.chunk = t.chunk;
  mp.edges = t.x ? (const int64_t *)(a.ws + t.o_edges) : nullptr;
  mp.nb = t.nb;
  mp.binres = (const int64_t *)(a.ws + t.o_binres);
  mp.partL = (const Partial *)(a.ws + t.o_partL);
  mp.partR = (const Partial *)(a.ws + t.o_partR);
  mp.m4 = t.algo == TS_M4;
  mp.sel = (int64_t *)(a.ws + t.o_sel);
  mp.cnt = (int64_t *)(a.ws + t.o_cnt);
  return mp;
}

__global__ __launch_bounds__(256) void k_batch_merge(BatchArgs a) {
  const int lane = lane_id();
  const int64_t slot = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (slot >= a.total_slots) return;
  const BatchTask &t = a.tasks[a.slot_task[slot]];
  const int64_t bin = slot - t.slot_begin;
  if (t.mode != 0 || bin >= t.nb) return;
  const MergeParams mp = task_merge_params(a, t);
  int64_t s, e;
  bin_range(mp, bin, s, e);
  if (s >= e) {
    if (lane == 0) mp.cnt[bin] = 0;
    return;
  }
  int64_t imn, imx;
  merged_bin(mp, s, e, bin, lane, imn, imx);
  if (lane == 0) mp.cnt[bin] = bin_selection(s, e, imn, imx, mp.m4, mp.sel + 4 * bin);
}

hipError_t launch_batch_merge(const BatchArgs &a, hipStream_t st) {
  if (a.total_slots == 0) return hipSuccess;
  k_batch_merge<<<dim3((unsigned)((a.total_slots + 3) / 4)), dim3(256), 0, st>>>(a);
  return hipGetLastError();
}

// One workgroup per task.  MinMax / M4 write their indices; MinMaxLTTB writes
// its candidates {0} + (preselection + 1) + {n-1} and their count.
__global__ __launch_bounds__(256) void k_batch_compact(BatchArgs a) {
  __shared__ int64_t lds[80];
  const BatchTask &t = a.tasks[blockIdx.x];
  const bool mml = t.algo == TS_MINMAXLTTB;
  if (t.mode == 1) {  // n <= n_out: every index
    const int64_t nall = mml ? t.nf : t.n;
    for (int64_t i = threadIdx.x; i < nall; i += blockDim.x) a.out[t.out_offset + i] = i;
    if (threadIdx.x == 0) a.counts[blockIdx.x] = nall;
    return;
  }
  if (t.mode == 2) return;  // MinMaxLTTB without preselection: the LTTB kernel reads all points
  const int64_t *cnt = (const int64_t *)(a.ws + t.o_cnt);
  const int64_t *sel = (const int64_t *)(a.ws + t.o_sel);
  int64_t *dst = mml ? (int64_t *)(a.ws + t.o_cand) + 1 : a.out + t.out_offset;
  const int64_t off_idx = mml ? 1 : 0;
  const int64_t per = (t.nb + blockDim.x - 1) / blockDim.x;
  const int64_t b0 = (int64_t)threadIdx.x * per;
  const int64_t b1 = b0 + per < t.nb ? b0 + per : t.nb;
  int64_t local = 0;
  for (int64_t b = b0; b < b1; b++) local += cnt[b];
  int64_t total;
  int64_t off = block_exclusive_scan(local, lds, total);
  for (int64_t b = b0; b < b1; b++) {
    const int64_t k = cnt[b];
    for (int64_t j = 0; j < k; j++) dst[off + j] = sel[4 * b + j] + off_idx;
    off += k;
  }
  if (threadIdx.x == 0) {
    if (mml) {
      dst[-1] = 0;
      dst[total] = t.nf - 1;
      *(int64_t *)(a.ws + t.o_m) = total + 2;
    } else {
      a.counts[blockIdx.x] = total;
    }
  }
}

hipError_t launch_batch_compact(const BatchArgs &a, hipStream_t st) {
  if (a.ntasks == 0) return hipSuccess;
  k_batch_compact<<<dim3((unsigned)a.ntasks), dim3(256), 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace tsds

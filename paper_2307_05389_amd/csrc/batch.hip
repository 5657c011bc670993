// batch.hip -- batched MinMax / M4 / MinMaxLTTB-preselection over hundreds
// of series of uneven length, dtype and n_out in one pass.
//
// The host plan (api_batch.cpp) lays every series out as a run of equal-byte
// chunks in the work list of its element type (per-task offset table
// `chunk_begin`) and one global list of bin slots (`slot_begin`, nb + 1
// slots per task).
//   k_batch_edges   one wavefront per bin slot of every task with x.
//   k_batch_scan<T> persistent, one launch per element type present: a
//                   fixed grid of wavefronts, each taking one contiguous
//                   range of that type's work list and walking the task list
//                   as it crosses series boundaries; each item is the same
//                   per-chunk reduction as the single-series scan.  One
//                   launch per type keeps each kernel's registers to its own
//                   type (a runtime type switch would size every wavefront
//                   for the widest path).
//   k_batch_merge   one wavefront per bin slot: merge + per-bin selection.
//   k_batch_compact one workgroup per task: scan of the per-bin counts and
//                   the compacted output (or MinMaxLTTB candidates).
// Results are identical to one plain call per series: every per-bin merge is
// order-independent and the per-task arithmetic is the same code.
#include "common.hpp"
#include "internal.hpp"
#include "scan_core.hpp"
#include "select_core.hpp"
#include "batch_core.hpp"

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
  sp.stage = t.stage;
  sp.x = nullptr;
  sp.xedges = nullptr;
  sp.xclass = 0;
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

// Persistent scan over one dtype group: a fixed grid of wavefronts, each
// taking one contiguous range of the group's work list.  Every item looks its
// task up again (two 64-wide probes of the L2-resident offset table) so that
// only the item index lives across iterations: carrying the task's
// parameters through the loop would push wave-uniform state out of scalar
// registers and double the vector registers per wavefront.
template <typename T, int U, int NB>
__global__ __launch_bounds__(256) void k_batch_scan(const BatchTask *__restrict__ tasks, const int64_t *__restrict__ cb,
                                                    const int32_t *__restrict__ tix, int64_t ntasks, int64_t total,
                                                    char *ws, int32_t small) {
  const int lane = lane_id();
  const int64_t W = (int64_t)gridDim.x * 4;
  const int64_t w = uniform((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  const int64_t i0 = total * w / W, i1 = total * (w + 1) / W;
#pragma nounroll
  for (int64_t item = i0; item < i1; item++) {
    const BatchTask *tk = tasks + group_task_of_item(cb, tix, ntasks, item, lane);
    const ScanParams sp = task_scan_params_uniform(ws, tk, small);
    scan_chunk<T, U, NB>(sp, item - uniform(tk->chunk_begin), lane);
  }
}

// The same over a group of staged tasks (chunks copied to LDS first).
template <typename T>
__global__ __launch_bounds__(256) void k_batch_scan_staged(const BatchTask *__restrict__ tasks,
                                                           const int64_t *__restrict__ cb,
                                                           const int32_t *__restrict__ tix, int64_t ntasks,
                                                           int64_t total, char *ws, int32_t small, int64_t lds_per) {
  extern __shared__ u32x4 stage_lds[];
  const int lane = lane_id();
  const int64_t W = (int64_t)gridDim.x * 4;
  const int64_t w = uniform((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  const int64_t i0 = total * w / W, i1 = total * (w + 1) / W;
  u32x4 *lds = stage_lds + (threadIdx.x >> 6) * lds_per;
#pragma nounroll
  for (int64_t item = i0; item < i1; item++) {
    const BatchTask *tk = tasks + group_task_of_item(cb, tix, ntasks, item, lane);
    const ScanParams sp = task_scan_params_uniform(ws, tk, small);
    scan_chunk_staged<T>(sp, item - uniform(tk->chunk_begin), lane, lds);
  }
}

__device__ inline MergeParams task_merge_params(const BatchArgs &a, const BatchTask &t);
__device__ inline MergeParams task_merge_params_uniform(const BatchArgs &a, const BatchTask *__restrict__ t);

// A group of tasks of one element type reduced one wavefront per bin (no
// chunks, no partials, no merge): work item = bin; the wavefront finds its
// task, reduces the whole bin with the single-series tile fold and writes the
// bin's selection.  (One launch for every type, with a wave-uniform type
// switch, sized every wavefront for the widest fold: 159 VGPRs, three
// wavefronts per SIMD.)
template <typename T, int U, int NB>
__global__ __launch_bounds__(256) void k_batch_direct(BatchArgs a, const int64_t *__restrict__ cb,
                                                      const int32_t *__restrict__ tix, int64_t ntasks, int64_t total) {
  const int lane = lane_id();
  const int64_t item = uniform((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  if (item >= total) return;
  const BatchTask *tk = a.tasks + group_task_of_item(cb, tix, ntasks, item, lane);
  const int64_t bin = item - uniform(tk->chunk_begin);
  const MergeParams mp = task_merge_params_uniform(a, tk);
  int64_t s, e;
  bin_range(mp, bin, s, e);
  if (s >= e) {
    if (lane == 0) mp.cnt[bin] = 0;
    return;
  }
  const u32x4 *__restrict__ base = (const u32x4 *)((const T *)uniform(tk->y) - mp.shift);
  u32x4 buf[NB][U];
  SegState<typename Elem<T>::C> st;
  wave_segment<T, U, NB>(base, mp.shift, s, e, lane, buf, 0, st);
  if (lane == 0) mp.cnt[bin] = bin_selection(s, e, st.imn, st.imx, mp.m4, mp.sel + 4 * bin);
}

static hipError_t launch_batch_direct(const BatchArgs &a, const BatchGroup &g, hipStream_t st) {
  const dim3 grid((unsigned)((g.total + 3) / 4)), block(256);
#define TSDS_DIRECT_ARGS a, g.cb, g.tix, g.ntasks, g.total
  // tile shapes of the single-series per-bin kernel (bytes 4x1, wider types
  // 4x2)
  switch (g.ydt) {
    case TS_I8: k_batch_direct<int8_t, 4, 1><<<grid, block, 0, st>>>(TSDS_DIRECT_ARGS); break;
    case TS_I16: k_batch_direct<int16_t, 4, 2><<<grid, block, 0, st>>>(TSDS_DIRECT_ARGS); break;
    case TS_I32: k_batch_direct<int32_t, 4, 2><<<grid, block, 0, st>>>(TSDS_DIRECT_ARGS); break;
    case TS_I64: k_batch_direct<int64_t, 4, 2><<<grid, block, 0, st>>>(TSDS_DIRECT_ARGS); break;
    case TS_U8: k_batch_direct<uint8_t, 4, 1><<<grid, block, 0, st>>>(TSDS_DIRECT_ARGS); break;
    case TS_U16: k_batch_direct<uint16_t, 4, 2><<<grid, block, 0, st>>>(TSDS_DIRECT_ARGS); break;
    case TS_U32: k_batch_direct<uint32_t, 4, 2><<<grid, block, 0, st>>>(TSDS_DIRECT_ARGS); break;
    case TS_U64: k_batch_direct<uint64_t, 4, 2><<<grid, block, 0, st>>>(TSDS_DIRECT_ARGS); break;
    case TS_F16: k_batch_direct<half_t, 4, 2><<<grid, block, 0, st>>>(TSDS_DIRECT_ARGS); break;
    case TS_F32: k_batch_direct<float, 4, 2><<<grid, block, 0, st>>>(TSDS_DIRECT_ARGS); break;
    case TS_F64: k_batch_direct<double, 4, 2><<<grid, block, 0, st>>>(TSDS_DIRECT_ARGS); break;
    default: return hipErrorInvalidValue;
  }
#undef TSDS_DIRECT_ARGS
  return hipGetLastError();
}

hipError_t launch_batch_scan(const BatchArgs &a, const BatchGroup &g, int64_t grid_blocks, hipStream_t st) {
  if (g.nan) return launch_batch_scan_nan(a, g, grid_blocks, st);
  if (g.total == 0) return hipSuccess;
  if (g.stage == 2) return launch_batch_direct(a, g, st);
  int64_t gb = grid_blocks;
  if (gb > (g.total + 3) / 4) gb = (g.total + 3) / 4;
  if (gb < 1) gb = 1;
  dim3 grid((unsigned)gb), block(256);
  if (g.stage) {
    // staged chunks are 8 KiB: 8192 / sizeof(T) elements, 513 vectors per wavefront
    const int64_t per = 8192 / 16 + 1;
    const size_t lds = 4 * sizeof(u32x4) * (size_t)per;
#define TSDS_STAGED(T) k_batch_scan_staged<T><<<grid, block, lds, st>>>(a.tasks, g.cb, g.tix, g.ntasks, g.total, a.ws, a.small, per)
    switch (g.ydt) {
      case TS_I8: TSDS_STAGED(int8_t); break;
      case TS_I16: TSDS_STAGED(int16_t); break;
      case TS_I32: TSDS_STAGED(int32_t); break;
      case TS_I64: TSDS_STAGED(int64_t); break;
      case TS_U8: TSDS_STAGED(uint8_t); break;
      case TS_U16: TSDS_STAGED(uint16_t); break;
      case TS_U32: TSDS_STAGED(uint32_t); break;
      case TS_U64: TSDS_STAGED(uint64_t); break;
      case TS_F16: TSDS_STAGED(half_t); break;
      case TS_F32: TSDS_STAGED(float); break;
      case TS_F64: TSDS_STAGED(double); break;
      default: return hipErrorInvalidValue;
    }
#undef TSDS_STAGED
    return hipGetLastError();
  }
#define TSDS_BATCH_ARGS a.tasks, g.cb, g.tix, g.ntasks, g.total, a.ws, a.small
  // tile shapes per element size as in the single-series scan (bytes: 4x1,
  // 16-bit: 4x2, 32/64-bit: 8x1 vectors per lane x tiles in flight)
  switch (g.ydt) {
    case TS_I8: k_batch_scan<int8_t, 4, 1><<<grid, block, 0, st>>>(TSDS_BATCH_ARGS); break;
    case TS_I16: k_batch_scan<int16_t, 4, 2><<<grid, block, 0, st>>>(TSDS_BATCH_ARGS); break;
    case TS_I32: k_batch_scan<int32_t, 8, 1><<<grid, block, 0, st>>>(TSDS_BATCH_ARGS); break;
    case TS_I64: k_batch_scan<int64_t, 8, 1><<<grid, block, 0, st>>>(TSDS_BATCH_ARGS); break;
    case TS_U8: k_batch_scan<uint8_t, 4, 1><<<grid, block, 0, st>>>(TSDS_BATCH_ARGS); break;
    case TS_U16: k_batch_scan<uint16_t, 4, 2><<<grid, block, 0, st>>>(TSDS_BATCH_ARGS); break;
    case TS_U32: k_batch_scan<uint32_t, 8, 1><<<grid, block, 0, st>>>(TSDS_BATCH_ARGS); break;
    case TS_U64: k_batch_scan<uint64_t, 8, 1><<<grid, block, 0, st>>>(TSDS_BATCH_ARGS); break;
    case TS_F16: k_batch_scan<half_t, 4, 2><<<grid, block, 0, st>>>(TSDS_BATCH_ARGS); break;
    case TS_F32: k_batch_scan<float, 8, 1><<<grid, block, 0, st>>>(TSDS_BATCH_ARGS); break;
    case TS_F64: k_batch_scan<double, 8, 1><<<grid, block, 0, st>>>(TSDS_BATCH_ARGS); break;
    default: return hipErrorInvalidValue;
  }
#undef TSDS_BATCH_ARGS
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
  mp.m4 = t.algo == TS_M4 || t.algo == TS_NAN_M4;
  mp.sel = (int64_t *)(a.ws + t.o_sel);
  mp.cnt = (int64_t *)(a.ws + t.o_cnt);
  return mp;
}

// The same with every field read as wave-uniform (scalar registers), for a
// task pointer that is itself wave-uniform.
__device__ inline MergeParams task_merge_params_uniform(const BatchArgs &a, const BatchTask *__restrict__ t) {
  MergeParams mp;
  mp.n = uniform(t->n);
  mp.shift = uniform(t->shift);
  mp.chunk = uniform(t->chunk);
  mp.edges = uniform(t->x) ? (const int64_t *)(a.ws + uniform(t->o_edges)) : nullptr;
  mp.nb = uniform(t->nb);
  mp.binres = (const int64_t *)(a.ws + uniform(t->o_binres));
  mp.partL = (const Partial *)(a.ws + uniform(t->o_partL));
  mp.partR = (const Partial *)(a.ws + uniform(t->o_partR));
  const int32_t algo = uniform(t->algo);
  mp.m4 = algo == TS_M4 || algo == TS_NAN_M4;
  mp.sel = (int64_t *)(a.ws + uniform(t->o_sel));
  mp.cnt = (int64_t *)(a.ws + uniform(t->o_cnt));
  return mp;
}

// Slots [0, wave_slots) belong to tasks whose bins span many chunks: one
// wavefront per slot.  The rest (bins spanning few chunks): one thread per
// slot, in k_batch_merge_lanes.
__global__ __launch_bounds__(256) void k_batch_merge(BatchArgs a) {
  const int lane = lane_id();
  const int64_t slot = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (slot >= a.wave_slots) return;
  const BatchTask &t = a.tasks[a.slot_task[slot]];
  const int64_t bin = slot - t.slot_begin;
  if (t.mode != 0 || t.stage == 2 || bin >= t.nb) return;
  const MergeParams mp = task_merge_params(a, t);
  int64_t s, e;
  bin_range(mp, bin, s, e);
  if (s >= e) {
    if (lane == 0) mp.cnt[bin] = 0;
    return;
  }
  int64_t imn, imx;
  merged_bin(mp, s, e, bin, lane, imn, imx);
  if (imn == INT64_MAX) imn = s;  // only NaN-aware tasks leave a bin without a value
  if (imx == INT64_MAX) imx = s;
  if (lane == 0) mp.cnt[bin] = bin_selection(s, e, imn, imx, mp.m4, mp.sel + 4 * bin);
}

__global__ __launch_bounds__(256) void k_batch_merge_lanes(BatchArgs a) {
  const int64_t slot = a.wave_slots + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (slot >= a.total_slots) return;
  const BatchTask &t = a.tasks[a.slot_task[slot]];
  const int64_t bin = slot - t.slot_begin;
  if (t.mode != 0 || t.stage == 2 || bin >= t.nb) return;
  const MergeParams mp = task_merge_params(a, t);
  int64_t s, e;
  bin_range(mp, bin, s, e);
  if (s >= e) {
    mp.cnt[bin] = 0;
    return;
  }
  int64_t imn, imx;
  merged_bin_lane(mp, s, e, bin, imn, imx);
  if (imn == INT64_MAX) imn = s;
  if (imx == INT64_MAX) imx = s;
  mp.cnt[bin] = bin_selection(s, e, imn, imx, mp.m4, mp.sel + 4 * bin);
}

hipError_t launch_batch_merge(const BatchArgs &a, hipStream_t st) {
  if (a.wave_slots > 0) k_batch_merge<<<dim3((unsigned)((a.wave_slots + 3) / 4)), dim3(256), 0, st>>>(a);
  const int64_t lanes = a.total_slots - a.wave_slots;
  if (lanes > 0) k_batch_merge_lanes<<<dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, st>>>(a);
  return hipGetLastError();
}

// One workgroup per task.  MinMax / M4 write their indices; MinMaxLTTB writes
// its candidates {0} + (preselection + 1) + {n-1} and their count.
__global__ __launch_bounds__(1024) void k_batch_compact(BatchArgs a) {
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
  const int64_t total = compact_bins(cnt, sel, 0, t.nb, dst, 0, off_idx, lds);
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
  k_batch_compact<<<dim3((unsigned)a.ntasks), dim3(1024), 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace tsds

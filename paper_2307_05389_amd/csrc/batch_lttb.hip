// batch_lttb.hip -- the LTTB step of every MinMaxLTTB task of a batch: one
// workgroup per task computes the bucket centres and walks the buckets with
// the transition map (see lttb.hip).  Built with IEEE mode and no FMA
// contraction, like the single-series LTTB kernels.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"
#include "lttb_core.hpp"

namespace tsds {

__device__ inline LttbParams task_lttb_params(const BatchArgs &a, const BatchTask &t, int64_t task) {
  LttbParams p{};
  p.x = t.xf;
  p.x_dtype = t.xf ? t.xdt : TS_NONE;
  p.y = t.yf;
  p.y_dtype = t.ydt;
  p.sel = t.mode == 0 ? (const int64_t *)(a.ws + t.o_cand) : nullptr;
  p.m = t.mode == 0 ? -1 : t.nf;
  p.m_dev = (const int64_t *)(a.ws + t.o_m);
  p.m_max = t.m_max;
  p.n_out = t.n_out;
  p.cx = (double *)(a.ws + t.o_cx);
  p.cy = (double *)(a.ws + t.o_cy);
  p.next = (int32_t *)(a.ws + t.o_next);
  p.entry = (int32_t *)(a.ws + t.o_entry);
  p.out = a.out + t.out_offset;
  p.out_count = a.counts + task;
  if (t.mode == 0) {
    p.gx = (uint64_t *)(a.ws + t.o_gx);
    p.gy = (uint64_t *)(a.ws + t.o_gy);
  }
  return p;
}

// The candidates' coordinates of every MinMaxLTTB task with a preselection
// (blockIdx.x = task, one thread per candidate strided over blockIdx.y).
__global__ __launch_bounds__(256) void k_batch_lttb_gather(BatchArgs a) {
  const int64_t task = a.lttb_tasks[blockIdx.x];
  const BatchTask &t = a.tasks[task];
  if (t.mode != 0) return;
  const LttbParams p = task_lttb_params(a, t, task);
  const int64_t m = points_m(p);
  for (int64_t j = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.y * blockDim.x) {
    const int64_t s = src_of(p, j);
    p.gx[j] = coord_word(p.x, p.x_dtype, s);
    p.gy[j] = coord_word(p.y, p.y_dtype, s);
  }
}

// Transition maps of every MinMaxLTTB task: blockIdx.x = task, one thread per
// anchor (strided over blockIdx.y); the centres are computed where they are
// needed (the same sequential means the single-series kernel stores first).
__global__ __launch_bounds__(256) void k_batch_lttb_map(BatchArgs a) {
  const int64_t task = a.lttb_tasks[blockIdx.x];
  const BatchTask &t = a.tasks[task];
  if (t.mode == 1) return;
  const LttbParams p = task_lttb_params(a, t, task);
  const int64_t m = points_m(p);
  if (m <= p.n_out) return;
  for (int64_t an = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; an < m - 1; an += (int64_t)gridDim.y * blockDim.x)
    p.next[an] = lttb_map_one(p, m, an, true);
}

// The walk of each task along its map, one workgroup per task.
__global__ __launch_bounds__(1024) void k_batch_lttb(BatchArgs a) {
  extern __shared__ int32_t smem[];
  const int64_t task = a.lttb_tasks[blockIdx.x];
  const BatchTask &t = a.tasks[task];
  if (t.mode == 1) return;  // written by the compaction
  const LttbParams p = task_lttb_params(a, t, task);
  const int64_t m = points_m(p);
  if (m <= p.n_out) {
    copy_all(p, m);
    return;
  }
  const bool lds = a.lds_ok && t.m_max <= a.lds_m;
  int32_t *next = p.next, *jump = p.next + p.m_max;
  if (lds) {
    copy_map(p.next, smem, m - 1);
    next = smem;
    jump = smem + a.lds_m;
    __syncthreads();
  }
  lttb_walk_map(p, m, next, jump, lttb_group_len(p.n_out - 2));
}

hipError_t launch_batch_lttb(const BatchArgs &a, hipStream_t st) {
  if (a.n_lttb == 0) return hipSuccess;
  const size_t lds = a.lds_ok ? (size_t)a.lds_m * 2 * sizeof(int32_t) : 0;
  const int64_t ychunks = std::min<int64_t>((a.max_m + 255) / 256, 1024);
  k_batch_lttb_gather<<<dim3((unsigned)a.n_lttb, (unsigned)std::max<int64_t>(ychunks, 1)), dim3(256), 0, st>>>(a);
  k_batch_lttb_map<<<dim3((unsigned)a.n_lttb, (unsigned)std::max<int64_t>(ychunks, 1)), dim3(256), 0, st>>>(a);
  k_batch_lttb<<<dim3((unsigned)a.n_lttb), dim3(1024), lds, st>>>(a);
  return hipGetLastError();
}

}  // namespace tsds

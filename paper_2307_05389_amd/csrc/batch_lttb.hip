// batch_lttb.hip -- the LTTB step of every MinMaxLTTB task of a batch: one
// workgroup per task computes the bucket centres and walks the buckets with
// the transition map (see lttb.hip).  Built with IEEE mode and no FMA
// contraction, like the single-series LTTB kernels.
#include "common.hpp"
#include "internal.hpp"
#include "lttb_core.hpp"

namespace tsds {

__global__ __launch_bounds__(1024) void k_batch_lttb(BatchArgs a) {
  extern __shared__ int32_t smem[];
  const BatchTask &t = a.tasks[a.lttb_tasks[blockIdx.x]];
  const int64_t task = a.lttb_tasks[blockIdx.x];
  if (t.mode == 1) return;  // written by the compaction
  LttbParams p;
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
  const int64_t m = points_m(p);
  if (m <= p.n_out) {
    copy_all(p, m);
    return;
  }
  lttb_block_centres(p, m);
  __syncthreads();
  const bool lds = a.lds_ok && t.m_max <= a.lds_m;
  lttb_small_walk(p, m, lds ? smem : p.next, lds ? smem + a.lds_m : p.next + p.m_max,
                  lttb_group_len(p.n_out - 2));
}

hipError_t launch_batch_lttb(const BatchArgs &a, hipStream_t st) {
  if (a.n_lttb == 0) return hipSuccess;
  const size_t lds = a.lds_ok ? (size_t)a.lds_m * 2 * sizeof(int32_t) : 0;
  k_batch_lttb<<<dim3((unsigned)a.n_lttb), dim3(1024), lds, st>>>(a);
  return hipGetLastError();
}

}  // namespace tsds

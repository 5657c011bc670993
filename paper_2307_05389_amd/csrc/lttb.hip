// lttb.hip -- LTTB bucket walk (Steinarsson's algorithm as used by the
// paper's LTTB and MinMaxLTTB downsamplers, Sec. 4) on gfx950, in FP64.
//
// Points are P_j = (X_j, Y_j) for j < m, taken through an optional index
// list `sel` (MinMaxLTTB's candidates).  X is the index when there is no x.
// The first and last point are kept; the m-2 interior points form n_out-2
// buckets by count; walking the buckets in order, each keeps the first point
// with the largest doubled triangle area
//     |(XA - Cx)(Yb - YA) - (XA - Xb)(Cy - YA)|
// against the previous pick A and the centre C of the next bucket (the last
// point for the last bucket).  This translation unit is compiled with
// -ffp-contract=off: every product and difference above is rounded on its
// own, exactly as written.
//
//   k_centres     one thread per bucket: the centre is a sequential FP64 sum
//                 in index order (exact 128-bit integer sum for integer
//                 coordinates), so it is rounded exactly like a plain loop.
//   k_lttb_small  MinMaxLTTB (buckets of a few candidates): the choice in
//                 bucket k depends only on the pick in bucket k-1, so the
//                 map next[a] (best point of bucket k for every possible
//                 anchor a in bucket k-1) is computed for all anchors at once;
//                 the walk then follows next[] in groups of S buckets
//                 (group exits in parallel, a short chain over groups, group
//                 interiors in parallel): about 2S + nb/S dependent steps in
//                 LDS instead of nb.
//   k_lttb_seq    plain LTTB (large buckets): one workgroup walks the buckets
//                 in order; in each, 1024 threads evaluate the areas and a
//                 DPP + LDS reduction returns the first maximum.
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"
#include "lttb_core.hpp"

namespace tsds {

// ---------------------------------------------------------------- centres

__global__ __launch_bounds__(256) void k_centres(LttbParams p) {
  const int64_t m = points_m(p);
  const int64_t nb = p.n_out - 2;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m <= p.n_out || k >= nb) return;
  if (k == nb - 1) {
    p.cx[k] = X_of(p, m - 1);
    p.cy[k] = Y_of(p, m - 1);
    return;
  }
  const int64_t lo = bucket_start(k + 1, m, nb), hi = bucket_start(k + 2, m, nb);
  p.cx[k] = coord_mean(p, 0, lo, hi);
  p.cy[k] = coord_mean(p, 1, lo, hi);
}

hipError_t launch_lttb_centres(const LttbParams &p, hipStream_t st) {
  const int64_t nb = p.n_out - 2;
  k_centres<<<dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st>>>(p);
  return hipGetLastError();
}

// ---------------------------------------------------------------- small

// next[] and jump[] live in LDS when `lds_ok`, else in global workspace.
__global__ __launch_bounds__(1024) void k_lttb_small(LttbParams p, int32_t group, int lds_ok) {
  extern __shared__ int32_t smem[];
  const int64_t m = points_m(p);
  if (m <= p.n_out) {
    copy_all(p, m);
    return;
  }
  lttb_small_walk(p, m, lds_ok ? smem : p.next, lds_ok ? smem + p.m_max : p.next + p.m_max, group);
}

hipError_t launch_lttb_small(const LttbParams &p, hipStream_t st) {
  const int32_t group = lttb_group_len(p.n_out - 2);
  const size_t lds = (size_t)p.m_max * 2 * sizeof(int32_t);
  const int lds_ok = lds <= 128 * 1024;
  k_lttb_small<<<dim3(1), dim3(1024), lds_ok ? lds : 0, st>>>(p, group, lds_ok);
  return hipGetLastError();
}

size_t lttb_group_count(int64_t n_out) {
  const int64_t nb = n_out - 2;
  const int64_t group = lttb_group_len(nb);
  return (size_t)((nb + group - 1) / group);
}

// ---------------------------------------------------------------- sequential

__global__ __launch_bounds__(1024) void k_lttb_seq(LttbParams p) {
  __shared__ double s_area[16];
  __shared__ int64_t s_idx[17];
  const int64_t m = points_m(p);
  if (m <= p.n_out) {
    copy_all(p, m);
    return;
  }
  const int64_t nb = p.n_out - 2;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = blockDim.x >> 6;
  int64_t A = 0;
  for (int64_t k = 0; k < nb; k++) {
    const int64_t lo = bucket_start(k, m, nb), hi = bucket_start(k + 1, m, nb);
    const double XA = X_of(p, A), YA = Y_of(p, A), Cx = p.cx[k], Cy = p.cy[k];
    double best = -1.0;
    int64_t arg = INT64_MAX;
    for (int64_t b = lo + t; b < hi; b += blockDim.x) {
      double a = area2(XA, YA, X_of(p, b), Y_of(p, b), Cx, Cy);
      if (a > best) { best = a; arg = b; }
    }
    const double wb = wave_max(best);
    const int64_t wa = wave_min(best == wb ? arg : INT64_MAX);
    if (lane == 0) {
      s_area[w] = wb;
      s_idx[w] = wa;
    }
    __syncthreads();
    if (w == 0) {
      double b2 = lane < nw ? s_area[lane] : -2.0;
      int64_t a2 = lane < nw ? s_idx[lane] : INT64_MAX;
      const double bb = wave_max(b2);
      const int64_t aa = wave_min(b2 == bb ? a2 : INT64_MAX);
      if (lane == 0) {
        s_idx[16] = aa;
        p.out[k + 1] = src_of(p, aa);
      }
    }
    __syncthreads();
    A = s_idx[16];
    __syncthreads();
  }
  if (t == 0) {
    p.out[0] = src_of(p, 0);
    p.out[p.n_out - 1] = src_of(p, m - 1);
    *p.out_count = p.n_out;
  }
}

hipError_t launch_lttb_seq(const LttbParams &p, hipStream_t st) {
  k_lttb_seq<<<dim3(1), dim3(1024), 0, st>>>(p);
  return hipGetLastError();
}

}  // namespace tsds

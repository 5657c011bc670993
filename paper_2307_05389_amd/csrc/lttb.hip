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

// Sums over a contiguous range [lo, hi) of one array (no index list), with
// eight loads in flight: integers exactly in 128 bits (order-free), floats
// widened to double and added strictly in index order, so the rounding is
// that of the plain sequential loop.
template <typename V>
__device__ inline __int128 range_sum_int(const V *a, int64_t lo, int64_t hi) {
  __int128 s = 0;
  int64_t j = lo;
  for (; j + 8 <= hi; j += 8) {
    V v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = a[j + u];
#pragma unroll
    for (int u = 0; u < 8; u++) s += (__int128)v[u];
  }
  for (; j < hi; j++) s += (__int128)a[j];
  return s;
}

template <typename V>
__device__ inline double range_sum_float(const V *a, int64_t lo, int64_t hi) {
  double s = 0.0;
  int64_t j = lo;
  for (; j + 8 <= hi; j += 8) {
    V v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = a[j + u];
#pragma unroll
    for (int u = 0; u < 8; u++) s += (double)v[u];
  }
  for (; j < hi; j++) s += (double)a[j];
  return s;
}

__device__ inline double range_sum_half(const uint16_t *a, int64_t lo, int64_t hi) {
  double s = 0.0;
  int64_t j = lo;
  for (; j + 8 <= hi; j += 8) {
    uint16_t v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = a[j + u];
#pragma unroll
    for (int u = 0; u < 8; u++) s += (double)(float)__builtin_bit_cast(_Float16, v[u]);
  }
  for (; j < hi; j++) s += (double)(float)__builtin_bit_cast(_Float16, a[j]);
  return s;
}

// Mean of one coordinate over points [lo, hi) of a series without an index
// list: the same value coord_mean computes (exact integer sum rounded once,
// or the sequential double sum), with the index sum in closed form.
__device__ double range_mean(const void *a, int dt, int64_t lo, int64_t hi) {
  const double cnt = (double)(hi - lo);
  switch (dt) {
    case TS_NONE: {
      const __int128 s = ((__int128)lo + (__int128)hi - 1) * (__int128)(hi - lo) / 2;
      return i128_to_double(s) / cnt;
    }
    case TS_I8: return i128_to_double(range_sum_int((const int8_t *)a, lo, hi)) / cnt;
    case TS_I16: return i128_to_double(range_sum_int((const int16_t *)a, lo, hi)) / cnt;
    case TS_I32: return i128_to_double(range_sum_int((const int32_t *)a, lo, hi)) / cnt;
    case TS_I64: return i128_to_double(range_sum_int((const int64_t *)a, lo, hi)) / cnt;
    case TS_U8: return i128_to_double(range_sum_int((const uint8_t *)a, lo, hi)) / cnt;
    case TS_U16: return i128_to_double(range_sum_int((const uint16_t *)a, lo, hi)) / cnt;
    case TS_U32: return i128_to_double(range_sum_int((const uint32_t *)a, lo, hi)) / cnt;
    case TS_U64: return i128_to_double(range_sum_int((const uint64_t *)a, lo, hi)) / cnt;
    case TS_F16: return range_sum_half((const uint16_t *)a, lo, hi) / cnt;
    case TS_F32: return range_sum_float((const float *)a, lo, hi) / cnt;
    case TS_F64: return range_sum_float((const double *)a, lo, hi) / cnt;
  }
  return 0.0;
}

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
  if (p.sel) {
    p.cx[k] = coord_mean(p, 0, lo, hi);
    p.cy[k] = coord_mean(p, 1, lo, hi);
  } else {
    p.cx[k] = range_mean(p.x, p.x_dtype, lo, hi);
    p.cy[k] = range_mean(p.y, p.y_dtype, lo, hi);
  }
}

// Centres of a plain series with long buckets, one wavefront per bucket.
// Integer coordinates: each lane sums its share exactly and lane 0 adds the
// 64 partial sums (exact, so the order is free).  Float coordinates: the
// wavefront copies the bucket to LDS a tile at a time (coalesced) and lane 0
// (Y) / lane 1 (X) add the tile strictly in index order, as the sequential
// loop does.  The index coordinate has a closed form.
constexpr int kCentreTile = 1024;

__device__ inline bool float_dtype(int dt) { return dt == TS_F16 || dt == TS_F32 || dt == TS_F64; }

__global__ __launch_bounds__(64) void k_centres_wave(LttbParams p) {
  __shared__ double tile[2][kCentreTile];
  __shared__ __int128 part[2][64];
  const int lane = threadIdx.x;
  const int64_t m = p.m, nb = p.n_out - 2;
  const int64_t k = blockIdx.x;
  if (k == nb - 1) {
    if (lane == 0) {
      p.cx[k] = X_of(p, m - 1);
      p.cy[k] = Y_of(p, m - 1);
    }
    return;
  }
  const int64_t lo = bucket_start(k + 1, m, nb), hi = bucket_start(k + 2, m, nb);
  const double cnt = (double)(hi - lo);
  const bool fx = p.x_dtype != TS_NONE && float_dtype(p.x_dtype), fy = float_dtype(p.y_dtype);
  // exact integer parts (lane shares, then lane 0 / lane 1 add them up)
  __int128 ix = 0, iy = 0;
  const bool ex = p.x_dtype != TS_NONE && !fx;
  if (ex || !fy) {
    for (int64_t j = lo + lane; j < hi; j += 64) {
      if (ex) ix += int_val(p.x, p.x_dtype, j);
      if (!fy) iy += int_val(p.y, p.y_dtype, j);
    }
  }
  part[0][lane] = ix;
  part[1][lane] = iy;
  // sequential float sums through LDS tiles
  double sx = 0.0, sy = 0.0;
  if (fx || fy) {
    for (int64_t t0 = lo; t0 < hi; t0 += kCentreTile) {
      const int64_t t1 = t0 + kCentreTile < hi ? t0 + kCentreTile : hi;
      for (int64_t j = t0 + lane; j < t1; j += 64) {
        if (fy) tile[0][j - t0] = dbl_val(p.y, p.y_dtype, j);
        if (fx) tile[1][j - t0] = dbl_val(p.x, p.x_dtype, j);
      }
      __syncthreads();
      if ((lane == 0 && fy) || (lane == 1 && fx)) {
        const double *tv = tile[lane];
        double acc = lane == 0 ? sy : sx;
        for (int64_t j = 0; j < t1 - t0; j++) acc += tv[j];
        if (lane == 0) sy = acc; else sx = acc;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (lane < 2) {
    double mean;
    const int c = lane;  // 0: y, 1: x
    if (c == 1 && p.x_dtype == TS_NONE) {
      mean = i128_to_double(((__int128)lo + (__int128)hi - 1) * (__int128)(hi - lo) / 2) / cnt;
    } else if (c == 0 ? fy : fx) {
      mean = (c == 0 ? sy : sx) / cnt;
    } else {
      __int128 s = 0;
      for (int i = 0; i < 64; i++) s += part[c == 0 ? 1 : 0][i];
      mean = i128_to_double(s) / cnt;
    }
    if (c == 0) p.cy[k] = mean; else p.cx[k] = mean;
  }
}

hipError_t launch_lttb_centres(const LttbParams &p, hipStream_t st) {
  const int64_t nb = p.n_out - 2;
  if (!p.sel && p.m >= 0 && (p.m - 2) / nb >= kHullMinBucket)
    k_centres_wave<<<dim3((unsigned)nb), dim3(64), 0, st>>>(p);
  else
    k_centres<<<dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st>>>(p);
  return hipGetLastError();
}

// ---------------------------------------------------------------- small

// The transition map of every anchor, one thread each over the whole GPU
// (the map is the bulk of the small-bucket walk: a few dependent loads per
// anchor through the candidate list), into p.next in global memory.
__global__ __launch_bounds__(256) void k_lttb_map(LttbParams p) {
  const int64_t m = points_m(p);
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m <= p.n_out || a >= m - 1) return;
  p.next[a] = lttb_map_one(p, m, a, false);
}

// The walk along the map by one workgroup; next[] (copied from global) and
// jump[] live in LDS when `lds_ok`, else in global workspace.
__global__ __launch_bounds__(1024) void k_lttb_small(LttbParams p, int32_t group, int lds_ok) {
  extern __shared__ int32_t smem[];
  const int64_t m = points_m(p);
  if (m <= p.n_out) {
    copy_all(p, m);
    return;
  }
  int32_t *next = p.next, *jump = p.next + p.m_max;
  if (lds_ok) {
    for (int64_t a = threadIdx.x; a < m - 1; a += blockDim.x) smem[a] = p.next[a];
    next = smem;
    jump = smem + p.m_max;
    __syncthreads();
  }
  lttb_walk_map(p, m, next, jump, group);
}

hipError_t launch_lttb_small(const LttbParams &p, hipStream_t st) {
  const int32_t group = lttb_group_len(p.n_out - 2);
  const size_t lds = (size_t)p.m_max * 2 * sizeof(int32_t);
  const int lds_ok = lds <= 128 * 1024;
  k_lttb_map<<<dim3((unsigned)((p.m_max + 255) / 256)), dim3(256), 0, st>>>(p);
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

// ---------------------------------------------------------------- hull

// Plain LTTB with long buckets.  With the anchor A and the centre C fixed, the
// doubled area of point b is |u X_b + v Y_b + w| (u = Cy - YA, v = XA - Cx),
// the absolute value of a linear function of b's coordinates, so over a
// bucket its maximum is reached at a vertex of the bucket's convex hull.  The
// hulls do not depend on the walk: k_lttb_hull builds every bucket's hull in
// parallel (one wavefront per bucket: each lane a monotone chain over its
// slice, then one lane per chain merges the 64 slices), and the walk only
// evaluates the hull vertices.
//
// First-occurrence ties: the points reaching the maximum form a vertex or a
// hull edge.  Points are in index order with X non-decreasing, so a
// non-vertical edge's smallest index is its left end, a vertex; vertical runs
// keep their first highest / lowest point; the only vertical extreme edge
// that can hold every maximum is the case where all points share one X (then
// v = 0 and every point ties), covered by always keeping the bucket's first
// point.  Collinear points are therefore dropped.  In floating point a point
// dropped as (near-)collinear can differ from a kept vertex only by rounding:
// the near-tie rule of the LTTB tolerance.

__device__ inline double cross3(double ox, double oy, double ax, double ay, double bx, double by) {
  return (ax - ox) * (by - oy) - (ay - oy) * (bx - ox);
}

// Turn pops per point in the branch-free slice chains.
constexpr int kHullPops = 3;

// Monotone chain over points added in index order (offsets from the bucket
// start `lo`), its stack (offset, Y and, with x, X) in LDS; without x, X is
// the index lo + offset.  upper: the upper hull (keeps clockwise turns), else
// the lower hull.
template <bool HX>
struct HullChain {
  int32_t *so;
  double *sx, *sy;
  int64_t lo;
  int n, cap, stride;  // entry i at [i * stride] (lane stacks interleave, stride 64)
  bool upper, over;
  // the top two entries are also kept in registers: a push reads no LDS and a
  // pop reads only the entry that becomes second
  double tx, ty, ux, uy;
  __device__ HullChain(int32_t *o, double *x, double *y, int64_t lo_, int capacity, int str, bool up)
      : so(o), sx(x), sy(y), lo(lo_), n(0), cap(capacity), stride(str), upper(up), over(false), tx(0), ty(0),
        ux(0), uy(0) {}
  // without x the X coordinate is the offset from the bucket start (cross
  // products of small integers, identical to those of the absolute index)
  __device__ double X(int i) const { return HX ? sx[i * stride] : (double)so[i * stride]; }
  __device__ double Y(int i) const { return sy[i * stride]; }
  __device__ void pop() {
    n--;
    tx = ux;
    ty = uy;
    if (n >= 2) {
      ux = X(n - 2);
      uy = Y(n - 2);
    }
  }
  // Branch-free variant for whole wavefronts of independent chains: at most
  // one pop for a repeated X and kHullPops turn pops per point (further pops
  // are skipped, so the stack may keep extra points but never loses a hull
  // vertex: every pop is justified by two points of the set).  The entries
  // that may become second are read from LDS up front, in one round trip.
  __device__ void add_bounded(int32_t j, double xj, double yj) {
    constexpr int K = HX ? kHullPops + 1 : kHullPops;  // without x no X repeats
    // ex/ey[i]: the entry that becomes second after i + 1 pops; popping
    // shifts this window (selects only, no indexed registers)
    double ex[K], ey[K];
#pragma unroll
    for (int i = 0; i < K; i++) {
      const int e = n - 3 - i >= 0 ? n - 3 - i : 0;
      ex[i] = X(e);
      ey[i] = Y(e);
    }
    const bool same = HX && n > 0 && xj == tx;
    const bool act = !over && !(same && (upper ? !(yj > ty) : !(yj < ty)));
    auto cond_pop = [&](bool pp) {
      if (pp) {
        n--;
        tx = ux;
        ty = uy;
        ux = ex[0];
        uy = ey[0];
#pragma unroll
        for (int i = 0; i + 1 < K; i++) {
          ex[i] = ex[i + 1];
          ey[i] = ey[i + 1];
        }
      }
    };
    cond_pop(act && same);
#pragma unroll
    for (int s = 0; s < kHullPops; s++) {
      const double c = cross3(ux, uy, tx, ty, xj, yj);
      cond_pop(act && n >= 2 && (upper ? c >= 0.0 : c <= 0.0));
    }
    if (act && n == cap) over = true;
    if (act && !over) {
      so[n * stride] = j;
      if (HX) sx[n * stride] = xj;
      sy[n * stride] = yj;
      n++;
      ux = tx;
      uy = ty;
      tx = xj;
      ty = yj;
    }
  }
  __device__ void add(int32_t j, double xj, double yj) {
    if (over) return;
    if (n > 0 && xj == tx) {  // same X as the top: keep the first highest (lowest)
      if (upper ? !(yj > ty) : !(yj < ty)) return;
      pop();
    }
    while (n >= 2) {
      const double c = cross3(ux, uy, tx, ty, xj, yj);
      if (upper ? c >= 0.0 : c <= 0.0)
        pop();
      else
        break;
    }
    if (n == cap) {
      over = true;
      return;
    }
    so[n * stride] = j;
    if (HX) sx[n * stride] = xj;
    sy[n * stride] = yj;
    n++;
    ux = tx;
    uy = ty;
    tx = xj;
    ty = yj;
  }
};

// Points loaded per lane before they are added (independent loads in flight).
constexpr int kHullBatch = 16;

// Elements j0 .. j0 + kHullBatch - 1 (clamped to jmax) of a series of dtype
// dt as the doubles the walk uses (dbl_val): the dtype switch is taken once
// per batch and the loads inside it are issued back to back.
template <typename V>
__device__ inline void batch_as_double(const V *a, int64_t j0, int64_t jmax, double (&out)[kHullBatch]) {
  V v[kHullBatch];
#pragma unroll
  for (int u = 0; u < kHullBatch; u++) v[u] = a[j0 + u < jmax ? j0 + u : jmax];
#pragma unroll
  for (int u = 0; u < kHullBatch; u++) out[u] = (double)v[u];
}

__device__ inline void load_batch(const void *a, int dt, int64_t j0, int64_t jmax, double (&out)[kHullBatch]) {
  switch (dt) {
    case TS_I8: batch_as_double((const int8_t *)a, j0, jmax, out); break;
    case TS_I16: batch_as_double((const int16_t *)a, j0, jmax, out); break;
    case TS_I32: batch_as_double((const int32_t *)a, j0, jmax, out); break;
    case TS_I64: batch_as_double((const int64_t *)a, j0, jmax, out); break;
    case TS_U8: batch_as_double((const uint8_t *)a, j0, jmax, out); break;
    case TS_U16: batch_as_double((const uint16_t *)a, j0, jmax, out); break;
    case TS_U32: batch_as_double((const uint32_t *)a, j0, jmax, out); break;
    case TS_U64: batch_as_double((const uint64_t *)a, j0, jmax, out); break;
    case TS_F16: {
      uint16_t v[kHullBatch];
      const uint16_t *h = (const uint16_t *)a;
#pragma unroll
      for (int u = 0; u < kHullBatch; u++) v[u] = h[j0 + u < jmax ? j0 + u : jmax];
#pragma unroll
      for (int u = 0; u < kHullBatch; u++) out[u] = (double)(float)__builtin_bit_cast(_Float16, v[u]);
      break;
    }
    case TS_F32: batch_as_double((const float *)a, j0, jmax, out); break;
    default: batch_as_double((const double *)a, j0, jmax, out); break;
  }
}

// Coordinates of a batch of points lo + j0 + u of the series.
template <bool HX>
__device__ inline void load_points(const LttbParams &p, int64_t lo, int64_t j0, int64_t jmax,
                                   double (&xs)[kHullBatch], double (&ys)[kHullBatch]) {
  load_batch(p.y, p.y_dtype, j0, jmax, ys);
  if (HX) {
    load_batch(p.x, p.x_dtype, j0, jmax, xs);
  } else {
    const double xb = (double)(j0 - lo);  // offset from the bucket start
#pragma unroll
    for (int u = 0; u < kHullBatch; u++) xs[u] = xb + (double)u;
  }
}

template <bool HX, bool HC>
__device__ void feed_raw(const LttbParams &p, int64_t lo, int64_t a, int64_t b, HullChain<HC> &h) {
  for (int64_t j0 = a; j0 < b; j0 += kHullBatch) {
    double xs[kHullBatch], ys[kHullBatch];
    load_points<HX>(p, lo, lo + j0, lo + b - 1, xs, ys);
#pragma unroll
    for (int u = 0; u < kHullBatch; u++)
      if (j0 + u < b) h.add((int32_t)(j0 + u), xs[u], ys[u]);
  }
}

// Group chains of the two-level merge: 8 groups of 8 slices per chain kind.
constexpr int kHullGroup = 32;

template <bool HX>
__global__ __launch_bounds__(64) void k_lttb_hull(LttbParams p) {
  // lane stacks, interleaved: entry i of lane l of chain c at [c][i * 64 + l]
  __shared__ int32_t so[2][64 * kHullLane];
  __shared__ double sx[HX ? 2 : 1][HX ? 64 * kHullLane : 1], sy[2][64 * kHullLane];
  __shared__ int32_t nsl[2][64];
  // group chains: entry i of group g of chain c at [i * 16 + c * 8 + g]
  __shared__ int32_t go[16 * kHullGroup];
  __shared__ double gx[HX ? 16 * kHullGroup : 1], gy[16 * kHullGroup];
  __shared__ int32_t ngr[16];
  __shared__ int32_t mo[2][kHullCand];
  __shared__ double mx[2][kHullCand], my[2][kHullCand];
  __shared__ int32_t mg_n[2];
  const int lane = threadIdx.x;
  const int64_t m = p.m, nb = p.n_out - 2;
  const int64_t k = blockIdx.x;
  const int64_t lo = bucket_start(k, m, nb), hi = bucket_start(k + 1, m, nb);
  const int64_t len = hi - lo;
  // 1. one slice per lane (slices in index order), points loaded in batches
  {
    const int64_t s0 = len * lane / 64, s1 = len * (lane + 1) / 64;
    HullChain<HX> up(so[0] + lane, HX ? sx[0] + lane : nullptr, sy[0] + lane, lo, kHullLane, 64, true);
    HullChain<HX> dn(so[1] + lane, HX ? sx[HX ? 1 : 0] + lane : nullptr, sy[1] + lane, lo, kHullLane, 64, false);
    for (int64_t j0 = s0; j0 < s1; j0 += kHullBatch) {
      double xs[kHullBatch], ys[kHullBatch];
      load_points<HX>(p, lo, lo + j0, lo + s1 - 1, xs, ys);
#pragma unroll
      for (int u = 0; u < kHullBatch; u++) {
        if (j0 + u < s1) {
          up.add_bounded((int32_t)(j0 + u), xs[u], ys[u]);
          dn.add_bounded((int32_t)(j0 + u), xs[u], ys[u]);
        }
      }
    }
    nsl[0][lane] = up.over ? -1 : up.n;  // -1: the slice's points are re-read
    nsl[1][lane] = dn.over ? -1 : dn.n;
  }
  __syncthreads();
  // 2. lanes 0-15 merge 8 slices each (lanes 0-7 upper, 8-15 lower); a
  //    slice's hull keeps every point of the bucket's hull in the slice
  if (lane < 16) {
    const int c = lane >> 3, g = lane & 7;
    HullChain<HX> h(go + lane, HX ? gx + lane : nullptr, gy + lane, lo, kHullGroup, 16, c == 0);
    for (int sl = 8 * g; sl < 8 * g + 8; sl++) {
      const int32_t cn = nsl[c][sl];
      if (cn < 0) {
        feed_raw<HX>(p, lo, len * sl / 64, len * (sl + 1) / 64, h);
        continue;
      }
      for (int e = 0; e < cn; e++) {
        const int q = e * 64 + sl;
        h.add(so[c][q], HX ? sx[HX ? c : 0][q] : (double)so[c][q], sy[c][q]);
      }
    }
    ngr[lane] = h.over ? -1 : h.n;
  }
  __syncthreads();
  // 3. lane 0 merges the upper group chains, lane 1 the lower ones
  if (lane < 2) {
    const int c = lane;
    HullChain<true> h(mo[c], mx[c], my[c], lo, kHullCand, 1, c == 0);
    for (int g = 0; g < 8; g++) {
      const int gi = c * 8 + g;
      const int32_t cn = ngr[gi];
      if (cn >= 0) {
        for (int e = 0; e < cn; e++) {
          const int q = e * 16 + gi;
          h.add(go[q], HX ? gx[q] : (double)go[q], gy[q]);
        }
        continue;
      }
      for (int sl = 8 * g; sl < 8 * g + 8; sl++) {  // the group's chain overflowed
        const int32_t sn = nsl[c][sl];
        if (sn < 0) {
          feed_raw<HX>(p, lo, len * sl / 64, len * (sl + 1) / 64, h);
          continue;
        }
        for (int e = 0; e < sn; e++) {
          const int q = e * 64 + sl;
          h.add(so[c][q], HX ? sx[HX ? c : 0][q] : (double)so[c][q], sy[c][q]);
        }
      }
    }
    mg_n[c] = h.over ? -1 : h.n;
  }
  __syncthreads();
  // 4. candidates: the bucket's first point and both chains, in index order
  if (lane == 0) {
    const int32_t nu = mg_n[0], nd = mg_n[1];
    int32_t total = 0;
    if (nu >= 0 && nd >= 0) {
      int32_t iu = 0, id = 0, last = -1;
      const int64_t base = k * (int64_t)kHullCand;
      bool fits = true;
      auto put = [&](int32_t j, double xj, double yj) {
        if (j == last) return;
        last = j;
        if (total == kHullCand) {
          fits = false;
          return;
        }
        p.cand_idx[base + total] = lo + j;
        p.cand_x[base + total] = HX ? xj : (double)(lo + j);  // absolute coordinates for the walk
        p.cand_y[base + total] = yj;
        total++;
      };
      put(0, X_of(p, lo), Y_of(p, lo));
      while (iu < nu || id < nd) {
        const int32_t a = iu < nu ? mo[0][iu] : INT32_MAX, b = id < nd ? mo[1][id] : INT32_MAX;
        if (a <= b) {
          put(a, mx[0][iu], my[0][iu]);
          iu++;
          if (a == b) id++;
        } else {
          put(b, mx[1][id], my[1][id]);
          id++;
        }
      }
      if (!fits) total = 0;
    }
    p.cand_cnt[k] = total;  // 0: walk every point of the bucket
  }
}

hipError_t launch_lttb_hull(const LttbParams &p, hipStream_t st) {
  const int64_t nb = p.n_out - 2;
  if (p.x_dtype == TS_NONE)
    k_lttb_hull<false><<<dim3((unsigned)nb), dim3(64), 0, st>>>(p);
  else
    k_lttb_hull<true><<<dim3((unsigned)nb), dim3(64), 0, st>>>(p);
  return hipGetLastError();
}

// The walk over the hull candidates, by one wavefront: lane i evaluates
// candidate i of the bucket (candidates of the next bucket are loaded while
// the current one is reduced); a bucket without candidates is walked in full.
__global__ __launch_bounds__(64) void k_lttb_hull_walk(LttbParams p) {
  if (*p.hflag) return;  // k_lttb_hull_chase has written the result
  const int lane = threadIdx.x;
  const int64_t m = p.m, nb = p.n_out - 2;
  double XA = X_of(p, 0), YA = Y_of(p, 0);
  // prefetched candidate and centre of bucket 0
  int32_t ncnt = p.cand_cnt[0];
  double nx = 0.0, ny = 0.0, ncx = p.cx[0], ncy = p.cy[0];
  int64_t ni = 0;
  if (lane < ncnt) {
    nx = p.cand_x[lane];
    ny = p.cand_y[lane];
    ni = p.cand_idx[lane];
  }
  for (int64_t k = 0; k < nb; k++) {
    const int32_t cnt = ncnt;
    const double cxb = nx, cyb = ny, Cx = ncx, Cy = ncy;
    const int64_t cib = ni;
    if (k + 1 < nb) {  // the next bucket's data does not depend on this pick
      ncnt = p.cand_cnt[k + 1];
      ncx = p.cx[k + 1];
      ncy = p.cy[k + 1];
      const int64_t base = (k + 1) * (int64_t)kHullCand;
      if (lane < ncnt) {
        nx = p.cand_x[base + lane];
        ny = p.cand_y[base + lane];
        ni = p.cand_idx[base + lane];
      }
    }
    double best = -1.0, bx = 0.0, by = 0.0;
    int64_t arg = INT64_MAX;
    if (cnt > 0) {
      if (lane < cnt) {
        best = area2(XA, YA, cxb, cyb, Cx, Cy);
        arg = cib;
        bx = cxb;
        by = cyb;
      }
    } else {
      const int64_t lo = bucket_start(k, m, nb), hi = bucket_start(k + 1, m, nb);
      for (int64_t b = lo + lane; b < hi; b += 64) {
        const double xb = X_of(p, b), yb = Y_of(p, b);
        const double a = area2(XA, YA, xb, yb, Cx, Cy);
        if (a > best) {
          best = a;
          arg = b;
          bx = xb;
          by = yb;
        }
      }
    }
    const double wb = wave_max(best);
    const int64_t wa = wave_min(best == wb ? arg : INT64_MAX);
    const int src = __builtin_ctzll(ballot(arg == wa && best == wb));
    XA = readlane(bx, src);
    YA = readlane(by, src);
    if (lane == 0) p.out[k + 1] = wa;
  }
  if (lane == 0) {
    p.out[0] = 0;
    p.out[p.n_out - 1] = m - 1;
    *p.out_count = p.n_out;
  }
}

// Transition maps over the hull candidates: for every bucket k and every
// candidate a of bucket k-1 taken as the anchor (point 0 for bucket 0),
// hnext[k][a] = the candidate of bucket k the walk would pick.  One
// wavefront per bucket, lane a = anchor; the candidates are read from LDS.
__global__ __launch_bounds__(64) void k_lttb_hull_next(LttbParams p) {
  __shared__ double qx[kHullCand], qy[kHullCand];
  const int lane = threadIdx.x;
  const int64_t nb = p.n_out - 2;
  const int64_t k = blockIdx.x;
  const int32_t cnt = p.cand_cnt[k];
  const int32_t na = k == 0 ? 1 : p.cand_cnt[k - 1];
  if (cnt == 0 || na == 0) return;  // the walk falls back to the sequential kernel
  const int64_t base = k * (int64_t)kHullCand;
  if (lane < cnt) {
    qx[lane] = p.cand_x[base + lane];
    qy[lane] = p.cand_y[base + lane];
  }
  __syncthreads();
  if (lane >= na) return;
  double XA, YA;
  if (k == 0) {
    XA = X_of(p, 0);
    YA = Y_of(p, 0);
  } else {
    XA = p.cand_x[base - kHullCand + lane];
    YA = p.cand_y[base - kHullCand + lane];
  }
  const double Cx = p.cx[k], Cy = p.cy[k];
  double best = -1.0;
  int arg = 0;
  for (int i = 0; i < cnt; i++) {
    const double a = area2(XA, YA, qx[i], qy[i], Cx, Cy);
    if (a > best) {
      best = a;
      arg = i;
    }
  }
  p.hnext[base + lane] = (uint8_t)arg;
  (void)nb;
}

int64_t lttb_hull_group(int64_t nb) {
  int64_t g = 1;
  while (g * g < nb) g++;
  return g;
}

// The walk along the maps, by one workgroup, when every bucket has hull
// candidates: the exit of each group of S buckets for each entry anchor (in
// parallel), the chain over the groups, then each group's picks (in
// parallel): about 3S + nb/S dependent steps instead of nb.  Sets hflag when
// it has written the result; otherwise k_lttb_hull_walk does the walk.
__global__ __launch_bounds__(1024) void k_lttb_hull_chase(LttbParams p, int64_t S) {
  __shared__ int bad;
  __shared__ uint8_t entry_s[4096];
  const int t = threadIdx.x;
  const int64_t m = p.m, nb = p.n_out - 2;
  const int64_t G = (nb + S - 1) / S;
  if (t == 0) bad = 0;
  __syncthreads();
  int mine = 0;
  for (int64_t k = t; k < nb; k += blockDim.x) mine |= p.cand_cnt[k] == 0;
  if (mine) bad = 1;
  __syncthreads();
  if (bad || G > 4096) {
    if (t == 0) *p.hflag = 0;
    return;
  }
  // 1. group exits
  for (int64_t idx = t; idx < G * kHullCand; idx += blockDim.x) {
    const int64_t g = idx / kHullCand, e = idx % kHullCand;
    const int32_t ne = g == 0 ? 1 : p.cand_cnt[g * S - 1];
    if (e >= ne) continue;
    const int64_t k1 = (g + 1) * S < nb ? (g + 1) * S : nb;
    int v = (int)e;
    for (int64_t k = g * S; k < k1; k++) v = p.hnext[k * kHullCand + v];
    p.hjump[g * kHullCand + e] = (uint8_t)v;
  }
  __threadfence_block();
  __syncthreads();
  // 2. chain over the groups
  if (t == 0) {
    int v = 0;
    for (int64_t g = 0; g < G; g++) {
      entry_s[g] = (uint8_t)v;
      v = p.hjump[g * kHullCand + v];
    }
  }
  __syncthreads();
  // 3. picks inside every group
  for (int64_t g = t; g < G; g += blockDim.x) {
    int v = entry_s[g];
    const int64_t k1 = (g + 1) * S < nb ? (g + 1) * S : nb;
    for (int64_t k = g * S; k < k1; k++) {
      v = p.hnext[k * kHullCand + v];
      p.out[k + 1] = p.cand_idx[k * kHullCand + v];
    }
  }
  if (t == 0) {
    p.out[0] = 0;
    p.out[p.n_out - 1] = m - 1;
    *p.out_count = p.n_out;
    *p.hflag = 1;
  }
}

hipError_t launch_lttb_hull_walk(const LttbParams &p, hipStream_t st) {
  const int64_t nb = p.n_out - 2;
  k_lttb_hull_next<<<dim3((unsigned)nb), dim3(64), 0, st>>>(p);
  k_lttb_hull_chase<<<dim3(1), dim3(1024), 0, st>>>(p, lttb_hull_group(nb));
  k_lttb_hull_walk<<<dim3(1), dim3(64), 0, st>>>(p);
  return hipGetLastError();
}

}  // namespace tsds

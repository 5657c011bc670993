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

// ---------------------------------------------------------------- raw batches

// Raw bits of elements j0 .. j0 + B - 1 (clamped to jmax) of an array of
// es-byte elements, loaded back to back and converted later, so the loads
// stay in flight while earlier data is used.
template <int B, typename R>
__device__ inline void load_raw(const void *a, int es, int64_t j0, int64_t jmax, R (&r)[B]) {
  switch (es) {
    case 1:
#pragma unroll
      for (int u = 0; u < B; u++) r[u] = ((const uint8_t *)a)[j0 + u < jmax ? j0 + u : jmax];
      break;
    case 2:
#pragma unroll
      for (int u = 0; u < B; u++) r[u] = ((const uint16_t *)a)[j0 + u < jmax ? j0 + u : jmax];
      break;
    case 4:
#pragma unroll
      for (int u = 0; u < B; u++) r[u] = ((const uint32_t *)a)[j0 + u < jmax ? j0 + u : jmax];
      break;
    default:
      if constexpr (sizeof(R) == 8) {
#pragma unroll
        for (int u = 0; u < B; u++) r[u] = ((const uint64_t *)a)[j0 + u < jmax ? j0 + u : jmax];
      }
      break;
  }
}

// Raw bits as the doubles the walk uses (dbl_val), one dtype switch per batch.
template <int B, typename R>
__device__ inline void convert_raw(const R (&r)[B], int dt, double (&out)[B]) {
  switch (dt) {
#define TS_RAW_CVT(code, expr)                                   \
  case code:                                                     \
    _Pragma("unroll") for (int u = 0; u < B; u++) out[u] = expr; \
    break;
    TS_RAW_CVT(TS_I8, (double)(int8_t)(uint8_t)r[u])
    TS_RAW_CVT(TS_U8, (double)(uint8_t)r[u])
    TS_RAW_CVT(TS_I16, (double)(int16_t)(uint16_t)r[u])
    TS_RAW_CVT(TS_U16, (double)(uint16_t)r[u])
    TS_RAW_CVT(TS_F16, (double)(float)__builtin_bit_cast(_Float16, (uint16_t)r[u]))
    TS_RAW_CVT(TS_F32, (double)__builtin_bit_cast(float, (uint32_t)r[u]))
    TS_RAW_CVT(TS_I32, (double)(int32_t)(uint32_t)r[u])
    TS_RAW_CVT(TS_U32, (double)(uint32_t)r[u])
    TS_RAW_CVT(TS_I64, (double)(int64_t)(uint64_t)r[u])
    TS_RAW_CVT(TS_U64, (double)(uint64_t)r[u])
    default:
#pragma unroll
      for (int u = 0; u < B; u++) out[u] = __builtin_bit_cast(double, (uint64_t)r[u]);
      break;
#undef TS_RAW_CVT
  }
}

// Exact sum of the raw integer elements j0 + u < hi of a batch, added to acc.
template <int B>
__device__ inline void add_int_raw(const uint64_t (&r)[B], int dt, int64_t j0, int64_t hi, __int128 &acc) {
  switch (dt) {
#define TS_RAW_INT(code, expr)                                               \
  case code:                                                                 \
    _Pragma("unroll") for (int u = 0; u < B; u++) if (j0 + u < hi) acc += expr; \
    break;
    TS_RAW_INT(TS_I8, (__int128)(int8_t)(uint8_t)r[u])
    TS_RAW_INT(TS_U8, (__int128)(uint8_t)r[u])
    TS_RAW_INT(TS_I16, (__int128)(int16_t)(uint16_t)r[u])
    TS_RAW_INT(TS_U16, (__int128)(uint16_t)r[u])
    TS_RAW_INT(TS_I32, (__int128)(int32_t)(uint32_t)r[u])
    TS_RAW_INT(TS_U32, (__int128)(uint32_t)r[u])
    TS_RAW_INT(TS_I64, (__int128)(int64_t)r[u])
    TS_RAW_INT(TS_U64, (__int128)(uint64_t)r[u])
    default:
      break;
#undef TS_RAW_INT
  }
}

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

// Centres of a plain series with long buckets, one workgroup per bucket.
//
// The sequential double sum of float coordinates (the rounding the centres
// must reproduce) is evaluated without walking every point in turn.  Every
// finite double is odd * 2^q; when a run of terms and the running sum s are
// all multiples of 2^q' (q' the smallest such exponent among them) and
// |s| + sum |v| < 2^(q' + 53), every partial sum of the run is a multiple of
// 2^q' below 2^(q' + 53), hence exactly representable: the sequential loop
// then makes no rounding at all over the run, and s + (the run's sum, added
// in any order) is the same double.  Whether a run qualifies is decided
// exactly from the same quantities computed in floating point: all terms are
// non-negative multiples of 2^q', so a computed sum of them reaches
// 2^(q' + 53) if and only if the exact sum does.
//
// The workgroup's wavefronts summarise tiles of kCentreTile consecutive
// points (coalesced loads, any order): sum, sum of |v|, smallest exponent q,
// or the exact 128-bit sum for integer coordinates.  Wavefront 0 then folds
// the tile summaries into the running sum in index order, one addition per
// tile that qualifies; a tile that does not is staged in LDS in index order
// and folded per 16-point segment, a segment that does not qualify point by
// point.  The result is bit-identical to the plain loop.  The index
// coordinate has a closed form.
constexpr int kCentreBatch = 16;
constexpr int kCentreTile = 64 * kCentreBatch;
constexpr int kCentreRound = 128;       // tile summaries held in LDS at a time
constexpr int kNoExp = 0x7fffffff;      // exponent of a run of zeros

__device__ inline bool float_dtype(int dt) { return dt == TS_F16 || dt == TS_F32 || dt == TS_F64; }

// q with v = odd * 2^q, for finite nonzero v.
__device__ inline int trailing_exp(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int e = (int)((b >> 52) & 0x7ff);
  const uint64_t f = b & ((1ull << 52) - 1);
  return e == 0 ? -1074 + __builtin_ctzll(f) : e - 1075 + __builtin_ctzll(f | (1ull << 52));
}

// True when adding terms that are multiples of 2^qa with absolute sum a to
// the running sum s makes no rounding (see above).
__device__ inline bool adds_exactly(double s, double a, int qa) {
  const int qs = s == 0.0 ? kNoExp : trailing_exp(s);
  const int q = qs < qa ? qs : qa;
  if (q == kNoExp) return true;  // zeros only
  const double t = __builtin_fabs(s) + a;
  if (q + 53 >= 1024) return t < __builtin_huge_val();
  return t < __builtin_bit_cast(double, (uint64_t)(q + 53 + 1023) << 52);
}

__device__ inline double wave_sum_dbl(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline int wave_min_int(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const int w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}
__device__ inline __int128 wave_sum_i128(__int128 v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint64_t lo = __shfl_xor((uint64_t)v, o, 64);
    const uint64_t hi = __shfl_xor((uint64_t)((unsigned __int128)v >> 64), o, 64);
    v += (__int128)(((unsigned __int128)hi << 64) | lo);
  }
  return v;
}

// Raw bits of elements j0 + u*64 + lane (u < kCentreBatch) below hi, 0 past
// it (R: 32-bit words for elements of up to 4 bytes, 64-bit for 8).
template <typename R>
__device__ inline void load_strided(const void *a, int es, int64_t j0, int64_t hi, int lane, R (&r)[kCentreBatch]) {
#pragma unroll
  for (int u = 0; u < kCentreBatch; u++) {
    const int64_t j = j0 + u * 64 + lane;
    R v = 0;
    if (j < hi) {
      if constexpr (sizeof(R) == 8) {
        v = ((const uint64_t *)a)[j];
      } else {
        switch (es) {
          case 1: v = ((const uint8_t *)a)[j]; break;
          case 2: v = ((const uint16_t *)a)[j]; break;
          default: v = ((const uint32_t *)a)[j]; break;
        }
      }
    }
    r[u] = v;
  }
}

struct TileSums {
  double s[kCentreRound], a[kCentreRound];
  int q[kCentreRound];
  __int128 i[kCentreRound];
};

template <typename R>
__device__ inline void tile_summary_r(const void *a, int dt, int64_t j0, int64_t hi, int lane, TileSums &ts, int t) {
  R r[kCentreBatch];
  load_strided<R>(a, elem_bytes(dt), j0, hi, lane, r);
  if (float_dtype(dt)) {
    double sum = 0.0, abs = 0.0;
    int q = kNoExp;
#pragma unroll
    for (int u = 0; u < kCentreBatch; u++) {
      double w[1];
      const R one[1] = {r[u]};
      convert_raw(one, dt, w);
      if (j0 + u * 64 + lane < hi) {
        sum += w[0];
        abs += __builtin_fabs(w[0]);
        if (w[0] != 0.0) {
          const int e = trailing_exp(w[0]);
          q = e < q ? e : q;
        }
      }
    }
    sum = wave_sum_dbl(sum);
    abs = wave_sum_dbl(abs);
    q = wave_min_int(q);
    if (lane == 0) {
      ts.s[t] = sum;
      ts.a[t] = abs;
      ts.q[t] = q;
    }
  } else {
    uint64_t r64[kCentreBatch];
#pragma unroll
    for (int u = 0; u < kCentreBatch; u++) r64[u] = (uint64_t)r[u];
    __int128 acc = 0;
    add_int_raw(r64, dt, 0, kCentreBatch, acc);  // elements past hi were loaded as 0
    acc = wave_sum_i128(acc);
    if (lane == 0) ts.i[t] = acc;
  }
}

// Summary of tile [j0, min(j0 + kCentreTile, hi)) of one coordinate (sum,
// sum of |v| and smallest exponent, or the exact integer sum), written to
// slot t by lane 0.
__device__ inline void tile_summary(const void *a, int dt, int64_t j0, int64_t hi, int lane, TileSums &ts, int t) {
  if (elem_bytes(dt) == 8)
    tile_summary_r<uint64_t>(a, dt, j0, hi, lane, ts, t);
  else
    tile_summary_r<uint32_t>(a, dt, j0, hi, lane, ts, t);
}

// Wavefront 0: the sequential sum continued over tile j0 point by point in
// index order, exact runs of 16 points added at once.
__device__ __noinline__ double fold_tile_points(const void *a, int dt, int64_t j0, int64_t hi, int lane, double run,
                                                double *buf) {
#pragma unroll
  for (int u = 0; u < kCentreBatch; u++) {
    const int64_t j = j0 + u * 64 + lane;
    buf[u * 64 + lane] = j < hi ? dbl_val(a, dt, j) : 0.0;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  const int c = (int)(hi - j0 < kCentreTile ? hi - j0 : kCentreTile);
  // segment of lane l: tile positions 16 l .. 16 l + 15
  double sum = 0.0, abs = 0.0;
  int q = kNoExp;
  for (int u = 0; u < kCentreBatch; u++) {
    const int i = lane * kCentreBatch + u;
    if (i < c) {
      const double w = buf[i];
      sum += w;
      abs += __builtin_fabs(w);
      if (w != 0.0) {
        const int e = trailing_exp(w);
        q = e < q ? e : q;
      }
    }
  }
  for (int l = 0; l * kCentreBatch < c; l++) {
    const double ls = __shfl(sum, l, 64), la = __shfl(abs, l, 64);
    const int lq = __shfl(q, l, 64);
    if (adds_exactly(run, la, lq)) {
      run += ls;
    } else {
      const int e = (l + 1) * kCentreBatch < c ? (l + 1) * kCentreBatch : c;
      for (int i = l * kCentreBatch; i < e; i++) run += buf[i];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  return run;
}

// Per-lane running summary of the points a lane reads.
struct LaneSum {
  double s, a;
  int q;
  __int128 i;
};
__device__ inline LaneSum lane_sum_zero() {
  LaneSum z;
  z.s = 0.0;
  z.a = 0.0;
  z.q = kNoExp;
  z.i = 0;
  return z;
}

template <typename R>
__device__ inline void lane_accumulate_r(const void *a, int dt, int64_t j0, int64_t hi, int lane, LaneSum &ls) {
  R r[kCentreBatch];
  load_strided<R>(a, elem_bytes(dt), j0, hi, lane, r);
  if (float_dtype(dt)) {
#pragma unroll
    for (int u = 0; u < kCentreBatch; u++) {
      double w[1];
      const R one[1] = {r[u]};
      convert_raw(one, dt, w);
      if (j0 + u * 64 + lane < hi) {
        ls.s += w[0];
        ls.a += __builtin_fabs(w[0]);
        if (w[0] != 0.0) {
          const int e = trailing_exp(w[0]);
          ls.q = e < ls.q ? e : ls.q;
        }
      }
    }
  } else {
    uint64_t r64[kCentreBatch];
#pragma unroll
    for (int u = 0; u < kCentreBatch; u++) r64[u] = (uint64_t)r[u];
    add_int_raw(r64, dt, 0, kCentreBatch, ls.i);  // elements past hi were loaded as 0
  }
}

__device__ inline void lane_accumulate(const void *a, int dt, int64_t j0, int64_t hi, int lane, LaneSum &ls) {
  if (elem_bytes(dt) == 8)
    lane_accumulate_r<uint64_t>(a, dt, j0, hi, lane, ls);
  else
    lane_accumulate_r<uint32_t>(a, dt, j0, hi, lane, ls);
}

// Workgroup-wide sum of the lane summaries (a fixed tree order), in thread 0.
template <int W>
__device__ inline LaneSum block_sum(LaneSum v, int lane, int wv, LaneSum *red) {
  v.s = wave_sum_dbl(v.s);
  v.a = wave_sum_dbl(v.a);
  v.q = wave_min_int(v.q);
  v.i = wave_sum_i128(v.i);
  if (lane == 0) red[wv] = v;
  __syncthreads();
  LaneSum t = red[0];
  for (int w = 1; w < W; w++) {
    t.s += red[w].s;
    t.a += red[w].a;
    t.q = red[w].q < t.q ? red[w].q : t.q;
    t.i += red[w].i;
  }
  __syncthreads();
  return t;
}

// The sequential sum of one float coordinate over [lo, hi), tile by tile
// (wavefront 0 folds what the workgroup summarised), for buckets whose whole
// sum is not exact.
template <int W>
__device__ double bucket_sum_by_tiles(const void *a, int dt, int64_t lo, int64_t hi, int lane, int wv, TileSums &ts,
                                      double *buf) {
  const int64_t ntiles = (hi - lo + kCentreTile - 1) / kCentreTile;
  double run = 0.0;
  for (int64_t r0 = 0; r0 < ntiles; r0 += kCentreRound) {
    const int rn = (int)(ntiles - r0 < kCentreRound ? ntiles - r0 : kCentreRound);
    for (int t = wv; t < rn; t += W) tile_summary(a, dt, lo + (r0 + t) * kCentreTile, hi, lane, ts, t);
    __syncthreads();
    if (wv == 0) {
      for (int t0 = 0; t0 < rn; t0 += 64) {
        const int t = t0 + lane;
        const double ms = t < rn ? ts.s[t] : 0.0, ma = t < rn ? ts.a[t] : 0.0;
        const int mq = t < rn ? ts.q[t] : kNoExp;
        const int e = rn - t0 < 64 ? rn - t0 : 64;
        for (int i = 0; i < e; i++) {
          const double sa = __shfl(ma, i, 64);
          const int sq = __shfl(mq, i, 64);
          if (adds_exactly(run, sa, sq))
            run += __shfl(ms, i, 64);
          else
            run = fold_tile_points(a, dt, lo + (r0 + t0 + i) * kCentreTile, hi, lane, run, buf);
        }
      }
    }
    __syncthreads();
  }
  return run;  // meaningful in wavefront 0
}

template <int W>
__global__ __launch_bounds__(64 * W) void k_centres_block(LttbParams p) {
  __shared__ TileSums tsum;
  __shared__ double buf[kCentreTile];   // a tile in index order (fallback)
  __shared__ LaneSum red[W];
  __shared__ int exact_sh[2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t m = p.m, nb = p.n_out - 2;
  const int64_t k = blockIdx.x;
  if (k == nb - 1) {
    if (threadIdx.x == 0) {
      p.cx[k] = X_of(p, m - 1);
      p.cy[k] = Y_of(p, m - 1);
    }
    return;
  }
  const int64_t lo = bucket_start(k + 1, m, nb), hi = bucket_start(k + 2, m, nb);
  const bool hx = p.x_dtype != TS_NONE;
  const bool fx = hx && float_dtype(p.x_dtype), fy = float_dtype(p.y_dtype);
  const int64_t ntiles = (hi - lo + kCentreTile - 1) / kCentreTile;
  // Whole bucket: lane summaries over tiles wv, wv + W, ...
  LaneSum ly = lane_sum_zero(), lx = lane_sum_zero();
  for (int64_t t = wv; t < ntiles; t += W) {
    const int64_t j0 = lo + t * kCentreTile;
    lane_accumulate(p.y, p.y_dtype, j0, hi, lane, ly);
    if (hx) lane_accumulate(p.x, p.x_dtype, j0, hi, lane, lx);
  }
  const LaneSum by = block_sum<W>(ly, lane, wv, red);
  const LaneSum bx = hx ? block_sum<W>(lx, lane, wv, red) : lane_sum_zero();
  // The sum in any order equals the sequential one when no partial sum can
  // round; otherwise fold tile by tile.
  if (threadIdx.x == 0) {
    exact_sh[0] = !fy || adds_exactly(0.0, by.a, by.q);
    exact_sh[1] = !fx || adds_exactly(0.0, bx.a, bx.q);
  }
  __syncthreads();
  double sy = by.s, sx = bx.s;
  if (!exact_sh[0]) sy = bucket_sum_by_tiles<W>(p.y, p.y_dtype, lo, hi, lane, wv, tsum, buf);
  if (!exact_sh[1]) sx = bucket_sum_by_tiles<W>(p.x, p.x_dtype, lo, hi, lane, wv, tsum, buf);
  if (threadIdx.x == 0) {
    const double cnt = (double)(hi - lo);
    p.cy[k] = fy ? sy / cnt : i128_to_double(by.i) / cnt;
    if (!hx)
      p.cx[k] = i128_to_double(((__int128)lo + (__int128)hi - 1) * (__int128)(hi - lo) / 2) / cnt;
    else
      p.cx[k] = fx ? sx / cnt : i128_to_double(bx.i) / cnt;
  }
}

hipError_t launch_lttb_centres(const LttbParams &p, hipStream_t st) {
  const int64_t nb = p.n_out - 2;
  if (!p.sel && p.m >= 0 && (p.m - 2) / nb >= kHullMinBucket) {
    if ((p.m - 2) / nb >= 8 * kCentreTile)
      k_centres_block<8><<<dim3((unsigned)nb), dim3(512), 0, st>>>(p);
    else
      k_centres_block<2><<<dim3((unsigned)nb), dim3(128), 0, st>>>(p);
  } else
    k_centres<<<dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st>>>(p);
  return hipGetLastError();
}

// MinMaxLTTB candidates' coordinates as 64-bit words (exact integers, or the
// doubles the walk uses), one thread per candidate: the centres and the map
// then read contiguous arrays instead of going through the index list.
__global__ __launch_bounds__(256) void k_lttb_gather(LttbParams p) {
  const int64_t m = points_m(p);
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int64_t s = src_of(p, j);
  p.gx[j] = coord_word(p.x, p.x_dtype, s);
  p.gy[j] = coord_word(p.y, p.y_dtype, s);
}

hipError_t launch_lttb_gather(const LttbParams &p, hipStream_t st) {
  if (p.m_max <= 0) return hipSuccess;
  k_lttb_gather<<<dim3((unsigned)((p.m_max + 255) / 256)), dim3(256), 0, st>>>(p);
  return hipGetLastError();
}

// ---------------------------------------------------------------- small

// The transition map of every anchor, one thread each over the whole GPU
// (the map is the bulk of the small-bucket walk: a few dependent loads per
// anchor through the candidate list), into p.next in global memory.  OWN:
// each anchor computes the centre it needs itself (the same sequential
// mean), so no centre pass runs before the map.
template <bool OWN>
__global__ __launch_bounds__(256) void k_lttb_map(LttbParams p) {
  const int64_t m = points_m(p);
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m <= p.n_out || a >= m - 1) return;
  p.next[a] = lttb_map_one(p, m, a, OWN);
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
    copy_map(p.next, smem, m - 1);
    next = smem;
    jump = smem + p.m_max;
    __syncthreads();
  }
  lttb_walk_map(p, m, next, jump, group);
}

hipError_t launch_lttb_small(const LttbParams &p, bool own_centres, hipStream_t st) {
  const int32_t group = lttb_group_len(p.n_out - 2);
  const size_t lds = (size_t)p.m_max * 2 * sizeof(int32_t);
  const int lds_ok = lds <= kWalkMapLds;
  const dim3 grid((unsigned)((p.m_max + 255) / 256));
  if (own_centres)
    k_lttb_map<true><<<grid, dim3(256), 0, st>>>(p);
  else
    k_lttb_map<false><<<grid, dim3(256), 0, st>>>(p);
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
// parallel (one wavefront per bucket: lanes 0-31 run the upper monotone
// chains of 32 slices and lanes 32-63 the lower ones, 16 lanes merge groups
// of 4 slices, one lane per chain merges the groups), and the walk only
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
// Slices per bucket: lane l < 32 builds the upper chain of slice l, lane
// 32 + l the lower chain of the same slice.
constexpr int kHullSlices = 32;

// Chain entries keep Y as a float when every value of the series' dtype is a
// float (exact), else as a double.
__host__ __device__ constexpr bool hull_float_y(int dt) {
  return dt == TS_I8 || dt == TS_U8 || dt == TS_I16 || dt == TS_U16 || dt == TS_F16 || dt == TS_F32;
}

// A chain entry: offset from the bucket start, Y and, with x, X (without x,
// X is the offset).
template <bool HX, typename YS>
struct HullEntry {
  int32_t o;
  YS y;
  double x;
};
template <typename YS>
struct HullEntry<false, YS> {
  int32_t o;
  YS y;
};

// Monotone chain over points added in index order, its stack in LDS (entry i
// at [i * stride], so the stacks of a wavefront's lanes interleave).  sg = +1
// keeps the upper hull (pops on clockwise or collinear turns), sg = -1 the
// lower hull; negating a product or a Y is exact, so both use one test.
template <bool HX, typename YS>
struct HullChain {
  using E = HullEntry<HX, YS>;
  E *s;
  int n, cap, stride;
  double sg;
  bool over;
  // the top two entries are also kept in registers: a push reads no LDS and a
  // pop reads only the entry that becomes second
  double tx, ty, ux, uy;
  __device__ HullChain(E *st, int capacity, int str, bool upper)
      : s(st), n(0), cap(capacity), stride(str), sg(upper ? 1.0 : -1.0), over(false), tx(0), ty(0), ux(0), uy(0) {}
  __device__ static double ex(const E &e) {
    if constexpr (HX)
      return e.x;
    else
      return (double)e.o;
  }
  __device__ E at(int i) const { return s[i * stride]; }
  __device__ void put(int i, int32_t o, double x, double y) {
    E e;
    e.o = o;
    e.y = (YS)y;  // exact: Y is a value of the series' dtype
    if constexpr (HX) e.x = x;
    s[i * stride] = e;
  }
  __device__ void pop() {
    n--;
    tx = ux;
    ty = uy;
    if (n >= 2) {
      const E v = at(n - 2);
      ux = ex(v);
      uy = (double)v.y;
    }
  }
  // Branch-free variant for a wavefront of independent chains: at most one
  // pop for a repeated X and kHullPops turn pops per point (further pops are
  // skipped, so the stack may keep extra points but never loses a hull
  // vertex: every pop is justified by two points of the set).  The entries
  // that may become second are read from LDS up front, in one round trip;
  // the turn test of every state the pops can reach is computed at once (the
  // pops taken are the leading run of passed tests), and the point is always
  // stored, at the slot above the top (slot cap, a spare one, when the stack
  // is full), so lanes branch only when a stack fills up: it is then rebuilt
  // with the exact chain (compact) and marked over only if still full.
  __device__ void add_bounded(int32_t j, double xj, double yj) {
    constexpr int K = HX ? kHullPops + 1 : kHullPops;  // without x no X repeats
    // state i (after i pops): second entry U[i], top T[i]; U[i] = entry n-2-i
    double Ux[K + 1], Uy[K + 1];
    Ux[0] = ux;
    Uy[0] = uy;
#pragma unroll
    for (int i = 0; i < K; i++) {
      const int e = n - 3 - i >= 0 ? n - 3 - i : 0;
      const E v = at(e);
      Ux[i + 1] = ex(v);
      Uy[i + 1] = (double)v.y;
    }
    bool tp[K];  // turn pop from state i
#pragma unroll
    for (int i = 0; i < K; i++) {
      const double Tx = i == 0 ? tx : Ux[i - 1], Ty = i == 0 ? ty : Uy[i - 1];
      const double c = sg * cross3(Ux[i], Uy[i], Tx, Ty, xj, yj);  // computed by every lane, no branch
      tp[i] = (n - i >= 2) & (c >= 0.0);
    }
    const bool same = HX && n > 0 && xj == tx;
    const bool act = !over && !(same && !(sg * yj > sg * ty));
    const bool sp = HX && act && same;  // the repeated-X pop
    int k = sp ? 1 : 0;
    bool go = act;
#pragma unroll
    for (int q = 0; q < kHullPops; q++) {
      go = go && (HX && sp ? tp[q + 1 < K ? q + 1 : K - 1] : tp[q]);
      k += go ? 1 : 0;
    }
    // top after the pops: T[k] (T[0] = t, T[i] = U[i-1])
    double nx = tx, ny = ty;
#pragma unroll
    for (int i = 1; i <= K; i++) {
      nx = k == i ? Ux[i - 1] : nx;
      ny = k == i ? Uy[i - 1] : ny;
    }
    const int m = n - k;
    if (act && m == cap) {  // full (no pop taken): rare, the lane branches off
      compact();
      add(j, xj, yj);
      return;
    }
    put(m < cap ? m : cap, j, xj, yj);  // !act with a full stack: the spare slot
    n = act ? m + 1 : m;
    // without a push no pop was taken: the top two stay as they are
    ux = act ? nx : ux;
    uy = act ? ny : uy;
    tx = act ? xj : tx;
    ty = act ? yj : ty;
  }
  // The exact chain over the stored entries, in place: the stack becomes the
  // hull of the points added so far (the bounded pops may have kept extra
  // points; the stored X are strictly increasing, so no repeated X is met).
  __device__ void compact() {
    int w = 0;
    double ax = 0, ay = 0, bx = 0, by = 0;  // second and top of the rebuilt stack
    for (int r = 0; r < n; r++) {
      const E v = at(r);
      const double xr = ex(v), yr = (double)v.y;
      while (w >= 2 && sg * cross3(ax, ay, bx, by, xr, yr) >= 0.0) {
        w--;
        bx = ax;
        by = ay;
        if (w >= 2) {
          const E q = at(w - 2);
          ax = ex(q);
          ay = (double)q.y;
        }
      }
      s[w * stride] = v;
      w++;
      ax = bx;
      ay = by;
      bx = xr;
      by = yr;
    }
    n = w;
    tx = bx;
    ty = by;
    ux = ax;
    uy = ay;
  }
  // Exact monotone chain step (merges and re-reads).
  __device__ void add(int32_t j, double xj, double yj) {
    if (over) return;
    if (HX && n > 0 && xj == tx) {  // same X as the top: keep the first highest (lowest)
      if (!(sg * yj > sg * ty)) return;
      pop();
    }
    while (n >= 2 && sg * cross3(ux, uy, tx, ty, xj, yj) >= 0.0) pop();
    if (n == cap) {
      over = true;
      return;
    }
    put(n, j, xj, yj);
    n++;
    ux = tx;
    uy = ty;
    tx = xj;
    ty = yj;
  }
  __device__ void add_entry(const E &v) { add(v.o, ex(v), (double)v.y); }
};

// Points loaded per lane before they are added (independent loads in flight).
constexpr int kHullBatch = 16;

// Points lo + a .. lo + b - 1 added one by one with the exact chain (the
// re-read of a slice or group whose chain overflowed), loaded in batches.
template <bool HX, typename YS>
__device__ void feed_raw(const LttbParams &p, int64_t lo, int64_t a, int64_t b, HullChain<HX, YS> &h) {
  using RY = typename std::conditional<sizeof(YS) == 4, uint32_t, uint64_t>::type;
  const int ysb = (int)elem_bytes(p.y_dtype), xsb = HX ? (int)elem_bytes(p.x_dtype) : 0;
  for (int64_t j0 = a; j0 < b; j0 += kHullBatch) {
    RY ry[kHullBatch];
    uint64_t rx[HX ? kHullBatch : 1];
    double ys[kHullBatch], xs[kHullBatch];
    load_raw(p.y, ysb, lo + j0, lo + b - 1, ry);
    if constexpr (HX) load_raw(p.x, xsb, lo + j0, lo + b - 1, rx);
    convert_raw(ry, p.y_dtype, ys);
    if constexpr (HX) convert_raw(rx, p.x_dtype, xs);
    for (int u = 0; u < kHullBatch && j0 + u < b; u++) h.add((int32_t)(j0 + u), HX ? xs[u] : (double)(j0 + u), ys[u]);
  }
}

// Group chains of the two-level merge: 8 groups of 4 slices per chain kind.
constexpr int kHullGroup = 32;

template <bool HX, typename YS>
__global__ __launch_bounds__(64) void k_lttb_hull(LttbParams p) {
  using E = HullEntry<HX, YS>;
  using RY = typename std::conditional<sizeof(YS) == 4, uint32_t, uint64_t>::type;
  // lane stacks: entry i of lane l at [i * 64 + l]; entry kHullLane is the spare slot
  __shared__ E ls[64 * (kHullLane + 1)];
  __shared__ int32_t nsl[64];
  // group chains: entry i of group chain c at [i * 16 + c] (c < 8 upper)
  __shared__ E gs[16 * kHullGroup];
  __shared__ int32_t ngr[16];
  __shared__ E ms[2][kHullCand];
  __shared__ int32_t mg_n[2];
  const int lane = threadIdx.x;
  const int64_t m = p.m, nb = p.n_out - 2;
  const int64_t k = blockIdx.x;
  const int64_t lo = bucket_start(k, m, nb), hi = bucket_start(k + 1, m, nb);
  const int64_t len = hi - lo;
  const int ys_bytes = (int)elem_bytes(p.y_dtype), xs_bytes = HX ? (int)elem_bytes(p.x_dtype) : 0;
  // 1. one chain per lane over its slice, batches of points prefetched
  {
    const int sl = lane & (kHullSlices - 1);
    const int64_t s0 = len * sl / kHullSlices, s1 = len * (sl + 1) / kHullSlices;
    HullChain<HX, YS> h(ls + lane, kHullLane, 64, lane < kHullSlices);
    const int64_t full = (len / kHullSlices) / kHullBatch;  // batches every lane has in full
    RY ry[kHullBatch];
    uint64_t rx[HX ? kHullBatch : 1];
    load_raw(p.y, ys_bytes, lo + s0, lo + s1 - 1, ry);
    if constexpr (HX) load_raw(p.x, xs_bytes, lo + s0, lo + s1 - 1, rx);
    int64_t j0 = s0;
    for (int64_t t = 0; t < full; t++, j0 += kHullBatch) {
      double ys[kHullBatch], xs[kHullBatch];
      convert_raw(ry, p.y_dtype, ys);
      if constexpr (HX) convert_raw(rx, p.x_dtype, xs);
      load_raw(p.y, ys_bytes, lo + j0 + kHullBatch, lo + s1 - 1, ry);
      if constexpr (HX) load_raw(p.x, xs_bytes, lo + j0 + kHullBatch, lo + s1 - 1, rx);
      const double xb = (double)j0;  // without x: X of point j0 + u is xb + u, exact
#pragma unroll
      for (int u = 0; u < kHullBatch; u++) h.add_bounded((int32_t)(j0 + u), HX ? xs[u] : xb + (double)u, ys[u]);
    }
    for (; j0 < s1; j0 += kHullBatch) {  // the rest of the slice (lengths differ by one between lanes)
      double ys[kHullBatch], xs[kHullBatch];
      convert_raw(ry, p.y_dtype, ys);
      if constexpr (HX) convert_raw(rx, p.x_dtype, xs);
      load_raw(p.y, ys_bytes, lo + j0 + kHullBatch, lo + s1 - 1, ry);
      if constexpr (HX) load_raw(p.x, xs_bytes, lo + j0 + kHullBatch, lo + s1 - 1, rx);
      const double xb = (double)j0;
#pragma unroll
      for (int u = 0; u < kHullBatch; u++)
        if (j0 + u < s1) h.add_bounded((int32_t)(j0 + u), HX ? xs[u] : xb + (double)u, ys[u]);
    }
    nsl[lane] = h.over ? -1 : h.n;  // -1: the slice's points are re-read
  }
  __syncthreads();
  // 2. lanes 0-15 merge 4 slices each (lanes 0-7 upper, 8-15 lower); a
  //    slice's hull keeps every point of the bucket's hull in the slice
  if (lane < 16) {
    const bool up = lane < 8;
    const int g = lane & 7;
    HullChain<HX, YS> h(gs + lane, kHullGroup, 16, up);
    for (int sl = 4 * g; sl < 4 * g + 4; sl++) {
      const int src = up ? sl : kHullSlices + sl;
      const int32_t cn = nsl[src];
      if (cn < 0) {
        feed_raw<HX>(p, lo, len * sl / kHullSlices, len * (sl + 1) / kHullSlices, h);
        continue;
      }
      for (int e = 0; e < cn; e++) h.add_entry(ls[e * 64 + src]);
    }
    ngr[lane] = h.over ? -1 : h.n;
  }
  __syncthreads();
  // 3. lane 0 merges the upper group chains, lane 1 the lower ones
  if (lane < 2) {
    const bool up = lane == 0;
    HullChain<HX, YS> h(ms[lane], kHullCand, 1, up);
    for (int g = 0; g < 8; g++) {
      const int gi = (up ? 0 : 8) + g;
      const int32_t cn = ngr[gi];
      if (cn >= 0) {
        for (int e = 0; e < cn; e++) h.add_entry(gs[e * 16 + gi]);
        continue;
      }
      for (int sl = 4 * g; sl < 4 * g + 4; sl++) {  // the group's chain overflowed
        const int src = up ? sl : kHullSlices + sl;
        const int32_t sn = nsl[src];
        if (sn < 0) {
          feed_raw<HX>(p, lo, len * sl / kHullSlices, len * (sl + 1) / kHullSlices, h);
          continue;
        }
        for (int e = 0; e < sn; e++) h.add_entry(ls[e * 64 + src]);
      }
    }
    mg_n[lane] = h.over ? -1 : h.n;
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
        const int32_t a = iu < nu ? ms[0][iu].o : INT32_MAX, b = id < nd ? ms[1][id].o : INT32_MAX;
        if (a <= b) {
          put(a, HullChain<HX, YS>::ex(ms[0][iu]), (double)ms[0][iu].y);
          iu++;
          if (a == b) id++;
        } else {
          put(b, HullChain<HX, YS>::ex(ms[1][id]), (double)ms[1][id].y);
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
  const dim3 grid((unsigned)nb), block(64);
  const bool fy = hull_float_y(p.y_dtype);
  if (p.x_dtype == TS_NONE) {
    if (fy)
      k_lttb_hull<false, float><<<grid, block, 0, st>>>(p);
    else
      k_lttb_hull<false, double><<<grid, block, 0, st>>>(p);
  } else {
    if (fy)
      k_lttb_hull<true, float><<<grid, block, 0, st>>>(p);
    else
      k_lttb_hull<true, double><<<grid, block, 0, st>>>(p);
  }
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
// parallel): about 3S + nb/S dependent steps instead of nb.  When the maps
// fit (lds), next[] is first copied to LDS in one round trip, so every
// dependent step is an LDS read, and the picks are recorded there and written
// out by all threads afterwards.  Sets hflag when it has written the result;
// otherwise k_lttb_hull_walk does the walk.
__global__ __launch_bounds__(1024) void k_lttb_hull_chase(LttbParams p, int64_t S, int lds) {
  extern __shared__ uint4 chase_lds[];
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
  const uint8_t *hn = p.hnext;
  uint8_t *hj = p.hjump, *pick = nullptr;
  if (lds) {  // layout: next [nb * kHullCand], jumps [G * kHullCand], picks [nb]
    const int64_t n16 = nb * kHullCand / 16;  // kHullCand is a multiple of 16
    const uint4 *src = (const uint4 *)p.hnext;
    for (int64_t i0 = t; i0 < n16; i0 += 8 * (int64_t)blockDim.x) {
      uint4 v[8];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const int64_t i = i0 + (int64_t)u * blockDim.x;
        v[u] = src[i < n16 ? i : n16 - 1];
      }
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const int64_t i = i0 + (int64_t)u * blockDim.x;
        if (i < n16) chase_lds[i] = v[u];
      }
    }
    hn = (const uint8_t *)chase_lds;
    hj = (uint8_t *)chase_lds + nb * kHullCand;
    pick = hj + G * kHullCand;
    __syncthreads();
  }
  // 1. group exits
  for (int64_t idx = t; idx < G * kHullCand; idx += blockDim.x) {
    const int64_t g = idx / kHullCand, e = idx % kHullCand;
    const int32_t ne = g == 0 ? 1 : p.cand_cnt[g * S - 1];
    if (e >= ne) continue;
    const int64_t k1 = (g + 1) * S < nb ? (g + 1) * S : nb;
    int v = (int)e;
    for (int64_t k = g * S; k < k1; k++) v = hn[k * kHullCand + v];
    hj[g * kHullCand + e] = (uint8_t)v;
  }
  __threadfence_block();
  __syncthreads();
  // 2. chain over the groups
  if (t == 0) {
    int v = 0;
    for (int64_t g = 0; g < G; g++) {
      entry_s[g] = (uint8_t)v;
      v = hj[g * kHullCand + v];
    }
  }
  __syncthreads();
  // 3. picks inside every group
  for (int64_t g = t; g < G; g += blockDim.x) {
    int v = entry_s[g];
    const int64_t k1 = (g + 1) * S < nb ? (g + 1) * S : nb;
    for (int64_t k = g * S; k < k1; k++) {
      v = hn[k * kHullCand + v];
      if (lds)
        pick[k] = (uint8_t)v;
      else
        p.out[k + 1] = p.cand_idx[k * kHullCand + v];
    }
  }
  if (lds) {
    __syncthreads();
    for (int64_t k = t; k < nb; k += blockDim.x) p.out[k + 1] = p.cand_idx[k * kHullCand + pick[k]];
  }
  if (t == 0) {
    p.out[0] = 0;
    p.out[p.n_out - 1] = m - 1;
    *p.out_count = p.n_out;
    *p.hflag = 1;
  }
}

// LDS of the chase when the maps fit (0: the maps stay in global memory).
static size_t chase_lds_bytes(int64_t nb, int64_t S) {
  const int64_t G = (nb + S - 1) / S;
  const size_t b = (size_t)(nb * kHullCand + G * kHullCand + nb);
  return b <= 144 * 1024 ? (b + 15) / 16 * 16 : 0;
}

hipError_t launch_lttb_hull_walk(const LttbParams &p, hipStream_t st) {
  const int64_t nb = p.n_out - 2;
  k_lttb_hull_next<<<dim3((unsigned)nb), dim3(64), 0, st>>>(p);
  const int64_t S = lttb_hull_group(nb);
  const size_t lds = chase_lds_bytes(nb, S);
  k_lttb_hull_chase<<<dim3(1), dim3(1024), lds, st>>>(p, S, lds > 0 ? 1 : 0);
  k_lttb_hull_walk<<<dim3(1), dim3(64), 0, st>>>(p);
  return hipGetLastError();
}

}  // namespace tsds

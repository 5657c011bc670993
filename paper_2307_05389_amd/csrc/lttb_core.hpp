// lttb_core.hpp -- device building blocks of the LTTB bucket walk, shared by
// the single-series kernels (lttb.hip) and the batched kernel
// (batch_lttb.hip).  Every unit that includes it is built with
// -ffp-contract=off and IEEE mode, so the FP64 expressions below are rounded
// exactly as written.
#pragma once

#include "common.hpp"
#include "internal.hpp"

namespace tsds {

__device__ inline int64_t src_of(const LttbParams &p, int64_t j) { return p.sel ? p.sel[j] : j; }

__device__ inline bool int_coord_x(const LttbParams &p) {
  return p.x_dtype == TS_NONE || p.x_dtype == TS_I32 || p.x_dtype == TS_I64 || p.x_dtype == TS_U32 ||
         p.x_dtype == TS_U64;
}
__device__ inline bool int_coord_y(const LttbParams &p) {
  return p.y_dtype != TS_F16 && p.y_dtype != TS_F32 && p.y_dtype != TS_F64;
}

// Bytes of one element of a ts dtype.
__device__ inline int elem_bytes(int dt) {
  switch (dt) {
    case TS_I8: case TS_U8: return 1;
    case TS_I16: case TS_U16: case TS_F16: return 2;
    case TS_I32: case TS_U32: case TS_F32: return 4;
  }
  return 8;
}

// Exact value of an integer element as a 128-bit integer.
__device__ inline __int128 int_val(const void *a, int dt, int64_t s) {
  switch (dt) {
    case TS_I8: return ((const int8_t *)a)[s];
    case TS_I16: return ((const int16_t *)a)[s];
    case TS_I32: return ((const int32_t *)a)[s];
    case TS_I64: return ((const int64_t *)a)[s];
    case TS_U8: return ((const uint8_t *)a)[s];
    case TS_U16: return ((const uint16_t *)a)[s];
    case TS_U32: return ((const uint32_t *)a)[s];
    case TS_U64: return (__int128)((const uint64_t *)a)[s];
  }
  return 0;
}

// Element widened to double: exact for <= 32-bit integers and floats, round
// to nearest for 64-bit integers.
__device__ inline double dbl_val(const void *a, int dt, int64_t s) {
  switch (dt) {
    case TS_I8: return (double)((const int8_t *)a)[s];
    case TS_I16: return (double)((const int16_t *)a)[s];
    case TS_I32: return (double)((const int32_t *)a)[s];
    case TS_I64: return (double)((const int64_t *)a)[s];
    case TS_U8: return (double)((const uint8_t *)a)[s];
    case TS_U16: return (double)((const uint16_t *)a)[s];
    case TS_U32: return (double)((const uint32_t *)a)[s];
    case TS_U64: return (double)((const uint64_t *)a)[s];
    case TS_F16: return (double)(float)__builtin_bit_cast(_Float16, ((const uint16_t *)a)[s]);
    case TS_F32: return (double)((const float *)a)[s];
    case TS_F64: return ((const double *)a)[s];
  }
  return 0.0;
}

// Gathered coordinate words (LttbParams::gx / gy): the exact integer for
// integer dtypes (and the index without x), the double for float dtypes.
__device__ inline bool float_dt(int dt) { return dt == TS_F16 || dt == TS_F32 || dt == TS_F64; }
__device__ inline uint64_t coord_word(const void *a, int dt, int64_t s) {
  if (dt == TS_NONE) return (uint64_t)s;
  if (float_dt(dt)) return __builtin_bit_cast(uint64_t, dbl_val(a, dt, s));
  if (dt == TS_U64) return ((const uint64_t *)a)[s];
  return (uint64_t)(int64_t)int_val(a, dt, s);
}
__device__ inline double word_dbl(uint64_t w, int dt) {
  if (float_dt(dt)) return __builtin_bit_cast(double, w);
  return dt == TS_U64 ? (double)w : (double)(int64_t)w;
}
__device__ inline __int128 word_int(uint64_t w, int dt) {
  return dt == TS_U64 ? (__int128)w : (__int128)(int64_t)w;
}

__device__ inline double X_of(const LttbParams &p, int64_t j) {
  if (p.gx) return word_dbl(p.gx[j], p.x_dtype);
  int64_t s = src_of(p, j);
  return p.x_dtype == TS_NONE ? (double)s : dbl_val(p.x, p.x_dtype, s);
}
__device__ inline double Y_of(const LttbParams &p, int64_t j) {
  if (p.gy) return word_dbl(p.gy[j], p.y_dtype);
  return dbl_val(p.y, p.y_dtype, src_of(p, j));
}

// Round a 128-bit integer to the nearest double (ties to even).  The top 64
// significant bits are kept with every discarded bit folded into the lowest
// kept bit (round-to-odd), which a single correctly rounded 64 -> 53 bit
// conversion then finishes without double rounding.
__device__ inline double i128_to_double(__int128 v) {
  bool neg = v < 0;
  unsigned __int128 u = neg ? (unsigned __int128)(-v) : (unsigned __int128)v;
  uint64_t hi = (uint64_t)(u >> 64), lo = (uint64_t)u;
  double r;
  if (hi == 0) {
    r = (double)lo;
  } else {
    int sh = 64 - __builtin_clzll(hi);  // bits of hi in use, 1..64
    uint64_t top = (sh == 64) ? hi : ((hi << (64 - sh)) | (lo >> sh));
    uint64_t rest = (sh == 64) ? lo : (lo << (64 - sh));
    if (rest) top |= 1;
    r = __builtin_ldexp((double)top, sh);
  }
  return neg ? -r : r;
}

// Mean of X (which == 0) or Y over points [lo, hi), in index order.
__device__ double coord_mean(const LttbParams &p, int which, int64_t lo, int64_t hi) {
  const double cnt = (double)(hi - lo);
  const uint64_t *g = which == 0 ? p.gx : p.gy;
  if (g) {  // gathered words: the same sums, read from contiguous arrays
    const int dt = which == 0 ? p.x_dtype : p.y_dtype;
    if (which == 0 ? int_coord_x(p) : int_coord_y(p)) {
      __int128 s = 0;
      for (int64_t j = lo; j < hi; j++) s += word_int(g[j], dt);
      return i128_to_double(s) / cnt;
    }
    double s = 0.0;
    for (int64_t j = lo; j < hi; j++) s += __builtin_bit_cast(double, g[j]);
    return s / cnt;
  }
  if (which == 0 && p.x_dtype == TS_NONE) {
    __int128 s = 0;
    for (int64_t j = lo; j < hi; j++) s += src_of(p, j);
    return i128_to_double(s) / cnt;
  }
  const void *a = which == 0 ? p.x : p.y;
  const int dt = which == 0 ? p.x_dtype : p.y_dtype;
  if (which == 0 ? int_coord_x(p) : int_coord_y(p)) {
    __int128 s = 0;
    for (int64_t j = lo; j < hi; j++) s += int_val(a, dt, src_of(p, j));
    return i128_to_double(s) / cnt;
  }
  double s = 0.0;
  for (int64_t j = lo; j < hi; j++) s += dbl_val(a, dt, src_of(p, j));
  return s / cnt;
}

// (the host guarantees m * nb < 2^63, so the products fit in 64 bits)
__device__ inline int64_t bucket_start(int64_t k, int64_t m, int64_t nb) {
  return 1 + (int64_t)(((uint64_t)k * (uint64_t)(m - 2)) / (uint64_t)nb);
}

// Bucket holding interior point j (1 <= j <= m-2).
__device__ inline int64_t bucket_of(int64_t j, int64_t m, int64_t nb) {
  int64_t k = (int64_t)(((uint64_t)j * (uint64_t)nb + (uint64_t)(m - 2) - 1) / (uint64_t)(m - 2)) - 1;
  if (k < 0) k = 0;
  if (k > nb - 1) k = nb - 1;
  while (k + 1 < nb && bucket_start(k + 1, m, nb) <= j) k++;
  while (k > 0 && bucket_start(k, m, nb) > j) k--;
  return k;
}

__device__ inline double area2(double XA, double YA, double Xb, double Yb, double Cx, double Cy) {
  return __builtin_fabs((XA - Cx) * (Yb - YA) - (XA - Xb) * (Cy - YA));
}

// Point count: fixed, or read from the device (clamped to the capacity, so a
// count never leads a kernel outside its buffers).
__device__ inline int64_t points_m(const LttbParams &p) {
  if (p.m >= 0) return p.m;
  const int64_t m = *p.m_dev;
  return m < 0 ? 0 : (m > p.m_max ? p.m_max : m);
}

// First point of bucket k (points [lo, hi)) with the largest area against
// anchor A and centre k.
__device__ int64_t best_in_bucket(const LttbParams &p, int64_t lo, int64_t hi, double XA, double YA, double Cx,
                                  double Cy) {
  double best = -1.0;
  int64_t arg = lo;
  for (int64_t b = lo; b < hi; b++) {
    double a = area2(XA, YA, X_of(p, b), Y_of(p, b), Cx, Cy);
    if (a > best) { best = a; arg = b; }
  }
  return arg;
}

__device__ void copy_all(const LttbParams &p, int64_t m) {
  for (int64_t j = threadIdx.x; j < m; j += blockDim.x) p.out[j] = src_of(p, j);
  if (threadIdx.x == 0) *p.out_count = m;
}

// Bucket centres of LTTB over m points, computed by the whole workgroup (one
// thread per bucket, sequential sums inside a bucket).
__device__ inline void lttb_block_centres(const LttbParams &p, int64_t m) {
  const int64_t nb = p.n_out - 2;
  for (int64_t k = threadIdx.x; k < nb; k += blockDim.x) {
    if (k == nb - 1) {
      p.cx[k] = X_of(p, m - 1);
      p.cy[k] = Y_of(p, m - 1);
    } else {
      const int64_t lo = bucket_start(k + 1, m, nb), hi = bucket_start(k + 2, m, nb);
      p.cx[k] = coord_mean(p, 0, lo, hi);
      p.cy[k] = coord_mean(p, 1, lo, hi);
    }
  }
}

// Transition map entry of anchor a (a = 0 stands for the first point, before
// bucket 0): the point of the next bucket the walk picks when the previous
// pick is a.  The centre of that bucket comes from cx/cy when given, else it
// is computed here (the same sequential mean).
__device__ inline int32_t lttb_map_one(const LttbParams &p, int64_t m, int64_t a, bool own_centres) {
  const int64_t nb = p.n_out - 2;
  const int64_t k = a == 0 ? -1 : bucket_of(a, m, nb);
  if (k == nb - 1) return (int32_t)(m - 1);
  const int64_t lo = bucket_start(k + 1, m, nb), hi = bucket_start(k + 2, m, nb);
  double Cx, Cy;
  if (!own_centres) {
    Cx = p.cx[k + 1];
    Cy = p.cy[k + 1];
  } else if (k + 1 == nb - 1) {
    Cx = X_of(p, m - 1);
    Cy = Y_of(p, m - 1);
  } else {
    const int64_t clo = bucket_start(k + 2, m, nb), chi = bucket_start(k + 3, m, nb);
    Cx = coord_mean(p, 0, clo, chi);
    Cy = coord_mean(p, 1, clo, chi);
  }
  return (int32_t)best_in_bucket(p, lo, hi, X_of(p, a), Y_of(p, a), Cx, Cy);
}

// dst[0 .. cnt) = src[0 .. cnt) by the whole workgroup, in 16-byte pieces
// with every piece's load issued before any store (one round trip for maps
// up to 16 pieces per thread).  Both buffers are 16-byte aligned and hold
// cnt rounded up to a multiple of 4.
__device__ inline void copy_map(const int32_t *src, int32_t *dst, int64_t cnt) {
  constexpr int U = 4;
  const int64_t n4 = (cnt + 3) / 4;
  const int4 *s4 = (const int4 *)src;
  int4 *d4 = (int4 *)dst;
  for (int64_t i0 = threadIdx.x; i0 < n4; i0 += (int64_t)U * blockDim.x) {
    int4 v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t i = i0 + (int64_t)u * blockDim.x;
      v[u] = s4[i < n4 ? i : n4 - 1];
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t i = i0 + (int64_t)u * blockDim.x;
      if (i < n4) d4[i] = v[u];
    }
  }
}

// LTTB walk over m > n_out points with buckets of a few points, by the whole
// workgroup, from the transition map next[] (entries 0 .. m-2; see
// lttb_map_one).  jump[] holds m int32 (LDS or global); it takes the group
// exits, then the picks of the buckets (nb < m).
constexpr int64_t kWalkEntriesLds = 2048;
constexpr int64_t kWalkSuperLds = 2048;  // super-group exits (super-groups x entries each)
constexpr int64_t kWalkSupers = 256;

__device__ void lttb_walk_map(const LttbParams &p, int64_t m, const int32_t *next, int32_t *jump, int32_t group) {
  const int64_t nb = p.n_out - 2;
  const int64_t G = (nb + group - 1) / group;
  // group entries: in LDS when they fit (read back right after the chain),
  // else the workspace copy
  __shared__ int32_t s_entry[kWalkEntriesLds];
  int32_t *entry = G <= kWalkEntriesLds ? s_entry : p.entry;

  // 1. group exits: for every possible entry a of group g (the first point
  //    for g = 0, else any point of bucket g*group - 1), follow next[] over
  //    the group's buckets.  (group, entry) pairs are spread over threads.
  const int64_t P = (m - 2 + nb - 1) / nb + 1;  // >= largest bucket
  for (int64_t idx = threadIdx.x; idx < G * P; idx += blockDim.x) {
    const int64_t g = idx / P, off = idx % P;
    const int64_t lo = g == 0 ? 0 : bucket_start(g * group - 1, m, nb);
    const int64_t hi = g == 0 ? 1 : bucket_start(g * group, m, nb);
    const int64_t a = lo + off;
    if (a >= hi) continue;
    const int64_t k1 = (g + 1) * group < nb ? (g + 1) * group : nb;
    int32_t v = (int32_t)a;
    for (int64_t s = g * group; s < k1; s++) v = next[v];
    jump[a] = v;
  }
  __syncthreads();

  // 2. chain over groups.  With many groups, in two levels: super-groups of
  //    T groups get their exits for every possible entry in parallel (2a),
  //    one thread chains the H super-groups (2b), and each super-group's
  //    group entries follow in parallel (2c): 2T + H dependent reads
  //    instead of G.
  int64_t T = 1;
  while (T * T < G) T++;
  const int64_t H = (G + T - 1) / T;
  __shared__ int32_t s_sup[kWalkSuperLds];
  __shared__ int64_t s_slo[kWalkSupers];
  __shared__ int32_t s_sent[kWalkSupers];
  if (T > 1 && H <= kWalkSupers && H * P <= kWalkSuperLds) {
    for (int64_t h = threadIdx.x; h < H; h += blockDim.x)
      s_slo[h] = h == 0 ? 0 : bucket_start(h * T * group - 1, m, nb);
    for (int64_t idx = threadIdx.x; idx < H * P; idx += blockDim.x) {
      const int64_t h = idx / P, off = idx % P;
      const int64_t lo = h == 0 ? 0 : bucket_start(h * T * group - 1, m, nb);
      const int64_t hi = h == 0 ? 1 : bucket_start(h * T * group, m, nb);
      const int64_t a = lo + off;
      if (a >= hi) continue;
      const int64_t g1 = (h + 1) * T < G ? (h + 1) * T : G;
      int32_t v = (int32_t)a;
      for (int64_t g = h * T; g < g1; g++) v = jump[v];
      s_sup[idx] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t v = 0;
      for (int64_t h = 0; h < H; h++) {
        s_sent[h] = v;
        v = s_sup[h * P + (v - s_slo[h])];
      }
    }
    __syncthreads();
    for (int64_t h = threadIdx.x; h < H; h += blockDim.x) {
      int32_t v = s_sent[h];
      const int64_t g1 = (h + 1) * T < G ? (h + 1) * T : G;
      for (int64_t g = h * T; g < g1; g++) {
        entry[g] = v;
        v = jump[v];
      }
    }
  } else if (threadIdx.x == 0) {
    int32_t v = 0;
    for (int64_t g = 0; g < G; g++) {
      entry[g] = v;
      v = jump[v];
    }
  }
  __syncthreads();

  // 3. group interiors in parallel; the picks go to jump[] (free again), then
  //    every thread writes outputs, so the index loads behind them are
  //    independent of the chain.
  for (int64_t g = threadIdx.x; g < G; g += blockDim.x) {
    int32_t v = entry[g];
    const int64_t k1 = (g + 1) * group < nb ? (g + 1) * group : nb;
    for (int64_t k = g * group; k < k1; k++) {
      v = next[v];
      jump[k] = v;
    }
  }
  __syncthreads();
  for (int64_t k = threadIdx.x; k < nb; k += blockDim.x) p.out[k + 1] = src_of(p, jump[k]);
  if (threadIdx.x == 0) {
    p.out[0] = src_of(p, 0);
    p.out[p.n_out - 1] = src_of(p, m - 1);
    *p.out_count = p.n_out;
  }
}

// The whole small-bucket walk in one workgroup: the map (all anchors in
// parallel), then lttb_walk_map.  next[] and jump[] hold m_max int32 each.
__device__ void lttb_small_walk(const LttbParams &p, int64_t m, int32_t *next, int32_t *jump, int32_t group) {
  for (int64_t a = threadIdx.x; a < m - 1; a += blockDim.x) next[a] = lttb_map_one(p, m, a, false);
  __syncthreads();
  lttb_walk_map(p, m, next, jump, group);
}

// Buckets per group of the walk: the smallest power of two S with 2 S^3 >= nb
// (the group and super-group chains then stay near nb^(1/3) each).
__host__ __device__ inline int32_t lttb_group_len(int64_t nb) {
  int32_t group = 1;
  while ((int64_t)group * group * group * 2 < nb) group *= 2;
  return group;
}

}  // namespace tsds

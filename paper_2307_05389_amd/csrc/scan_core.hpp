// scan_core.hpp -- device body of the argmin/argmax scan (one chunk of one
// series per wavefront), shared by the single-series kernel (scan.hip) and
// the batched persistent kernel (batch.hip).  See scan.hip for the design.
#pragma once

#include <limits>
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace tsds {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ edges
//
// Start of bin b (0 <= b <= nb) over a sorted x: the first index whose x is
// >= the bin's edge value (a left search-sorted, Sec. 2.2), edges[0] = 0 and
// edges[nb] = n.  Integer x: edge value x0 + ceil(b R / nb), R = x_last - x0,
// exact.  Float x: x0 + ((double)b R) / nb, each operation rounded to
// nearest (the unit is built without FMA contraction).

template <typename X> struct XKey;
template <> struct XKey<int32_t> { using K = int64_t; };
template <> struct XKey<int64_t> { using K = int64_t; };
template <> struct XKey<uint32_t> { using K = uint64_t; };
template <> struct XKey<uint64_t> { using K = uint64_t; };
template <> struct XKey<float> { using K = double; };
template <> struct XKey<double> { using K = double; };

// ceil(b * R / nb) exactly although b*R may need 128 bits: with R = q*nb + r,
// b*R/nb = b*q + b*r/nb, and b*r < nb^2 < 2^64 (the host keeps nb < 2^31).
__device__ inline uint64_t ceil_mul_div(uint64_t b, uint64_t R, uint64_t nb) {
  uint64_t q = R / nb, r = R % nb;
  uint64_t br = b * r;
  uint64_t t = br / nb;
  return b * q + t + (t * nb == br ? 0 : 1);
}

// Wavefront-cooperative lower bound: the first index i in [lo, hi) with
// x[i] >= v (hi if none).  Each round probes 64 evenly spaced positions.
template <typename X, typename K>
__device__ int64_t wave_lower_bound(const X *x, int64_t lo, int64_t hi, K v, int lane) {
  while (hi > lo) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t q = lo + (int64_t)lane * step;
    const bool less = q < hi && (K)x[q] < v;
    const int cnt = __builtin_popcountll(ballot(less));  // lanes 0..cnt-1 are below v
    if (cnt == 0) {
      hi = lo;
    } else {
      const int64_t nlo = lo + (int64_t)(cnt - 1) * step + 1;
      const int64_t nhi = lo + (int64_t)cnt * step;
      lo = nlo;
      hi = nhi < hi ? nhi : hi;
    }
  }
  return lo;
}

template <typename X>
__device__ inline typename XKey<X>::K edge_value(X x0, X xl, int64_t nb, int64_t b) {
  using K = typename XKey<X>::K;
  if constexpr (std::is_floating_point<X>::value) {
    const double d0 = (double)x0, R = (double)xl - d0;
    return d0 + ((double)b * R) / (double)nb;
  } else {
    const uint64_t R = (uint64_t)(K)xl - (uint64_t)(K)x0;  // exact modulo 2^64, x sorted
    return (K)((uint64_t)(K)x0 + ceil_mul_div((uint64_t)b, R, (uint64_t)nb));
  }
}

template <typename X>
__device__ int64_t edge_start(const X *x, int64_t n, int64_t nb, int64_t b, int lane) {
  using K = typename XKey<X>::K;
  if (b >= nb) return n;
  if (b == 0 || n == 0) return 0;
  const K E = edge_value<X>(x[0], x[n - 1], nb, b);
  return wave_lower_bound<X, K>(x, 0, n, E, lane);
}


// ------------------------------------------------------------------ scan

// ceil(b N / nb) for 0 <= b <= nb < 2^31 without a 64-bit division (a long
// instruction sequence on this GPU): N = q nb + r is split once, with q from
// a double-precision estimate corrected exactly; b r < nb^2 < 2^62 is then
// divided by a double multiply with 1/nb (off by at most one) and corrected
// exactly.  Products wrap modulo 2^64, so only the small remainders matter.
struct CeilMulDiv {
  uint64_t q, r;
  int64_t nb;
  double inv_nb;
  __device__ CeilMulDiv(uint64_t N, int64_t nb_) : nb(nb_) {
    inv_nb = 1.0 / (double)nb;
    const double qd = (double)N * inv_nb;  // |error| < 2^13
    int64_t qe = qd >= 18446744073709551615.0 ? (int64_t)~0ull : (int64_t)(uint64_t)qd;
    int64_t rem = (int64_t)(N - (uint64_t)qe * (uint64_t)nb);  // |rem| < 2^45
    qe += (int64_t)floor((double)rem * inv_nb);
    rem = (int64_t)(N - (uint64_t)qe * (uint64_t)nb);
    while (rem < 0) { qe--; rem += nb; }
    while (rem >= nb) { qe++; rem -= nb; }
    q = (uint64_t)qe;
    r = (uint64_t)rem;
  }
  __device__ uint64_t at(int64_t b) const {
    const uint64_t br = (uint64_t)b * r;
    int64_t t = (int64_t)((double)br * inv_nb);
    int64_t rem = (int64_t)(br - (uint64_t)t * (uint64_t)nb);
    while (rem < 0) { t--; rem += nb; }
    while (rem >= nb) { t++; rem -= nb; }
    return (uint64_t)b * q + (uint64_t)t + (rem != 0 ? 1u : 0u);
  }
};

// Closed-form bins of a series without x: bin b starts at ceil(b (n-1) / nb).
__device__ inline CeilMulDiv closed_bins(int64_t n, int64_t nb) { return CeilMulDiv(n > 0 ? (uint64_t)(n - 1) : 0u, nb); }

// Start of bin b (b <= nb); b >= nb gives the end of the last bin.  `cm` is
// closed_bins(n, nb) (used only when edges is NULL).
__device__ inline int64_t edge_at(const int64_t *edges, const CeilMulDiv &cm, int64_t n, int64_t nb, int64_t b) {
  if (b >= nb) return edges ? edges[nb] : n;
  if (edges) return edges[b];
  return (int64_t)cm.at(b);
}

// First bin whose range can intersect [c0, ...): the last b with start <= c0.
__device__ int64_t first_bin(const int64_t *edges, const CeilMulDiv &cm, int64_t n, int64_t nb, int64_t c0,
                             int lane) {
  if (!edges) {
    if (n <= 1) return 0;
    // start(b) <= c0  <=>  b <= c0 nb / (n-1): estimate, then correct exactly
    const double est = (double)c0 * (double)nb / (double)(n - 1);
    int64_t b = 0;
    if (est >= 1.0) b = est >= (double)(nb - 1) ? nb - 1 : (int64_t)est;
    while (b + 1 < nb && (int64_t)cm.at(b + 1) <= c0) b++;
    while (b > 0 && (int64_t)cm.at(b) > c0) b--;
    return b;
  }
  if (edges[0] > c0) return 0;
  int64_t lo = 0, hi = nb;  // edges[lo] <= c0; the answer is < hi
  while (hi - lo > 1) {
    int64_t step = (hi - lo + 63) / 64;
    int64_t q = lo + (int64_t)lane * step;
    bool le = q < hi && edges[q] <= c0;
    int cnt = __builtin_popcountll(ballot(le));
    int64_t nlo = lo + (int64_t)(cnt - 1) * step;
    int64_t nhi = lo + (int64_t)cnt * step;
    lo = nlo;
    hi = nhi < hi ? nhi : hi;
  }
  return lo;
}

template <typename T>
__device__ inline typename Elem<T>::C extract(const u32x4 &d, int j) {
  constexpr int VEC = 16 / (int)sizeof(T);
  T tmp[VEC];
  __builtin_memcpy(tmp, &d, 16);
  return Elem<T>::load(&tmp[j]);
}

template <typename T>
__device__ inline void write_result(const ScanParams &p, int64_t c, int64_t bin, bool before, bool after,
                                    typename Elem<T>::C vmn, int64_t imn, typename Elem<T>::C vmx,
                                    int64_t imx) {
  if (!before && !after) {
    p.binres[2 * bin] = imn;
    p.binres[2 * bin + 1] = imx;
  } else {
    Partial q;
    q.kmin = Elem<T>::key(vmn);
    q.imin = imn;
    q.kmax = Elem<T>::key(vmx);
    q.imax = imx;
    (before ? p.partL : p.partR)[c] = q;
  }
}

// ---- per-vector reductions and searches ------------------------------------
//
// A tile is U 16-byte vectors per lane; vector u of lane l holds tile
// positions (u*64 + l)*VEC + j, j < VEC, so tile order is (u, lane, j).
// VecOps<T>::minmax reduces one vector to its minimum and maximum value;
// narrow types use packed 16-bit min/max (two elements per instruction),
// bytes being spread into two 16-bit pairs first (signed bytes biased by 0x80
// so that unsigned order is numeric order).  VecOps<T>::first returns the
// first j whose element equals a value (VEC if none); bytes and halves test
// four or two elements per instruction with the zero-lane bit trick.

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

template <typename V>
__device__ inline V as2(uint32_t w) { return __builtin_bit_cast(V, w); }

// Lowest 8-bit (B = 8) or 16-bit (B = 16) lane of t that is zero, or -1.
template <int B>
__device__ inline int first_zero_lane(uint32_t t) {
  constexpr uint32_t ONES = B == 8 ? 0x01010101u : 0x00010001u;
  constexpr uint32_t HIGH = B == 8 ? 0x80808080u : 0x80008000u;
  const uint32_t z = (t - ONES) & ~t & HIGH;  // lowest set bit marks the lowest zero lane
  return z ? (int)(__builtin_ctz(z) / B) : -1;
}

template <typename T> struct VecOps {
  using C = typename Elem<T>::C;
  static constexpr int VEC = 16 / (int)sizeof(T);
  static __device__ inline void minmax(const u32x4 &d, C &mn, C &mx) {
    mn = extract<T>(d, 0);
    mx = mn;
#pragma unroll
    for (int j = 1; j < VEC; j++) {
      const C v = extract<T>(d, j);
      mn = vmin(mn, v);
      mx = vmax(mx, v);
    }
  }
  static __device__ inline int first(const u32x4 &d, C target) {
    int r = VEC;
#pragma unroll
    for (int j = VEC - 1; j >= 0; j--)
      if (extract<T>(d, j) == target) r = j;
    return r;
  }
};

// Bits [lo, hi) of a 64-bit word (bounds clamped to [0, 64]).
__device__ inline uint64_t bit_range64(int lo, int hi) {
  lo = lo < 0 ? 0 : lo > 64 ? 64 : lo;
  hi = hi < 0 ? 0 : hi > 64 ? 64 : hi;
  const uint64_t below_hi = hi >= 64 ? ~0ull : (1ull << hi) - 1;
  const uint64_t below_lo = lo >= 64 ? ~0ull : (1ull << lo) - 1;
  return below_hi & ~below_lo;
}

// First element j in [a, b) of a vector of B-bit lanes (B = 8 or 16) whose
// bits, under magmask, equal the repeated pattern; 128 / B if none.  Each
// dword takes the exact zero-lane test (7-bit sums: no borrow from one lane
// into the next, so every lane's flag is exact, not only the lowest), the
// flags of lanes outside [a, b) are cleared with a bit range over the two
// 64-bit halves, and the lowest flag left is the answer.  Branch-free, with
// no test per element.
template <int B>
__device__ inline int first_equal_in(const u32x4 &d, uint32_t pat, uint32_t magmask, int a, int b) {
  constexpr uint32_t LOW = B == 8 ? 0x7f7f7f7fu : 0x7fff7fffu;
  uint32_t z[4];
#pragma unroll
  for (int c = 0; c < 4; c++) {
    const uint32_t t = (d[c] & magmask) ^ pat;
    z[c] = ~(((t & LOW) + LOW) | t | LOW);  // top bit of a lane set iff the lane is zero
  }
  const uint64_t zlo = (uint64_t)z[1] << 32 | z[0], zhi = (uint64_t)z[3] << 32 | z[2];
  const uint64_t mlo = zlo & bit_range64(a * B, b * B), mhi = zhi & bit_range64(a * B - 64, b * B - 64);
  if (mlo) return __builtin_ctzll(mlo) / B;
  if (mhi) return (64 + __builtin_ctzll(mhi)) / B;
  return 128 / B;
}

template <typename V>
__device__ inline void pk_vec_minmax(const u32x4 &d, V &a, V &b) {
  a = as2<V>(d.x);
  b = a;
#pragma unroll
  for (int c = 1; c < 4; c++) {
    const V v = as2<V>(d[c]);
    a = __builtin_elementwise_min(a, v);
    b = __builtin_elementwise_max(b, v);
  }
}

template <typename T, uint32_t SIGNMASK>
__device__ inline int first16(const u32x4 &d, uint32_t pattern16) {
  const uint32_t pat = pattern16 | (pattern16 << 16);
#pragma unroll
  for (int c = 0; c < 4; c++) {
    const int k = first_zero_lane<16>((d[c] & ~SIGNMASK) ^ pat);
    if (k >= 0) return 2 * c + k;
  }
  return 8;
}

template <> struct VecOps<uint16_t> {
  static __device__ inline void minmax(const u32x4 &d, uint32_t &mn, uint32_t &mx) {
    u16x2 a, b;
    pk_vec_minmax(d, a, b);
    mn = a.x < a.y ? a.x : a.y;
    mx = b.x < b.y ? b.y : b.x;
  }
  static __device__ inline int first(const u32x4 &d, uint32_t t) { return first16<uint16_t, 0u>(d, t & 0xffffu); }
};
template <> struct VecOps<int16_t> {
  static __device__ inline void minmax(const u32x4 &d, int32_t &mn, int32_t &mx) {
    i16x2 a, b;
    pk_vec_minmax(d, a, b);
    mn = a.x < a.y ? a.x : a.y;
    mx = b.x < b.y ? b.y : b.x;
  }
  static __device__ inline int first(const u32x4 &d, int32_t t) {
    return first16<int16_t, 0u>(d, (uint32_t)t & 0xffffu);
  }
};
template <> struct VecOps<half_t> {
  static __device__ inline void minmax(const u32x4 &d, _Float16 &mn, _Float16 &mx) {
    f16x2 a, b;
    pk_vec_minmax(d, a, b);
    mn = vmin(a.x, a.y);
    mx = vmax(b.x, b.y);
  }
  // Equal values have equal bits except for the two zeros: a zero target
  // compares magnitudes only.
  static __device__ inline int first(const u32x4 &d, _Float16 t) {
    const uint32_t bits = __builtin_bit_cast(uint16_t, t);
    if ((bits & 0x7fffu) == 0) return first16<half_t, 0x80008000u>(d, 0u);
    return first16<half_t, 0u>(d, bits);
  }
};

// Bytes: w = [b0 b1 b2 b3] -> (b0, b2) and (b1, b3) as 16-bit pairs.
template <uint32_t BIAS>
__device__ inline void byte_vec_minmax(const u32x4 &d, uint32_t &mn, uint32_t &mx) {
  u16x2 a, b;
#pragma unroll
  for (int c = 0; c < 4; c++) {
    const uint32_t w = d[c] ^ BIAS;
    const u16x2 lo = as2<u16x2>(w & 0x00ff00ffu), hi = as2<u16x2>((w >> 8) & 0x00ff00ffu);
    const u16x2 m0 = __builtin_elementwise_min(lo, hi), m1 = __builtin_elementwise_max(lo, hi);
    a = c == 0 ? m0 : __builtin_elementwise_min(a, m0);
    b = c == 0 ? m1 : __builtin_elementwise_max(b, m1);
  }
  mn = a.x < a.y ? a.x : a.y;
  mx = b.x < b.y ? b.y : b.x;
}
__device__ inline int first8(const u32x4 &d, uint32_t raw_byte) {
  const uint32_t pat = raw_byte * 0x01010101u;
#pragma unroll
  for (int c = 0; c < 4; c++) {
    const int k = first_zero_lane<8>(d[c] ^ pat);
    if (k >= 0) return 4 * c + k;
  }
  return 16;
}
template <> struct VecOps<uint8_t> {
  static __device__ inline void minmax(const u32x4 &d, uint32_t &mn, uint32_t &mx) {
    byte_vec_minmax<0u>(d, mn, mx);
  }
  static __device__ inline int first(const u32x4 &d, uint32_t t) { return first8(d, t & 0xffu); }
  static __device__ inline int first_in(const u32x4 &d, uint32_t t, int a, int b) {
    return first_equal_in<8>(d, (t & 0xffu) * 0x01010101u, ~0u, a, b);
  }
};
template <> struct VecOps<int8_t> {
  static __device__ inline void minmax(const u32x4 &d, int32_t &mn, int32_t &mx) {
    uint32_t a, b;
    byte_vec_minmax<0x80808080u>(d, a, b);
    mn = (int32_t)a - 128;
    mx = (int32_t)b - 128;
  }
  static __device__ inline int first(const u32x4 &d, int32_t t) { return first8(d, (uint32_t)t & 0xffu); }
  static __device__ inline int first_in(const u32x4 &d, int32_t t, int a, int b) {
    return first_equal_in<8>(d, ((uint32_t)t & 0xffu) * 0x01010101u, ~0u, a, b);
  }
};

// Masked versions (segment ends): positions outside [rlo, rhi) are ignored.
// Only a vector that a segment end cuts takes this path, at most two per
// tile.  The bounds are made relative to the vector, so that each test
// compares an immediate j (tests of absolute positions q0 + j depend only on
// the lane, and the compiler would compute them all before the tile loop and
// keep them in registers).
template <typename T>
__device__ inline void vec_minmax_masked(const u32x4 &d, uint32_t q0, uint32_t rlo, uint32_t rhi,
                                         typename Elem<T>::C &mn, typename Elem<T>::C &mx) {
  using E = Elem<T>;
  constexpr int VEC = 16 / (int)sizeof(T);
  const int a = (int)rlo - (int)q0, b = (int)rhi - (int)q0;
  mn = E::highest();
  mx = E::lowest();
#pragma unroll
  for (int j = 0; j < VEC; j++) {
    const bool ok = j >= a && j < b;
    const typename E::C v = extract<T>(d, j);
    mn = vmin(mn, ok ? v : E::highest());
    mx = vmax(mx, ok ? v : E::lowest());
  }
}
// Bytes use the branch-free lane test (VecOps<T>::first_in); with sixteen
// elements a test per element costs more instructions and registers.
template <typename T>
__device__ inline int vec_first_masked(const u32x4 &d, typename Elem<T>::C target, uint32_t q0, uint32_t rlo,
                                       uint32_t rhi) {
  constexpr int VEC = 16 / (int)sizeof(T);
  const int a = (int)rlo - (int)q0, b = (int)rhi - (int)q0;
  if constexpr (VEC == 16) {
    return VecOps<T>::first_in(d, target, a, b);
  } else {
    int r = VEC;
#pragma unroll
    for (int j = VEC - 1; j >= 0; j--)
      if (j >= a && j < b && extract<T>(d, j) == target) r = j;
    return r;
  }
}

// Running result of one bin segment (wave-uniform).
template <typename C> struct SegState {
  C vmn, vmx;
  int64_t imn, imx;
  bool has;
};

// Load tile vt (vectors vt + u*64 + lane); vectors outside [vlo, vhi) are not
// read (zero).
template <int U>
__device__ inline void load_tile(const u32x4 *__restrict__ base, int64_t vt, int64_t vlo, int64_t vhi, int lane,
                                 u32x4 (&d)[U]) {
  if (vt >= vlo && vt + (int64_t)kWave * U <= vhi) {
#pragma unroll
    for (int u = 0; u < U; u++) d[u] = __builtin_nontemporal_load(base + vt + u * kWave + lane);
  } else {
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t v = vt + u * kWave + lane;
      d[u] = (v >= vlo && v < vhi) ? __builtin_nontemporal_load(base + v) : u32x4{0u, 0u, 0u, 0u};
    }
  }
}

// Tile position of the first element equal to `target` (which some valid
// element holds): the first vector index u whose per-vector extreme equals
// the target on some lane, the lowest such lane, then the first j in that
// lane's vector.  All branches are wave-uniform.
template <typename T, int U>
__device__ inline uint32_t locate(const u32x4 (&d)[U], const typename Elem<T>::C (&ve)[U], typename Elem<T>::C target,
                                  bool full, uint32_t rlo, uint32_t rhi, int lane) {
  constexpr int VEC = 16 / (int)sizeof(T);
  uint32_t pos = 0;
  bool found = false;
#pragma unroll
  for (int u = 0; u < U; u++) {
    if (!found) {
      const uint32_t q0 = (uint32_t)((u * kWave + lane) * VEC);
      const bool hv = full || (q0 + VEC > rlo && q0 < rhi);
      const uint64_t m = ballot(hv && ve[u] == target);
      if (m) {
        const int l = __builtin_ctzll(m);
        const int jl = full ? VecOps<T>::first(d[u], target) : vec_first_masked<T>(d[u], target, q0, rlo, rhi);
        const int j = __builtin_amdgcn_readlane(jl, l);
        pos = (uint32_t)((u * kWave + l) * VEC + j);
        found = true;
      }
    }
  }
  return pos;
}

// Fold one tile into the running result of segment [lo, hi).  Values are
// reduced per vector and per lane, DPP gives the wavefront's extremes, and a
// tile is searched for the position of its extreme only when that extreme
// strictly beats the running one: equal values in later tiles never replace
// an earlier index.
template <typename T, int U>
__device__ inline void fold_tile(const u32x4 (&d)[U], int64_t vt, int64_t shift, int64_t lo, int64_t hi, int lane,
                                 SegState<typename Elem<T>::C> &st) {
  using E = Elem<T>;
  using C = typename E::C;
  constexpr int VEC = 16 / (int)sizeof(T);
  constexpr int64_t TE = (int64_t)kWave * U * VEC;  // elements per tile
  const int64_t g0 = vt * VEC - shift;               // index of tile position 0
  const bool full = g0 >= lo && g0 + TE <= hi;
  const uint32_t rlo = (uint32_t)(lo > g0 ? lo - g0 : 0);
  const uint32_t rhi = (uint32_t)(hi < g0 + TE ? hi - g0 : TE);
  C vm[U], vx[U];
  if (full) {
#pragma unroll
    for (int u = 0; u < U; u++) VecOps<T>::minmax(d[u], vm[u], vx[u]);
  } else {
    // A segment end cuts at most two vectors of the tile: every other vector
    // is wholly inside (reduced as in a full tile) or wholly outside
    // (neutral); only a cut vector is reduced element by element.
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint32_t q0 = (uint32_t)((u * kWave + lane) * VEC);
      VecOps<T>::minmax(d[u], vm[u], vx[u]);
      const bool out = q0 + VEC <= rlo || q0 >= rhi;
      vm[u] = out ? E::highest() : vm[u];
      vx[u] = out ? E::lowest() : vx[u];
      if (!out && (q0 < rlo || q0 + VEC > rhi)) vec_minmax_masked<T>(d[u], q0, rlo, rhi, vm[u], vx[u]);
    }
  }
  C tmn = vm[0], tmx = vx[0];
#pragma unroll
  for (int u = 1; u < U; u++) {
    tmn = vmin(tmn, vm[u]);
    tmx = vmax(tmx, vx[u]);
  }
  const C wmn = wave_min(tmn), wmx = wave_max(tmx);
  if (!st.has || wmn < st.vmn) {
    st.imn = g0 + locate<T, U>(d, vm, wmn, full, rlo, rhi, lane);
    st.vmn = wmn;
  }
  if (!st.has || st.vmx < wmx) {
    st.imx = g0 + locate<T, U>(d, vx, wmx, full, rlo, rhi, lane);
    st.vmx = wmx;
  }
  st.has = true;
}

// Whole-wavefront argmin/argmax of y[lo, hi) (lo < hi, wave-uniform), tile by
// tile with NB tiles in flight.  The first `npre` tiles may already be in buf
// (the chunk prefetch).
template <typename T, int U, int NB>
__device__ void wave_segment(const u32x4 *__restrict__ base, int64_t shift, int64_t lo, int64_t hi, int lane,
                             u32x4 (&buf)[NB][U], int npre, SegState<typename Elem<T>::C> &st) {
  constexpr int VEC = 16 / (int)sizeof(T);
  constexpr int64_t TV = (int64_t)kWave * U;  // vectors per tile
  const int64_t v_lo = (lo + shift) / VEC;
  const int64_t v_hi = (hi + shift + VEC - 1) / VEC;
  const int64_t ntiles = (v_hi - v_lo + TV - 1) / TV;
  st.has = false;
#pragma unroll
  for (int k = 0; k < NB; k++)
    if (k >= npre && k < ntiles) load_tile<U>(base, v_lo + k * TV, v_lo, v_hi, lane, buf[k]);
  for (int64_t t = 0; t < ntiles; t += NB) {
#pragma unroll
    for (int k = 0; k < NB; k++) {
      if (t + k < ntiles) {
        const int64_t vt = v_lo + (t + k) * TV;
        fold_tile<T, U>(buf[k], vt, shift, lo, hi, lane, st);
        if (t + k + NB < ntiles) load_tile<U>(base, vt + NB * TV, v_lo, v_hi, lane, buf[k]);
      }
    }
  }
}

// Reduce chunk c of the series described by p: every bin segment inside the
// chunk goes to binres (bins that start and end in the chunk) or to the
// chunk's partial slots (bins that straddle a chunk boundary).
template <typename T, int U, int NB>
__device__ void scan_chunk(const ScanParams &p, int64_t c, int lane) {
  using E = Elem<T>;
  using C = typename E::C;
  constexpr int VEC = 16 / (int)sizeof(T);
  constexpr int64_t TV = (int64_t)kWave * U;
  const T *__restrict__ y = (const T *)p.y;
  const u32x4 *__restrict__ base = (const u32x4 *)(y - p.shift);
  int64_t c0 = c * p.chunk - p.shift;
  if (c0 < 0) c0 = 0;
  int64_t c1 = (c + 1) * p.chunk - p.shift;
  if (c1 > p.n) c1 = p.n;
  if (p.edges) {  // caller bins may not cover the whole series
    const int64_t e0 = p.edges[0], en = p.edges[p.nb];
    if (c0 < e0) c0 = e0;
    if (c1 > en) c1 = en;
  }
  if (c0 >= c1) return;

  // Prefetch the chunk's first tiles: they do not depend on the bins, so
  // their latency overlaps the bin search below.  A big segment starting at
  // the chunk start (the usual case) consumes them.
  const int64_t vc0 = (c0 + p.shift) / VEC, vc1 = (c1 + p.shift + VEC - 1) / VEC;
  u32x4 buf[NB][U];
#pragma unroll
  for (int k = 0; k < NB; k++) load_tile<U>(base, vc0 + k * TV, vc0, vc1, lane, buf[k]);
  int npre = NB;

  const CeilMulDiv cm = closed_bins(p.n, p.nb);
  int64_t b = uniform(first_bin(p.edges, cm, p.n, p.nb, c0, lane));
  for (;;) {
    const int64_t bb = b + lane;
    const bool inb = bb < p.nb;
    const int64_t s = edge_at(p.edges, cm, p.n, p.nb, bb);
    const int64_t e = edge_at(p.edges, cm, p.n, p.nb, bb + 1);
    const int64_t lo = s > c0 ? s : c0;
    const int64_t hi = e < c1 ? e : c1;
    const bool valid = inb && lo < hi;
    const bool before = s < c0, after = e > c1;
    const bool small = valid && (hi - lo) < p.small;
    if (small) {
      C vmn = E::load(y + lo), vmx = vmn;
      int64_t imn = lo, imx = lo;
      for (int64_t i = lo + 1; i < hi; i++) {
        C v = E::load(y + i);
        if (v < vmn) { vmn = v; imn = i; }
        if (vmx < v) { vmx = v; imx = i; }
      }
      write_result<T>(p, c, bb, before, after, vmn, imn, vmx, imx);
    }
    uint64_t big = ballot(valid && !small);
    while (big) {
      const int k = __builtin_ctzll(big);
      big &= big - 1;
      const int64_t slo = readlane(lo, k), shi = readlane(hi, k);
      SegState<C> st;
      wave_segment<T, U, NB>(base, p.shift, slo, shi, lane, buf, slo == c0 ? npre : 0, st);
      npre = 0;
      const bool sb = readlane(s, k) < c0, sa = readlane(e, k) > c1;
      if (lane == 0) write_result<T>(p, c, b + k, sb, sa, st.vmn, st.imn, st.vmx, st.imx);
    }
    const int64_t e63 = readlane(e, 63);
    if (e63 >= c1 || b + kWave >= p.nb) break;
    b += kWave;
  }
}

// ---- chunks streamed tile by tile (bins of a few kilobytes) -----------------

// Largest chunk of the streamed variant (its tile grid starts at the chunk).
constexpr int64_t kStreamChunkBytes = 65536;

// The same reduction as scan_chunk, for chunks that hold several bins: the
// chunk's tiles are walked once, in order, on the chunk's own grid, with the
// next tile in flight while the current one is folded; each bin segment folds
// the tiles it overlaps (masked at its ends), and a segment that starts in
// the previous segment's last tile folds that tile again from registers.  So
// a bin boundary costs a fold, not a fresh round trip to memory.
template <typename T, int U>
__device__ void scan_chunk_stream(const ScanParams &p, int64_t c, int lane) {
  using E = Elem<T>;
  using C = typename E::C;
  constexpr int VEC = 16 / (int)sizeof(T);
  constexpr int64_t TV = (int64_t)kWave * U;
  const T *__restrict__ y = (const T *)p.y;
  const u32x4 *__restrict__ base = (const u32x4 *)(y - p.shift);
  int64_t c0 = c * p.chunk - p.shift;
  if (c0 < 0) c0 = 0;
  int64_t c1 = (c + 1) * p.chunk - p.shift;
  if (c1 > p.n) c1 = p.n;
  if (p.edges) {
    const int64_t e0 = p.edges[0], en = p.edges[p.nb];
    if (c0 < e0) c0 = e0;
    if (c1 > en) c1 = en;
  }
  if (c0 >= c1) return;
  const int64_t vc0 = (c0 + p.shift) / VEC, vc1 = (c1 + p.shift + VEC - 1) / VEC;
  const int64_t ntiles = (vc1 - vc0 + TV - 1) / TV;
  // cur holds tile tc (vectors vc0 + tc*TV ...), nxt tile tc + 1 (in flight)
  u32x4 cur[U], nxt[U];
  int64_t tc = 0;
  load_tile<U>(base, vc0, vc0, vc1, lane, cur);
  if (ntiles > 1) load_tile<U>(base, vc0 + TV, vc0, vc1, lane, nxt);
  auto advance = [&]() {
#pragma unroll
    for (int u = 0; u < U; u++) cur[u] = nxt[u];
    tc++;
    if (tc + 1 < ntiles) load_tile<U>(base, vc0 + (tc + 1) * TV, vc0, vc1, lane, nxt);
  };

  const CeilMulDiv cm = closed_bins(p.n, p.nb);
  int64_t b = uniform(first_bin(p.edges, cm, p.n, p.nb, c0, lane));
  for (;;) {
    const int64_t bb = b + lane;
    const bool inb = bb < p.nb;
    const int64_t s = edge_at(p.edges, cm, p.n, p.nb, bb);
    const int64_t e = edge_at(p.edges, cm, p.n, p.nb, bb + 1);
    const int64_t lo = s > c0 ? s : c0;
    const int64_t hi = e < c1 ? e : c1;
    const bool valid = inb && lo < hi;
    const bool before = s < c0, after = e > c1;
    const bool small = valid && (hi - lo) < p.small;
    if (small) {
      C vmn = E::load(y + lo), vmx = vmn;
      int64_t imn = lo, imx = lo;
      for (int64_t i = lo + 1; i < hi; i++) {
        C v = E::load(y + i);
        if (v < vmn) { vmn = v; imn = i; }
        if (vmx < v) { vmx = v; imx = i; }
      }
      write_result<T>(p, c, bb, before, after, vmn, imn, vmx, imx);
    }
    uint64_t big = ballot(valid && !small);
    while (big) {
      const int k = __builtin_ctzll(big);
      big &= big - 1;
      const int64_t slo = readlane(lo, k), shi = readlane(hi, k);
      // segments come in index order, so the tiles only move forward
      const int64_t t_first = ((slo + p.shift) / VEC - vc0) / TV;
      const int64_t t_last = ((shi - 1 + p.shift) / VEC - vc0) / TV;
#pragma nounroll
      while (tc < t_first) advance();
      SegState<C> st;
      st.has = false;
#pragma nounroll
      for (;;) {
        fold_tile<T, U>(cur, vc0 + tc * TV, p.shift, slo, shi, lane, st);
        if (tc >= t_last) break;
        advance();
      }
      const bool sb = readlane(s, k) < c0, sa = readlane(e, k) > c1;
      if (lane == 0) write_result<T>(p, c, b + k, sb, sa, st.vmn, st.imn, st.vmx, st.imx);
    }
    const int64_t e63 = readlane(e, 63);
    if (e63 >= c1 || b + kWave >= p.nb) break;
    b += kWave;
  }
}

// ---- chunks classified from x (large bins) ----------------------------------
//
// Instead of looking its bins up in an edge array, the wavefront reads x at
// the chunk's ends (one round trip, overlapped with the tile prefetch) and
// maps them to bins with the edge values of the edge search: x_i lies in bin
// b iff E_b <= x_i < E_{b+1} (the first bin also takes everything below E_1,
// the last everything from E_{nb-1} on).  A bin boundary inside the chunk
// (rare when bins are much longer than chunks) is found by a 64-wide search
// of x inside the chunk, and runs of empty bins are skipped in one step.
// The scan writes the edge array itself as a by-product: every bin start is
// either a chunk start or a boundary found inside a chunk, so each edge is
// written by exactly one wavefront and no separate edge search runs.

// Edge values E_b = x0 + ceil(b R / nb) of int64 x, R = x_last - x0, with
// R = q nb + r split once so that no evaluation needs a 64-bit division:
// ceil(b R / nb) = b q + ceil(b r / nb), where b r < nb^2 < 2^62 is divided
// by a double-precision multiply with 1/nb (off by at most one) and then
// corrected exactly.  The values equal edge_value<int64_t>, which the edge
// search uses.
struct XEdges {
  int64_t x0, nb;
  uint64_t R;
  CeilMulDiv cm;
  double scale;  // nb / R
  __device__ XEdges(int64_t x0_, int64_t xl, int64_t nb_)
      : x0(x0_), nb(nb_), R((uint64_t)xl - (uint64_t)x0_), cm((uint64_t)xl - (uint64_t)x0_, nb_) {
    scale = uniform((double)nb / (double)R);
    cm.q = uniform(cm.q);
    cm.r = uniform(cm.r);
    cm.inv_nb = uniform(cm.inv_nb);
  }
  __device__ int64_t at(int64_t b) const { return uniform((int64_t)((uint64_t)x0 + cm.at(b))); }
  // Bin of xi (x0 <= xi <= x_last): the largest b < nb with E_b <= xi.  Also
  // gives E_{b+1} (`next`), the first value of a later bin (INT64_MAX with
  // next_inf set for the last bin, which takes everything from E_{nb-1} on).
  __device__ int64_t bin(int64_t xi, int64_t &next, bool &next_inf) const {
    if (R == 0) {
      next_inf = true;
      next = INT64_MAX;
      return nb - 1;
    }
    const double est = (double)((uint64_t)xi - (uint64_t)x0) * scale;
    int64_t b = 0;
    if (est >= 1.0) b = est >= (double)(nb - 1) ? nb - 1 : (int64_t)est;
    int64_t eb = at(b), en = b + 1 < nb ? at(b + 1) : INT64_MAX;
    while (b + 1 < nb && en <= xi) {
      b++;
      eb = en;
      en = b + 1 < nb ? at(b + 1) : INT64_MAX;
    }
    while (b > 0 && eb > xi) {
      b--;
      en = eb;
      eb = at(b);
    }
    b = uniform(b);
    next_inf = b + 1 >= nb;
    next = uniform(en);
    return b;
  }
};

// edges[lo .. hi] = v (wave-cooperative; lo > hi writes nothing).
__device__ inline void xc_fill(int64_t *edges, int64_t lo, int64_t hi, int64_t v, int lane) {
  for (int64_t j = lo + lane; j <= hi; j += kWave) edges[j] = v;
}

// First index i in (start, c1) with x[i] >= v, given x[start] = xs < v <=
// x[c1-1] = xe.  Timestamps are close to evenly spaced, so a linear
// interpolation usually lands within a 64-element window holding the answer
// (one or two cache lines); otherwise the window narrows the range for the
// 64-ary search.
__device__ inline int64_t xc_boundary(const int64_t *__restrict__ x, int64_t start, int64_t c1, int64_t xs,
                                      int64_t xe, int64_t v, int lane) {
  int64_t lo = start + 1, hi = c1;
  const double f = (double)((uint64_t)v - (uint64_t)xs) / (double)((uint64_t)xe - (uint64_t)xs);
  int64_t w0 = start + (int64_t)(f * (double)(c1 - 1 - start)) - 32;
  if (w0 > hi - kWave) w0 = hi - kWave;
  if (w0 < lo) w0 = lo;
  const int64_t q = w0 + lane;
  const uint64_t m = ballot(q < hi && x[q] >= v);
  if (m) {
    const int first = __builtin_ctzll(m);
    if (first > 0 || w0 == lo) return w0 + first;
    hi = w0 + 1;  // x[w0] >= v already
  } else {
    lo = w0 + kWave < hi ? w0 + kWave : hi;
  }
  return wave_lower_bound<int64_t, int64_t>(x, lo, hi, v, lane);
}

template <typename T, int U, int NB>
__device__ void scan_chunk_xc(const ScanParams &p, int64_t c, int lane) {
  using C = typename Elem<T>::C;
  constexpr int VEC = 16 / (int)sizeof(T);
  constexpr int64_t TV = (int64_t)kWave * U;
  const T *__restrict__ y = (const T *)p.y;
  const int64_t *__restrict__ x = (const int64_t *)p.x;
  const u32x4 *__restrict__ base = (const u32x4 *)(y - p.shift);
  int64_t c0 = c * p.chunk - p.shift;
  if (c0 < 0) c0 = 0;
  int64_t c1 = (c + 1) * p.chunk - p.shift;
  if (c1 > p.n) c1 = p.n;
  if (c0 >= c1) return;
  const int64_t vc0 = (c0 + p.shift) / VEC, vc1 = (c1 + p.shift + VEC - 1) / VEC;
  u32x4 buf[NB][U];
#pragma unroll
  for (int k = 0; k < NB; k++) load_tile<U>(base, vc0 + k * TV, vc0, vc1, lane, buf[k]);
  int npre = NB;
  // lanes 0..5 read x[0], x[n-1], x[c0-1], x[c0], x[c1-1], x[c1]
  const int64_t pos = lane == 0 ? 0 : lane == 1 ? p.n - 1 : lane == 2 ? c0 - 1 : lane == 3 ? c0 : lane == 4 ? c1 - 1 : c1;
  const int64_t xv = (lane < 6 && pos >= 0 && pos < p.n) ? x[pos] : 0;
  const int64_t nb = p.nb;
  const XEdges E(readlane(xv, 0), readlane(xv, 1), nb);
  const int64_t xa = readlane(xv, 2), xs = readlane(xv, 3), xe = readlane(xv, 4), xb = readlane(xv, 5);
  int64_t n0, n1;
  bool inf0, inf1;
  const int64_t b0 = E.bin(xs, n0, inf0);
  const int64_t b1 = E.bin(xe, n1, inf1);
  // x[c0-1] <= x[c0]: it shares b0 iff it is >= E_{b0}; x[c1] >= x[c1-1]:
  // it shares b1 iff it is below E_{b1+1}
  int64_t bprev = -1, bnext = nb, dummy;
  bool dinf;
  if (c0 > 0) bprev = (b0 == 0 || xa >= E.at(b0)) ? b0 : E.bin(xa, dummy, dinf);
  if (c1 < p.n) bnext = (inf1 || xb < n1) ? b1 : E.bin(xb, dummy, dinf);
  xc_fill(p.xedges, bprev + 1, b0, c0, lane);  // bins starting at c0 (and empty ones before)
  if (c1 == p.n) xc_fill(p.xedges, b1 + 1, nb, p.n, lane);
  int64_t bin = b0, start = c0, next = n0, xstart = xs;
  for (;;) {
    int64_t end = c1, nbin = 0;
    if (bin != b1) {
      // first index after start with x >= E_{bin+1}; it exists inside the
      // chunk because x[c1-1] lies in a later bin
      end = xc_boundary(x, start, c1, xstart, xe, next, lane);
      xstart = x[end];
      nbin = E.bin(xstart, next, dinf);
      xc_fill(p.xedges, bin + 1, nbin, end, lane);  // nbin starts at end; bins between are empty
    }
    SegState<C> st;
    wave_segment<T, U, NB>(base, p.shift, start, end, lane, buf, npre, st);
    npre = 0;
    const bool before = bin == b0 && bprev == b0, after = bin == b1 && bnext == b1;
    if (lane == 0) write_result<T>(p, c, bin, before, after, st.vmn, st.imn, st.vmx, st.imx);
    if (bin == b1) break;
    bin = nbin;
    start = end;
  }
}

template <typename T, int U, int NB>
__global__ __launch_bounds__(256) void k_scan_xc(ScanParams p) {
  const int64_t c = uniform((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  if (c >= p.nchunks) return;
  scan_chunk_xc<T, U, NB>(p, c, lane_id());
}

// ---- staged chunks (many small bins) ---------------------------------------
//
// The whole chunk is first copied into the wavefront's LDS slice with
// coalesced 16-byte loads (all issued together), then every bin segment of
// the chunk is reduced from LDS: one lane per segment for segments shorter
// than kStageLane elements (64 segments per wavefront at a time), the whole
// wavefront for longer ones.  A chunk holding hundreds of bins thus costs one
// HBM round trip instead of one per bin.  `lds` holds chunk/VEC + 1 vectors.

constexpr int64_t kStageLane = 64;

// Lexicographic (value, offset) minimum and maximum inside aligned groups of
// G lanes (4 or 16): xor 1 and xor 2 inside quads, then the half-row mirror
// (the other quad of 8) and the row mirror (the other 8 of 16).  Equal values
// keep the smaller offset, so the result is the group's first occurrence.
template <int CTRL, typename C>
__device__ inline void lex_step(C &vmn, int32_t &jmn, C &vmx, int32_t &jmx) {
  const C omn = dpp_any<CTRL, 0xf>(vmn), omx = dpp_any<CTRL, 0xf>(vmx);
  const int32_t pmn = (int32_t)dpp32<CTRL, 0xf>((uint32_t)jmn), pmx = (int32_t)dpp32<CTRL, 0xf>((uint32_t)jmx);
  if (omn < vmn || (omn == vmn && pmn < jmn)) { vmn = omn; jmn = pmn; }
  if (vmx < omx || (omx == vmx && pmx < jmx)) { vmx = omx; jmx = pmx; }
}

template <int G, typename C>
__device__ inline void group_lex(C &vmn, int32_t &jmn, C &vmx, int32_t &jmx) {
  lex_step<0xB1>(vmn, jmn, vmx, jmx);    // quad_perm [1,0,3,2]
  lex_step<0x4E>(vmn, jmn, vmx, jmx);    // quad_perm [2,3,0,1]
  if constexpr (G >= 16) {
    lex_step<0x141>(vmn, jmn, vmx, jmx);  // row_half_mirror
    lex_step<0x140>(vmn, jmn, vmx, jmx);  // row_mirror
  }
}

// One round of a staged chunk with G lanes per bin (G = 1, 4 or 16): lane l
// takes bin b + l / G and, inside the chunk, its elements l % G, l % G + G,
// ... in index order; the group then reduces (value, offset) pairs.  Returns
// false after the round that reaches the chunk's end.
template <typename T, int G>
__device__ inline bool staged_round(const ScanParams &p, const CeilMulDiv &cm, int64_t c, int64_t c0, int64_t c1,
                                    const T *lt, int64_t g_base, int64_t &b, int lane) {
  using E = Elem<T>;
  using C = typename E::C;
  const int sub = lane % G;
  const int64_t bb = b + lane / G;
  const bool inb = bb < p.nb;
  const int64_t s = edge_at(p.edges, cm, p.n, p.nb, bb);
  const int64_t e = edge_at(p.edges, cm, p.n, p.nb, bb + 1);
  const int64_t lo = s > c0 ? s : c0;
  const int64_t hi = e < c1 ? e : c1;
  const bool valid = inb && lo < hi;
  C vmn = E::highest(), vmx = E::lowest();
  int32_t jmn = INT32_MAX, jmx = INT32_MAX;
  if (valid) {
    const int32_t o1 = (int32_t)(hi - g_base);
    int32_t j = (int32_t)(lo - g_base) + sub;
    for (; j + 3 * G < o1; j += 4 * G) {  // four LDS reads in flight
      C v[4];
#pragma unroll
      for (int u = 0; u < 4; u++) v[u] = E::load(lt + j + u * G);
#pragma unroll
      for (int u = 0; u < 4; u++) {
        if (jmn == INT32_MAX || v[u] < vmn) { vmn = v[u]; jmn = j + u * G; }
        if (jmx == INT32_MAX || vmx < v[u]) { vmx = v[u]; jmx = j + u * G; }
      }
    }
    for (; j < o1; j += G) {
      const C v = E::load(lt + j);
      if (jmn == INT32_MAX || v < vmn) { vmn = v; jmn = j; }
      if (jmx == INT32_MAX || vmx < v) { vmx = v; jmx = j; }
    }
  }
  if constexpr (G > 1) group_lex<G>(vmn, jmn, vmx, jmx);
  if (valid && sub == 0) write_result<T>(p, c, bb, s < c0, e > c1, vmn, g_base + jmn, vmx, g_base + jmx);
  const int64_t elast = readlane(e, 63);
  b += kWave / G;
  return !(elast >= c1 || b >= p.nb);
}

// The same round over whole 16-byte vectors (types of at most four bytes; bins
// of at least a vector per lane): lane l takes its bin's vectors l % G,
// l % G + G, ... from LDS, reduces each with the packed per-vector fold (the
// vectors a bin end cuts element by element) and keeps the first vector that
// strictly improves its extremes; the group reduces (value, vector) pairs,
// and the group's first lane finds the first element equal to each extreme
// inside the winning vector.  About two instructions per element where the
// element-wise round takes eight or nine.
template <typename T, int G>
__device__ inline bool staged_round_vec(const ScanParams &p, const CeilMulDiv &cm, int64_t c, int64_t c0, int64_t c1,
                                        const u32x4 *lv, int64_t g_base, int64_t &b, int lane) {
  using E = Elem<T>;
  using C = typename E::C;
  constexpr int VEC = 16 / (int)sizeof(T);
  const int sub = lane % G;
  const int64_t bb = b + lane / G;
  const bool inb = bb < p.nb;
  const int64_t s = edge_at(p.edges, cm, p.n, p.nb, bb);
  const int64_t e = edge_at(p.edges, cm, p.n, p.nb, bb + 1);
  const int64_t lo = s > c0 ? s : c0;
  const int64_t hi = e < c1 ? e : c1;
  const bool valid = inb && lo < hi;
  C vmn = E::highest(), vmx = E::lowest();
  int32_t kmn = INT32_MAX, kmx = INT32_MAX;
  const uint32_t r0 = valid ? (uint32_t)(lo - g_base) : 0u, r1 = valid ? (uint32_t)(hi - g_base) : 0u;
  if (valid) {
    const int32_t k1 = (int32_t)((r1 + VEC - 1) / VEC);
    for (int32_t k = (int32_t)(r0 / VEC) + sub; k < k1; k += G) {
      const u32x4 d = lv[k];
      const uint32_t q0 = (uint32_t)k * VEC;
      C a, x;
      if (q0 >= r0 && q0 + VEC <= r1) {
        VecOps<T>::minmax(d, a, x);
      } else {
        vec_minmax_masked<T>(d, q0, r0, r1, a, x);
      }
      if (kmn == INT32_MAX || a < vmn) { vmn = a; kmn = k; }
      if (kmx == INT32_MAX || vmx < x) { vmx = x; kmx = k; }
    }
  }
  group_lex<G>(vmn, kmn, vmx, kmx);
  if (valid && sub == 0) {
    const uint32_t qn = (uint32_t)kmn * VEC, qx = (uint32_t)kmx * VEC;
    const int jn = vec_first_masked<T>(lv[kmn], vmn, qn, r0, r1);
    const int jx = vec_first_masked<T>(lv[kmx], vmx, qx, r0, r1);
    write_result<T>(p, c, bb, s < c0, e > c1, vmn, g_base + qn + jn, vmx, g_base + qx + jx);
  }
  const int64_t elast = readlane(e, 63);
  b += kWave / G;
  return !(elast >= c1 || b >= p.nb);
}

// Lanes per bin for a staged chunk of `len` elements with bins of about
// `avg` elements, from a cost model in instructions: rounds x (strided
// element steps + the group reduction + fixed per-round work).  64 means one
// bin at a time across the whole wavefront.
__device__ inline int staged_group(double len, double avg) {
  const double bins = len / avg + 1.0;
  double best = 0.0;
  int g = 1;
  const int gs[3] = {1, 4, 16};
  for (int k = 0; k < 3; k++) {
    const double G = gs[k];
    const double rounds = ceil(bins * G / 64.0);
    const double cost = rounds * (avg / G * 4.0 + 16.0 * (k == 0 ? 0 : (k == 1 ? 2 : 4)) + 40.0);
    if (k == 0 || cost < best) { best = cost; g = gs[k]; }
  }
  const double wave = bins * (avg / 64.0 * 4.0 + 200.0);
  return wave < best ? 64 : g;
}

template <typename T>
__device__ void scan_chunk_staged(const ScanParams &p, int64_t c, int lane, u32x4 *lds) {
  using E = Elem<T>;
  using C = typename E::C;
  constexpr int VEC = 16 / (int)sizeof(T);
  const T *__restrict__ y = (const T *)p.y;
  const u32x4 *__restrict__ base = (const u32x4 *)(y - p.shift);
  int64_t c0 = c * p.chunk - p.shift;
  if (c0 < 0) c0 = 0;
  int64_t c1 = (c + 1) * p.chunk - p.shift;
  if (c1 > p.n) c1 = p.n;
  if (p.edges) {
    const int64_t e0 = p.edges[0], en = p.edges[p.nb];
    if (c0 < e0) c0 = e0;
    if (c1 > en) c1 = en;
  }
  if (c0 >= c1) return;
  const int64_t vc0 = (c0 + p.shift) / VEC, vc1 = (c1 + p.shift + VEC - 1) / VEC;
  const int64_t nv = vc1 - vc0;
  for (int64_t k0 = 0; k0 < nv; k0 += (int64_t)kWave * 8) {
    u32x4 d[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int64_t v = k0 + u * kWave + lane;
      d[u] = v < nv ? __builtin_nontemporal_load(base + vc0 + v) : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int64_t v = k0 + u * kWave + lane;
      if (v < nv) lds[v] = d[u];
    }
  }
  // The wavefront's own LDS writes complete in order before its later LDS
  // reads; the fences keep the compiler from moving the reads above them.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const T *lt = (const T *)lds;
  const int64_t g_base = vc0 * VEC - p.shift;  // global index of lt[0]

  const CeilMulDiv cm = closed_bins(p.n, p.nb);
  int64_t b = uniform(first_bin(p.edges, cm, p.n, p.nb, c0, lane));
  const int G = staged_group((double)(c1 - c0), (double)p.n / (double)p.nb);
  if (G == 1) {
    while (staged_round<T, 1>(p, cm, c, c0, c1, lt, g_base, b, lane)) {}
    return;
  }
  // whole vectors per lane once bins average at least a vector per lane, for
  // types of at most four bytes (f64 pairs gain nothing: 1-6% slower)
  const bool vec = VEC >= 4 && (double)p.n / (double)p.nb >= (double)(G * VEC);
  if (G == 4) {
    if (vec) {
      while (staged_round_vec<T, 4>(p, cm, c, c0, c1, lds, g_base, b, lane)) {}
    } else {
      while (staged_round<T, 4>(p, cm, c, c0, c1, lt, g_base, b, lane)) {}
    }
    return;
  }
  if (G == 16) {
    if (vec) {
      while (staged_round_vec<T, 16>(p, cm, c, c0, c1, lds, g_base, b, lane)) {}
    } else {
      while (staged_round<T, 16>(p, cm, c, c0, c1, lt, g_base, b, lane)) {}
    }
    return;
  }
  // long bins: one segment at a time across the wavefront (short pieces at
  // the chunk's ends one per lane)
  for (;;) {
    const int64_t bb = b + lane;
    const bool inb = bb < p.nb;
    const int64_t s = edge_at(p.edges, cm, p.n, p.nb, bb);
    const int64_t e = edge_at(p.edges, cm, p.n, p.nb, bb + 1);
    const int64_t lo = s > c0 ? s : c0;
    const int64_t hi = e < c1 ? e : c1;
    const bool valid = inb && lo < hi;
    const bool before = s < c0, after = e > c1;
    const bool small = valid && (hi - lo) < kStageLane;
    if (small) {
      const T *q = lt + (lo - g_base);
      const int32_t len = (int32_t)(hi - lo);
      C vmn = E::load(q), vmx = vmn;
      int32_t jmn = 0, jmx = 0;
      for (int32_t j = 1; j < len; j++) {
        const C v = E::load(q + j);
        if (v < vmn) { vmn = v; jmn = j; }
        if (vmx < v) { vmx = v; jmx = j; }
      }
      write_result<T>(p, c, bb, before, after, vmn, lo + jmn, vmx, lo + jmx);
    }
    uint64_t big = ballot(valid && !small);
    while (big) {
      const int k = __builtin_ctzll(big);
      big &= big - 1;
      const int64_t slo = readlane(lo, k), shi = readlane(hi, k);
      if constexpr (VEC >= 4) {
        // whole vectors across the wavefront: the per-vector fold, then the
        // first vector holding each extreme and the first element in it
        const uint32_t r0 = (uint32_t)(slo - g_base), r1 = (uint32_t)(shi - g_base);
        const int32_t k1 = (int32_t)((r1 + VEC - 1) / VEC);
        C vmn = E::highest(), vmx = E::lowest();
        int32_t kmn = INT32_MAX, kmx = INT32_MAX;
        for (int32_t kv = (int32_t)(r0 / VEC) + lane; kv < k1; kv += kWave) {
          const u32x4 d = lds[kv];
          const uint32_t q0 = (uint32_t)kv * VEC;
          C a, x;
          if (q0 >= r0 && q0 + VEC <= r1) {
            VecOps<T>::minmax(d, a, x);
          } else {
            vec_minmax_masked<T>(d, q0, r0, r1, a, x);
          }
          if (kmn == INT32_MAX || a < vmn) { vmn = a; kmn = kv; }
          if (kmx == INT32_MAX || vmx < x) { vmx = x; kmx = kv; }
        }
        const C wmn = wave_min(vmn), wmx = wave_max(vmx);
        const int32_t vn = (int32_t)uniform(wave_min((int64_t)(kmn != INT32_MAX && vmn == wmn ? kmn : INT32_MAX)));
        const int32_t vx = (int32_t)uniform(wave_min((int64_t)(kmx != INT32_MAX && vmx == wmx ? kmx : INT32_MAX)));
        const int jn = vec_first_masked<T>(lds[vn], wmn, (uint32_t)vn * VEC, r0, r1);
        const int jx = vec_first_masked<T>(lds[vx], wmx, (uint32_t)vx * VEC, r0, r1);
        const bool sb = readlane(s, k) < c0, sa = readlane(e, k) > c1;
        if (lane == 0)
          write_result<T>(p, c, b + k, sb, sa, wmn, g_base + (int64_t)vn * VEC + jn, wmx,
                          g_base + (int64_t)vx * VEC + jx);
        continue;
      }
      // per lane: elements slo + lane + 64 i in index order, strict compares,
      // four LDS reads in flight per step
      C vmn = E::highest(), vmx = E::lowest();
      int32_t jmn = INT32_MAX, jmx = INT32_MAX;  // offsets from slo
      const T *q = lt + (slo - g_base);
      const int32_t len = (int32_t)(shi - slo);
      for (int32_t j0 = lane; j0 < len; j0 += 4 * kWave) {
        C v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int32_t j = j0 + u * kWave;
          v[u] = E::load(q + (j < len ? j : 0));
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int32_t j = j0 + u * kWave;
          if (j < len) {
            if (jmn == INT32_MAX || v[u] < vmn) { vmn = v[u]; jmn = j; }
            if (jmx == INT32_MAX || vmx < v[u]) { vmx = v[u]; jmx = j; }
          }
        }
      }
      const int64_t imn = jmn == INT32_MAX ? INT64_MAX : slo + jmn;
      const int64_t imx = jmx == INT32_MAX ? INT64_MAX : slo + jmx;
      const C wmn = wave_min(vmn), wmx = wave_max(vmx);
      const int64_t rmn = wave_min(imn != INT64_MAX && vmn == wmn ? imn : INT64_MAX);
      const int64_t rmx = wave_min(imx != INT64_MAX && vmx == wmx ? imx : INT64_MAX);
      const bool sb = readlane(s, k) < c0, sa = readlane(e, k) > c1;
      if (lane == 0) write_result<T>(p, c, b + k, sb, sa, wmn, rmn, wmx, rmx);
    }
    const int64_t e63 = readlane(e, 63);
    if (e63 >= c1 || b + kWave >= p.nb) break;
    b += kWave;
  }
}

// LDS vectors one wavefront needs for a staged chunk of `chunk` elements.
__host__ __device__ inline int64_t staged_lds_vectors(int64_t chunk_elems, int vec) { return chunk_elems / vec + 1; }

template <typename T>
__global__ __launch_bounds__(256) void k_scan_staged(ScanParams p) {
  extern __shared__ u32x4 stage_lds[];
  const int64_t c = uniform((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  if (c >= p.nchunks) return;
  constexpr int VEC = 16 / (int)sizeof(T);
  const int64_t per = staged_lds_vectors(p.chunk, VEC);
  scan_chunk_staged<T>(p, c, lane_id(), stage_lds + (threadIdx.x >> 6) * per);
}

template <typename T, int U, int NB>
__global__ __launch_bounds__(256) void k_scan(ScanParams p) {
  const int64_t c = uniform((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  if (c >= p.nchunks) return;
  scan_chunk<T, U, NB>(p, c, lane_id());
}

template <typename T, int U>
__global__ __launch_bounds__(256) void k_scan_stream(ScanParams p) {
  const int64_t c = uniform((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  if (c >= p.nchunks) return;
  scan_chunk_stream<T, U>(p, c, lane_id());
}


// ------------------------------------------------------------------ merge

// Per bin: the final (argmin, argmax), merged lexicographically from the
// partials of every chunk the bin touches when it straddles chunks.
__device__ void merged_bin(const MergeParams &p, int64_t s, int64_t e, int64_t bin, int lane, int64_t &imn,
                           int64_t &imx) {
  const int64_t cs = (s + p.shift) / p.chunk, ce = (e - 1 + p.shift) / p.chunk;
  if (cs == ce) {
    imn = p.binres[2 * bin];
    imx = p.binres[2 * bin + 1];
    return;
  }
  uint64_t kmn = ~0ull, kmx = 0;
  int64_t jmn = INT64_MAX, jmx = INT64_MAX;
  for (int64_t c = cs + lane; c <= ce; c += kWave) {
    const Partial q = (c == cs) ? p.partR[c] : p.partL[c];
    lex_min(kmn, jmn, q.kmin, q.imin);
    lex_max(kmx, jmx, q.kmax, q.imax);
  }
  const uint64_t wkmn = wave_min(kmn), wkmx = wave_max(kmx);
  imn = wave_min(kmn == wkmn ? jmn : INT64_MAX);
  imx = wave_min(kmx == wkmx ? jmx : INT64_MAX);
}

// The same merge by one lane alone, the bin's partials in chunk order (the
// lexicographic minimum does not depend on the order): for bins that span a
// few chunks, where a wavefront per bin would leave most lanes idle.
__device__ inline void merged_bin_lane(const MergeParams &p, int64_t s, int64_t e, int64_t bin, int64_t &imn,
                                       int64_t &imx) {
  const int64_t cs = (s + p.shift) / p.chunk, ce = (e - 1 + p.shift) / p.chunk;
  if (cs == ce) {
    imn = p.binres[2 * bin];
    imx = p.binres[2 * bin + 1];
    return;
  }
  uint64_t kmn = ~0ull, kmx = 0;
  int64_t jmn = INT64_MAX, jmx = INT64_MAX;
  for (int64_t c = cs; c <= ce; c++) {
    const Partial q = (c == cs) ? p.partR[c] : p.partL[c];
    lex_min(kmn, jmn, q.kmin, q.imin);
    lex_max(kmx, jmx, q.kmax, q.imax);
  }
  imn = jmn;
  imx = jmx;
}

// Bin b clipped to [0, n) (caller edges are not trusted to stay in range).
__device__ inline void bin_range(const MergeParams &p, int64_t bin, int64_t &s, int64_t &e) {
  const CeilMulDiv cm = closed_bins(p.n, p.nb);
  s = edge_at(p.edges, cm, p.n, p.nb, bin);
  e = edge_at(p.edges, cm, p.n, p.nb, bin + 1);
  s = s < 0 ? 0 : (s > p.n ? p.n : s);
  e = e < s ? s : (e > p.n ? p.n : e);
}


// Sorted distinct selection of bin [s, e): MinMax keeps {argmin, argmax},
// M4 adds the first and last index.  Writes up to 4 indices, returns the count.
__device__ inline int bin_selection(int64_t s, int64_t e, int64_t imn, int64_t imx, int m4, int64_t *dst) {
  // the four candidates (MinMax: the argmin and argmax twice), sorted by a
  // five-comparator network in registers, then written without repeats
  int64_t v0 = m4 ? s : imn, v1 = imn, v2 = imx, v3 = m4 ? e - 1 : imx;
  const auto cswap = [](int64_t &a, int64_t &b) {
    const int64_t lo = a < b ? a : b, hi = a < b ? b : a;
    a = lo;
    b = hi;
  };
  cswap(v0, v1);
  cswap(v2, v3);
  cswap(v0, v2);
  cswap(v1, v3);
  cswap(v1, v2);
  int m = 0;
  dst[m++] = v0;
  if (v1 != v0) dst[m++] = v1;
  if (v2 != v1) dst[m++] = v2;
  if (v3 != v2) dst[m++] = v3;
  return m;
}

// Exclusive scan of one int64 per thread over a 1024-thread block.
__device__ int64_t block_exclusive_scan(int64_t v, int64_t *lds, int64_t &total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int64_t incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t o = __shfl_up(incl, d, 64);
    if (lane >= d) incl += o;
  }
  if (lane == 63) lds[w] = incl;
  __syncthreads();
  if (w == 0) {
    int64_t ws = lane < (int)(blockDim.x >> 6) ? lds[lane] : 0;
    int64_t wi = ws;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      int64_t o = __shfl_up(wi, d, 64);
      if (lane >= d) wi += o;
    }
    if (lane < (int)(blockDim.x >> 6)) lds[32 + lane] = wi - ws;
    if (lane == 63) lds[64] = wi;
  }
  __syncthreads();
  total = lds[64];
  int64_t r = lds[32 + w] + incl - v;
  __syncthreads();
  return r;
}

}  // namespace tsds

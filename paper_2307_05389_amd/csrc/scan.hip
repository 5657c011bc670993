// scan.hip -- the argmin/argmax hot path of MinMax, M4 and the MinMax
// preselection of MinMaxLTTB on gfx950.
//
// The paper's kernel (Sec. 2.1, Listing 1) keeps per-SIMD-lane running
// minima/maxima with strict compares and resolves the lanes at the end; its
// bins come from a search-sorted over x and run in parallel (Sec. 2.2).  Here:
//
//   k_edges_x   one wavefront per bin edge: 64-ary search of the edge value
//               in x (a few dependent rounds instead of log2(n)).
//   k_scan<T>   one wavefront per fixed-size chunk of y, independent of the
//               bins, so the load is balanced whatever the bin sizes.  Each
//               bin segment inside the chunk is reduced either by the whole
//               wavefront (16-byte coalesced loads, tile-wise value reduction
//               through DPP, index recovered only when a tile beats the
//               running extreme) or, for short segments, by one lane per bin
//               (64 bins per wavefront).  Bins that end in the chunk where
//               they start are final; the segments of straddling bins are
//               written as (key, index) partials.
//   k_merge     one wavefront per bin: lexicographic merge of the partials of
//               a straddling bin, then the bin's sorted distinct selection.
//   k_compact   one workgroup: exclusive scan of the per-bin counts and the
//               compaction into strictly increasing indices.
#include <limits>
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace tsds {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ edges

template <typename X> struct XKey;
template <> struct XKey<int32_t> { using K = int64_t; };
template <> struct XKey<int64_t> { using K = int64_t; };
template <> struct XKey<uint32_t> { using K = uint64_t; };
template <> struct XKey<uint64_t> { using K = uint64_t; };

// Integer edge value E_b = x0 + ceil(b * R / nb) with R = x_last - x0 >= 0,
// exact although b*R may need 128 bits: with R = q*nb + r,
// b*R/nb = b*q + b*r/nb, and b*r < nb^2 < 2^64 (the host keeps nb < 2^32).
__device__ inline uint64_t ceil_mul_div(uint64_t b, uint64_t R, uint64_t nb) {
  uint64_t q = R / nb, r = R % nb;
  uint64_t br = b * r;
  uint64_t t = br / nb;
  return b * q + t + (t * nb == br ? 0 : 1);
}

// Wavefront-cooperative lower bound: the first index i in [0, n) with
// x[i] >= v (n if none).  Each round probes 64 evenly spaced positions.
template <typename X, typename K>
__device__ int64_t wave_lower_bound(const X *x, int64_t n, K v, int lane) {
  int64_t lo = 0, hi = n;  // answer in [lo, hi]; x[lo-1] < v, x[hi] >= v
  while (hi > lo) {
    int64_t span = hi - lo;
    int64_t step = (span + 63) / 64;
    int64_t q = lo + (int64_t)lane * step;
    bool less = q < hi && (K)x[q] < v;
    int cnt = __builtin_popcountll(ballot(less));  // lanes 0..cnt-1 are below v
    if (cnt == 0) {
      hi = lo;
    } else {
      int64_t nlo = lo + (int64_t)(cnt - 1) * step + 1;
      int64_t nhi = lo + (int64_t)cnt * step;
      lo = nlo;
      hi = nhi < hi ? nhi : hi;
    }
  }
  return lo;
}

template <typename X>
__global__ __launch_bounds__(256) void k_edges_int(const X *x, int64_t n, int64_t nb, int64_t *edges) {
  using K = typename XKey<X>::K;
  const int lane = lane_id();
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b > nb) return;
  if (b == nb) {
    if (lane == 0) edges[nb] = n;
    return;
  }
  if (b == 0) {
    if (lane == 0) edges[0] = 0;
    return;
  }
  K x0 = (K)x[0], xl = (K)x[n - 1];
  uint64_t R = (uint64_t)xl - (uint64_t)x0;  // exact modulo 2^64, x sorted
  K E = (K)((uint64_t)x0 + ceil_mul_div((uint64_t)b, R, (uint64_t)nb));
  int64_t s = wave_lower_bound<X, K>(x, n, E, lane);
  if (lane == 0) edges[b] = s;
}

template <typename X>
__global__ __launch_bounds__(256) void k_edges_float(const X *x, int64_t n, int64_t nb, int64_t *edges) {
  const int lane = lane_id();
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b > nb) return;
  if (b == nb) {
    if (lane == 0) edges[nb] = n;
    return;
  }
  if (b == 0) {
    if (lane == 0) edges[0] = 0;
    return;
  }
  double x0 = (double)x[0], R = (double)x[n - 1] - x0;
  // E_b = x0 + (b * R) / nb, each operation rounded to nearest (the unit is
  // built with -ffp-contract=off, so no FMA joins the product and the sum).
  double E = x0 + ((double)b * R) / (double)nb;
  // lower bound on the widened values
  int64_t lo = 0, hi = n;
  while (hi > lo) {
    int64_t step = (hi - lo + 63) / 64;
    int64_t q = lo + (int64_t)lane * step;
    bool less = q < hi && (double)x[q] < E;
    int cnt = __builtin_popcountll(ballot(less));
    if (cnt == 0) {
      hi = lo;
    } else {
      int64_t nlo = lo + (int64_t)(cnt - 1) * step + 1;
      int64_t nhi = lo + (int64_t)cnt * step;
      lo = nlo;
      hi = nhi < hi ? nhi : hi;
    }
  }
  if (lane == 0) edges[b] = lo;
}

__global__ void k_edges_nox(int64_t n, int64_t nb, int64_t *edges) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nb) return;
  if (b == nb || n == 0) { edges[b] = b == nb ? n : 0; return; }
  uint64_t num = (uint64_t)b * (uint64_t)(n - 1);
  edges[b] = (int64_t)((num + (uint64_t)nb - 1) / (uint64_t)nb);
}

hipError_t launch_edges_nox(int64_t n, int64_t nb, int64_t *edges, hipStream_t st) {
  int64_t threads = nb + 1;
  k_edges_nox<<<dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st>>>(n, nb, edges);
  return hipGetLastError();
}

hipError_t launch_edges_x(const void *x, int xdt, int64_t n, int64_t nb, int64_t *edges, hipStream_t st) {
  dim3 grid((unsigned)((nb + 1 + 3) / 4)), block(256);
  switch (xdt) {
    case TS_I32: k_edges_int<int32_t><<<grid, block, 0, st>>>((const int32_t *)x, n, nb, edges); break;
    case TS_I64: k_edges_int<int64_t><<<grid, block, 0, st>>>((const int64_t *)x, n, nb, edges); break;
    case TS_U32: k_edges_int<uint32_t><<<grid, block, 0, st>>>((const uint32_t *)x, n, nb, edges); break;
    case TS_U64: k_edges_int<uint64_t><<<grid, block, 0, st>>>((const uint64_t *)x, n, nb, edges); break;
    case TS_F32: k_edges_float<float><<<grid, block, 0, st>>>((const float *)x, n, nb, edges); break;
    case TS_F64: k_edges_float<double><<<grid, block, 0, st>>>((const double *)x, n, nb, edges); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ scan

// Start of bin b (b <= nb); b >= nb gives the end of the last bin.
__device__ inline int64_t edge_at(const int64_t *edges, int64_t n, int64_t nb, int64_t b) {
  if (b >= nb) return edges ? edges[nb] : n;
  if (edges) return edges[b];
  uint64_t num = (uint64_t)b * (uint64_t)(n - 1);
  return (int64_t)((num + (uint64_t)nb - 1) / (uint64_t)nb);
}

// First bin whose range can intersect [c0, ...): the last b with start <= c0.
__device__ int64_t first_bin(const int64_t *edges, int64_t n, int64_t nb, int64_t c0, int lane) {
  if (!edges) {
    if (n <= 1) return 0;
    uint64_t q = (uint64_t)c0 * (uint64_t)nb / (uint64_t)(n - 1);
    return q < (uint64_t)nb ? (int64_t)q : nb - 1;
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

// Whole-wavefront argmin/argmax of y[lo, hi) (lo < hi, wave-uniform).
// Vector v of the 16-byte aligned base holds elements v*VEC - shift + j.
// A tile is U vectors per lane, lane-interleaved (fully coalesced).  Per
// tile the lanes reduce values only; the wavefront min/max comes from DPP;
// only a tile whose extreme strictly beats the running one is searched for
// the first position of that value (so ties keep the earlier tile).
template <typename T, int U>
__device__ void wave_segment(const u32x4 *__restrict__ base, int64_t shift, int64_t lo, int64_t hi, int lane,
                             typename Elem<T>::C &rmn, int64_t &rimn, typename Elem<T>::C &rmx,
                             int64_t &rimx) {
  using E = Elem<T>;
  using C = typename E::C;
  constexpr int VEC = 16 / (int)sizeof(T);
  constexpr int64_t TV = (int64_t)kWave * U;  // vectors per tile
  const int64_t v_lo = (lo + shift) / VEC;
  const int64_t v_hi = (hi + shift + VEC - 1) / VEC;
  bool has = false;

  u32x4 buf[2][U];
  auto interior = [&](int64_t vt) {
    return vt * VEC - shift >= lo && (vt + TV) * VEC - shift <= hi;
  };
  auto load = [&](int64_t vt, u32x4 (&d)[U]) {
    if (interior(vt)) {
#pragma unroll
      for (int u = 0; u < U; u++) d[u] = __builtin_nontemporal_load(base + vt + u * kWave + lane);
    } else {
#pragma unroll
      for (int u = 0; u < U; u++) {
        int64_t v = vt + u * kWave + lane;
        d[u] = (v >= v_lo && v < v_hi) ? __builtin_nontemporal_load(base + v) : u32x4{0u, 0u, 0u, 0u};
      }
    }
  };
  auto process = [&](int64_t vt, const u32x4 (&d)[U]) {
    const bool full = interior(vt);
    C tmn = E::highest(), tmx = E::lowest();
    if (full) {
#pragma unroll
      for (int u = 0; u < U; u++)
#pragma unroll
        for (int j = 0; j < VEC; j++) {
          C xv = extract<T>(d[u], j);
          tmn = vmin(tmn, xv);
          tmx = vmax(tmx, xv);
        }
    } else {
#pragma unroll
      for (int u = 0; u < U; u++)
#pragma unroll
        for (int j = 0; j < VEC; j++) {
          int64_t g = (vt + u * kWave + lane) * VEC + j - shift;
          bool ok = g >= lo && g < hi;
          C xv = extract<T>(d[u], j);
          tmn = vmin(tmn, ok ? xv : E::highest());
          tmx = vmax(tmx, ok ? xv : E::lowest());
        }
    }
    C wmn = wave_min(tmn), wmx = wave_max(tmx);
    const int64_t g0 = vt * VEC - shift;  // global index of tile position 0
    if (!has || wmn < rmn) {
      uint32_t pos = 0xffffffffu;
#pragma unroll
      for (int u = U - 1; u >= 0; u--)
#pragma unroll
        for (int j = VEC - 1; j >= 0; j--) {
          uint32_t q = (uint32_t)((u * kWave + lane) * VEC + j);
          int64_t g = g0 + q;
          bool ok = full || (g >= lo && g < hi);
          if (ok && extract<T>(d[u], j) == wmn) pos = q;
        }
      pos = wave_min(pos);
      rmn = wmn;
      rimn = g0 + pos;
    }
    if (!has || rmx < wmx) {
      uint32_t pos = 0xffffffffu;
#pragma unroll
      for (int u = U - 1; u >= 0; u--)
#pragma unroll
        for (int j = VEC - 1; j >= 0; j--) {
          uint32_t q = (uint32_t)((u * kWave + lane) * VEC + j);
          int64_t g = g0 + q;
          bool ok = full || (g >= lo && g < hi);
          if (ok && extract<T>(d[u], j) == wmx) pos = q;
        }
      pos = wave_min(pos);
      rmx = wmx;
      rimx = g0 + pos;
    }
    has = true;
  };

  const int64_t ntiles = (v_hi - v_lo + TV - 1) / TV;
  load(v_lo, buf[0]);
  int64_t t = 0;
  for (; t + 1 < ntiles; t += 2) {
    const int64_t vt = v_lo + t * TV;
    load(vt + TV, buf[1]);
    process(vt, buf[0]);
    if (t + 2 < ntiles) load(vt + 2 * TV, buf[0]);
    process(vt + TV, buf[1]);
  }
  if (t < ntiles) process(v_lo + t * TV, buf[0]);
}

template <typename T, int U>
__global__ __launch_bounds__(256) void k_scan(ScanParams p) {
  using E = Elem<T>;
  using C = typename E::C;
  constexpr int VEC = 16 / (int)sizeof(T);
  const int lane = lane_id();
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= p.nchunks) return;
  const T *__restrict__ y = (const T *)p.y;
  const u32x4 *__restrict__ base = (const u32x4 *)(y - p.shift);
  int64_t c0 = c * p.chunk - p.shift;
  if (c0 < 0) c0 = 0;
  int64_t c1 = (c + 1) * p.chunk - p.shift;
  if (c1 > p.n) c1 = p.n;
  if (p.edges) {  // caller bins may not cover the whole series
    int64_t e0 = p.edges[0], en = p.edges[p.nb];
    if (c0 < e0) c0 = e0;
    if (c1 > en) c1 = en;
  }
  if (c0 >= c1) return;
  (void)VEC;

  int64_t b = first_bin(p.edges, p.n, p.nb, c0, lane);
  for (;;) {
    const int64_t bb = b + lane;
    const bool inb = bb < p.nb;
    const int64_t s = edge_at(p.edges, p.n, p.nb, bb);
    const int64_t e = edge_at(p.edges, p.n, p.nb, bb + 1);
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
      C vmn, vmx;
      int64_t imn = 0, imx = 0;
      wave_segment<T, U>(base, p.shift, slo, shi, lane, vmn, imn, vmx, imx);
      const bool sb = readlane(s, k) < c0, sa = readlane(e, k) > c1;
      if (lane == 0) write_result<T>(p, c, b + k, sb, sa, vmn, imn, vmx, imx);
    }
    const int64_t e63 = readlane(e, 63);
    if (e63 >= c1 || b + kWave >= p.nb) break;
    b += kWave;
  }
}

template <typename T>
static hipError_t scan_t(const ScanParams &p, hipStream_t st) {
  dim3 grid((unsigned)((p.nchunks + 3) / 4)), block(256);
  k_scan<T, 4><<<grid, block, 0, st>>>(p);
  return hipGetLastError();
}

hipError_t launch_scan(int ydt, const ScanParams &p, hipStream_t st) {
  switch (ydt) {
    case TS_I8: return scan_t<int8_t>(p, st);
    case TS_I16: return scan_t<int16_t>(p, st);
    case TS_I32: return scan_t<int32_t>(p, st);
    case TS_I64: return scan_t<int64_t>(p, st);
    case TS_U8: return scan_t<uint8_t>(p, st);
    case TS_U16: return scan_t<uint16_t>(p, st);
    case TS_U32: return scan_t<uint32_t>(p, st);
    case TS_U64: return scan_t<uint64_t>(p, st);
    case TS_F16: return scan_t<half_t>(p, st);
    case TS_F32: return scan_t<float>(p, st);
    case TS_F64: return scan_t<double>(p, st);
  }
  return hipErrorInvalidValue;
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

// Bin b clipped to [0, n) (caller edges are not trusted to stay in range).
__device__ inline void bin_range(const MergeParams &p, int64_t bin, int64_t &s, int64_t &e) {
  s = edge_at(p.edges, p.n, p.nb, bin);
  e = edge_at(p.edges, p.n, p.nb, bin + 1);
  s = s < 0 ? 0 : (s > p.n ? p.n : s);
  e = e < s ? s : (e > p.n ? p.n : e);
}

__global__ __launch_bounds__(256) void k_merge(MergeParams p) {
  const int lane = lane_id();
  const int64_t bin = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (bin >= p.nb) return;
  int64_t s, e;
  bin_range(p, bin, s, e);
  if (s >= e) {
    if (lane == 0) p.cnt[bin] = 0;
    return;
  }
  int64_t imn, imx;
  merged_bin(p, s, e, bin, lane, imn, imx);
  if (lane != 0) return;
  int64_t v[4];
  int k = 0;
  if (p.m4) v[k++] = s;
  v[k++] = imn;
  v[k++] = imx;
  if (p.m4) v[k++] = e - 1;
  for (int a = 1; a < k; a++)
    for (int c = a; c > 0 && v[c - 1] > v[c]; c--) {
      int64_t t = v[c]; v[c] = v[c - 1]; v[c - 1] = t;
    }
  int m = 0;
  for (int a = 0; a < k; a++)
    if (a == 0 || v[a] != v[a - 1]) p.sel[4 * bin + m++] = v[a];
  p.cnt[bin] = m;
}

hipError_t launch_merge(const MergeParams &p, hipStream_t st) {
  k_merge<<<dim3((unsigned)((p.nb + 3) / 4)), dim3(256), 0, st>>>(p);
  return hipGetLastError();
}

// Per-bin argmin/argmax to caller arrays (-1 for empty bins).
__global__ __launch_bounds__(256) void k_binres_out(MergeParams p, int64_t *omin, int64_t *omax) {
  const int lane = lane_id();
  const int64_t bin = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (bin >= p.nb) return;
  int64_t s, e;
  bin_range(p, bin, s, e);
  int64_t imn = -1, imx = -1;
  if (s < e) merged_bin(p, s, e, bin, lane, imn, imx);
  if (lane == 0) {
    omin[bin] = imn;
    omax[bin] = imx;
  }
}

hipError_t launch_binres_to_outputs(const MergeParams &p, int64_t *imin, int64_t *imax, hipStream_t st) {
  k_binres_out<<<dim3((unsigned)((p.nb + 3) / 4)), dim3(256), 0, st>>>(p, imin, imax);
  return hipGetLastError();
}

// ------------------------------------------------------------------ compact

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

__global__ __launch_bounds__(1024) void k_compact(CompactParams p) {
  __shared__ int64_t lds[80];
  const int t = threadIdx.x;
  int64_t *out = p.out;
  if (p.all_n >= 0) {
    for (int64_t i = t; i < p.all_n; i += blockDim.x) out[i] = i;
    if (t == 0) *p.out_count = p.all_n;
    return;
  }
  const int64_t per = (p.nb + blockDim.x - 1) / blockDim.x;
  const int64_t b0 = (int64_t)t * per;
  const int64_t b1 = b0 + per < p.nb ? b0 + per : p.nb;
  int64_t local = 0;
  for (int64_t b = b0; b < b1; b++) local += p.cnt[b];
  int64_t total;
  int64_t off = block_exclusive_scan(local, lds, total);
  for (int64_t b = b0; b < b1; b++) {
    const int64_t k = p.cnt[b];
    for (int64_t j = 0; j < k; j++) out[off + j] = p.sel[4 * b + j] + p.index_offset;
    off += k;
  }
  if (t == 0) {
    if (p.endpoints_n > 0) {
      out[-1] = 0;
      out[total] = p.endpoints_n - 1;
      *p.out_count = total + 2;
    } else {
      *p.out_count = total;
    }
  }
}

hipError_t launch_compact(const CompactParams &p, hipStream_t st) {
  k_compact<<<dim3(1), dim3(1024), 0, st>>>(p);
  return hipGetLastError();
}

// ------------------------------------------------------------------ window

template <typename X>
__global__ void k_window(const X *x, int64_t n, int64_t xa, int64_t xb, int64_t *range) {
  using K = typename XKey<X>::K;
  const int lane = lane_id();
  const int w = threadIdx.x >> 6;
  // wave 0: first index with x >= xa; wave 1: first index with x > xb
  // (= first index with x >= xb + 1 for integers; xb + 1 saturates).
  K v;
  if (w == 0) {
    v = (K)xa;
    if (std::is_unsigned<K>::value && xa < 0) v = 0;
  } else {
    if (std::is_unsigned<K>::value && xb < 0) v = 0;
    else v = (K)xb == (K)(std::numeric_limits<K>::max()) ? (K)xb : (K)((K)xb + 1);
  }
  int64_t r = wave_lower_bound<X, K>(x, n, v, lane);
  if (w == 1 && !(std::is_unsigned<K>::value && xb < 0) && (K)xb == std::numeric_limits<K>::max()) r = n;
  if (lane == 0) range[w] = r;
}

hipError_t launch_window(const void *x, int xdt, int64_t n, int64_t xa, int64_t xb, int64_t *range,
                         hipStream_t st) {
  switch (xdt) {
    case TS_I32: k_window<int32_t><<<1, 128, 0, st>>>((const int32_t *)x, n, xa, xb, range); break;
    case TS_I64: k_window<int64_t><<<1, 128, 0, st>>>((const int64_t *)x, n, xa, xb, range); break;
    case TS_U32: k_window<uint32_t><<<1, 128, 0, st>>>((const uint32_t *)x, n, xa, xb, range); break;
    case TS_U64: k_window<uint64_t><<<1, 128, 0, st>>>((const uint64_t *)x, n, xa, xb, range); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tsds

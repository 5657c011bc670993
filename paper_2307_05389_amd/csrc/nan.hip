// nan.hip -- NaN-aware argmin/argmax scan for floating-point y.
//
// The paper notes that floats need a different initial value once NaN is
// handled (Sec. 2.1, Listing 1) but gives NaN no meaning.  The NaN-aware
// MinMax and M4 read it this way: NaN values are skipped, and a bin whose
// values are all NaN keeps its first index as both argmin and argmax (so M4
// keeps {first, last} there).  This file is compiled with NaN semantics on:
// every compare below relies on NaN comparing false.
//
// One wavefront reduces one fixed chunk, bin segment by bin segment (short
// segments one per lane, long ones across the wavefront with 16-byte loads).
// A lane's running result takes the first non-NaN value and then strictly
// smaller / larger ones in index order, so it holds its first occurrence;
// the wavefront keeps the least index among lanes holding the extreme.
// Results go to the same per-bin slots and per-chunk partials as the plain
// scan, keyed by the order-preserving 64-bit keys, with a segment that saw
// no value written as an absent partial (minimum key ~0 / maximum key 0,
// index INT64_MAX), which loses to every real key in the merge; a bin left
// with no index at all after the merge takes its first index.
#include <stdint.h>

#include "common.hpp"
#include "internal.hpp"
#include "scan_core.hpp"
#include "batch_core.hpp"

namespace tsds {

// Segments shorter than this are reduced by one lane.
constexpr int64_t kNanLane = 64;

template <typename T>
struct NanRun {
  using E = Elem<T>;
  using C = typename E::C;
  C vmn, vmx;
  int64_t imn, imx;
  __device__ void init() {
    vmn = E::highest();
    vmx = E::lowest();
    imn = INT64_MAX;
    imx = INT64_MAX;
  }
  __device__ void add(C v, int64_t i) {
    const bool num = v == v;
    if (v < vmn || (num && imn == INT64_MAX)) { vmn = v; imn = i; }
    if (vmx < v || (num && imx == INT64_MAX)) { vmx = v; imx = i; }
  }
  __device__ uint64_t kmin() const { return imn == INT64_MAX ? ~0ull : E::key(vmn); }
  __device__ uint64_t kmax() const { return imx == INT64_MAX ? 0ull : E::key(vmx); }
};

// Bin segment result: the bin's own slots when the bin lies inside the chunk
// (an all-NaN bin resolved to its first index s there), else the chunk's
// partial for the bin that starts before / continues after it.
__device__ inline void write_nan(const ScanParams &p, int64_t c, int64_t bin, int64_t s, bool before, bool after,
                                 uint64_t kmn, int64_t imn, uint64_t kmx, int64_t imx) {
  if (!before && !after) {
    p.binres[2 * bin] = imn == INT64_MAX ? s : imn;
    p.binres[2 * bin + 1] = imx == INT64_MAX ? s : imx;
  } else {
    Partial q;
    q.kmin = kmn;
    q.imin = imn;
    q.kmax = kmx;
    q.imax = imx;
    (before ? p.partL : p.partR)[c] = q;
  }
}

template <typename T>
__device__ void scan_chunk_nan(const ScanParams &p, int64_t c, int lane) {
  using E = Elem<T>;
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
    const bool small = valid && (hi - lo) < kNanLane;
    if (small) {
      NanRun<T> r;
      r.init();
      for (int64_t i = lo; i < hi; i++) r.add(E::load(y + i), i);
      write_nan(p, c, bb, s, before, after, r.kmin(), r.imn, r.kmax(), r.imx);
    }
    uint64_t big = ballot(valid && !small);
    while (big) {
      const int k = __builtin_ctzll(big);
      big &= big - 1;
      const int64_t slo = readlane(lo, k), shi = readlane(hi, k), sk = readlane(s, k), ek = readlane(e, k);
      const int64_t vlo = (slo + p.shift) / VEC, vhi = (shi + p.shift + VEC - 1) / VEC;
      NanRun<T> r;
      r.init();
      for (int64_t v0 = vlo + lane; v0 < vhi; v0 += 4 * kWave) {
        u32x4 d[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int64_t v = v0 + u * kWave;
          d[u] = v < vhi ? __builtin_nontemporal_load(base + v) : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int64_t v = v0 + u * kWave;
          if (v < vhi) {
#pragma unroll
            for (int j = 0; j < VEC; j++) {
              const int64_t i = v * VEC - p.shift + j;
              if (i >= slo && i < shi) r.add(extract<T>(d[u], j), i);
            }
          }
        }
      }
      const uint64_t kmn = r.kmin(), kmx = r.kmax();
      const uint64_t wkmn = wave_min(kmn), wkmx = wave_max(kmx);
      const int64_t rmn = wave_min(kmn == wkmn ? r.imn : INT64_MAX);
      const int64_t rmx = wave_min(kmx == wkmx ? r.imx : INT64_MAX);
      if (lane == 0) write_nan(p, c, b + k, sk, sk < c0, ek > c1, wkmn, rmn, wkmx, rmx);
    }
    const int64_t e63 = readlane(e, 63);
    if (e63 >= c1 || b + kWave >= p.nb) break;
    b += kWave;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_nan(ScanParams p) {
  const int64_t c = uniform((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  if (c >= p.nchunks) return;
  scan_chunk_nan<T>(p, c, lane_id());
}

// Batched mode: the persistent scan over one element type's NaN-aware tasks
// (same work split and task lookup as k_batch_scan).
template <typename T>
__global__ __launch_bounds__(256) void k_batch_scan_nan(const BatchTask *__restrict__ tasks,
                                                        const int64_t *__restrict__ cb,
                                                        const int32_t *__restrict__ tix, int64_t ntasks,
                                                        int64_t total, char *ws) {
  const int lane = lane_id();
  const int64_t W = (int64_t)gridDim.x * 4;
  const int64_t w = uniform((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  const int64_t i0 = total * w / W, i1 = total * (w + 1) / W;
#pragma nounroll
  for (int64_t item = i0; item < i1; item++) {
    const BatchTask *tk = tasks + group_task_of_item(cb, tix, ntasks, item, lane);
    const ScanParams sp = task_scan_params_uniform(ws, tk, 0);
    scan_chunk_nan<T>(sp, item - uniform(tk->chunk_begin), lane);
  }
}

hipError_t launch_batch_scan_nan(const BatchArgs &a, const BatchGroup &g, int64_t grid_blocks, hipStream_t st) {
  if (g.total == 0) return hipSuccess;
  int64_t gb = grid_blocks;
  if (gb > (g.total + 3) / 4) gb = (g.total + 3) / 4;
  if (gb < 1) gb = 1;
  const dim3 grid((unsigned)gb), block(256);
  switch (g.ydt) {
    case TS_F16: k_batch_scan_nan<half_t><<<grid, block, 0, st>>>(a.tasks, g.cb, g.tix, g.ntasks, g.total, a.ws); break;
    case TS_F32: k_batch_scan_nan<float><<<grid, block, 0, st>>>(a.tasks, g.cb, g.tix, g.ntasks, g.total, a.ws); break;
    case TS_F64: k_batch_scan_nan<double><<<grid, block, 0, st>>>(a.tasks, g.cb, g.tix, g.ntasks, g.total, a.ws); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_scan_nan(int ydt, const ScanParams &p, hipStream_t st) {
  const dim3 grid((unsigned)((p.nchunks + 3) / 4)), block(256);
  switch (ydt) {
    case TS_F16: k_scan_nan<half_t><<<grid, block, 0, st>>>(p); break;
    case TS_F32: k_scan_nan<float><<<grid, block, 0, st>>>(p); break;
    case TS_F64: k_scan_nan<double><<<grid, block, 0, st>>>(p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tsds

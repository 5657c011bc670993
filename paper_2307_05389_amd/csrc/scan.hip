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
//
// The merge of straddling bins and the compaction are in select.hip.
#include <hip/hip_ext.h>

#include <limits>
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"
#include "scan_core.hpp"

namespace tsds {

// ------------------------------------------------------------------ edges

template <typename X>
__global__ __launch_bounds__(256) void k_edges_x(const X *x, int64_t n, int64_t nb, int64_t *edges) {
  const int lane = lane_id();
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b > nb) return;
  const int64_t s = edge_start<X>(x, n, nb, b, lane);
  if (lane == 0) edges[b] = s;
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
    case TS_I32: k_edges_x<int32_t><<<grid, block, 0, st>>>((const int32_t *)x, n, nb, edges); break;
    case TS_I64: k_edges_x<int64_t><<<grid, block, 0, st>>>((const int64_t *)x, n, nb, edges); break;
    case TS_U32: k_edges_x<uint32_t><<<grid, block, 0, st>>>((const uint32_t *)x, n, nb, edges); break;
    case TS_U64: k_edges_x<uint64_t><<<grid, block, 0, st>>>((const uint64_t *)x, n, nb, edges); break;
    case TS_F32: k_edges_x<float><<<grid, block, 0, st>>>((const float *)x, n, nb, edges); break;
    case TS_F64: k_edges_x<double><<<grid, block, 0, st>>>((const double *)x, n, nb, edges); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// With events, the launch goes through hipExtLaunchKernel, which stamps
// them with the dispatch's own start and end times (no marker packets
// around the kernel).
static void launch_k(void (*k)(ScanParams), dim3 grid, dim3 block, size_t lds, hipStream_t st, hipEvent_t e0,
                     hipEvent_t e1, const ScanParams &p) {
  if (e0 || e1) {
    void *args[] = {(void *)&p};
    (void)hipExtLaunchKernel((const void *)k, grid, block, args, lds, st, e0, e1, 0);
  } else {
    hipLaunchKernelGGL(k, grid, block, (uint32_t)lds, st, p);
  }
}

// Tile shapes: 16-byte vectors per lane per tile x tiles in flight.
template <typename T>
static hipError_t scan_t(const ScanParams &p, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  dim3 grid((unsigned)((p.nchunks + 3) / 4)), block(256);
  if (p.stage) {
    const size_t lds = 4 * sizeof(u32x4) * (size_t)staged_lds_vectors(p.chunk, 16 / (int)sizeof(T));
    launch_k(k_scan_staged<T>, grid, block, lds, st, e0, e1, p);
    return hipGetLastError();
  }
  void (*k)(ScanParams);
  if (p.variant == kScanStreamVariant && !p.xclass) {
    launch_k(k_scan_stream<T, sizeof(T) >= 4 ? 8 : sizeof(T) == 2 ? 4 : 2>, grid, block, 0, st, e0, e1, p);
    return hipGetLastError();
  }
  if (p.xclass) {
    switch (p.variant) {
      case 0: k = k_scan_xc<T, 4, 2>; break;
      case 1: k = k_scan_xc<T, 4, 1>; break;
      case 2: k = k_scan_xc<T, 8, 1>; break;
      default: k = k_scan_xc<T, 2, 2>; break;
    }
  } else {
    switch (p.variant) {
      case 0: k = k_scan<T, 4, 2>; break;
      case 1: k = k_scan<T, 4, 1>; break;
      case 2: k = k_scan<T, 8, 1>; break;
      default: k = k_scan<T, 2, 2>; break;
    }
  }
  launch_k(k, grid, block, 0, st, e0, e1, p);
  return hipGetLastError();
}

hipError_t launch_scan(int ydt, const ScanParams &p, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  switch (ydt) {
    case TS_I8: return scan_t<int8_t>(p, st, e0, e1);
    case TS_I16: return scan_t<int16_t>(p, st, e0, e1);
    case TS_I32: return scan_t<int32_t>(p, st, e0, e1);
    case TS_I64: return scan_t<int64_t>(p, st, e0, e1);
    case TS_U8: return scan_t<uint8_t>(p, st, e0, e1);
    case TS_U16: return scan_t<uint16_t>(p, st, e0, e1);
    case TS_U32: return scan_t<uint32_t>(p, st, e0, e1);
    case TS_U64: return scan_t<uint64_t>(p, st, e0, e1);
    case TS_F16: return scan_t<half_t>(p, st, e0, e1);
    case TS_F32: return scan_t<float>(p, st, e0, e1);
    case TS_F64: return scan_t<double>(p, st, e0, e1);
  }
  return hipErrorInvalidValue;
}

}  // namespace tsds

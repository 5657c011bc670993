// window.hip -- x-window bounds and the serving loop's host transfers.
//
// A window [xa, xb] of a sorted x is turned into an index range by two
// wavefront searches (the zoom requests of the serving loop, and the
// ts_window entry point).  The serving loop moves its request table, window
// ranges and results through host-mapped pinned memory with the small copy
// kernels below instead of memcpy calls.
#include <limits>
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"
#include "scan_core.hpp"

namespace tsds {

// ------------------------------------------------------------------ window

// First index i in [0, n) with x[i] >= xa (w = 0) or x[i] > xb (w = 1), by a
// 64-ary wavefront search; values are compared in 64 bits (int64 or uint64).
template <typename X>
__device__ int64_t window_bound(const X *x, int64_t n, int64_t xa, int64_t xb, int w, int lane) {
  using K = typename XKey<X>::K;
  if (w == 0) {
    if (std::is_unsigned<K>::value && xa < 0) return 0;
    return wave_lower_bound<X, K>(x, 0, n, (K)xa, lane);
  }
  if (std::is_unsigned<K>::value && xb < 0) return 0;
  if ((K)xb == std::numeric_limits<K>::max()) return n;
  return wave_lower_bound<X, K>(x, 0, n, (K)((K)xb + 1), lane);
}

__device__ int64_t window_bound_any(const void *x, int xdt, int64_t n, int64_t xa, int64_t xb, int w, int lane) {
  switch (xdt) {
    case TS_I32: return window_bound<int32_t>((const int32_t *)x, n, xa, xb, w, lane);
    case TS_I64: return window_bound<int64_t>((const int64_t *)x, n, xa, xb, w, lane);
    case TS_U32: return window_bound<uint32_t>((const uint32_t *)x, n, xa, xb, w, lane);
    case TS_U64: return window_bound<uint64_t>((const uint64_t *)x, n, xa, xb, w, lane);
  }
  return 0;
}

__global__ void k_window(const void *x, int xdt, int64_t n, int64_t xa, int64_t xb, int64_t *range) {
  const int lane = lane_id(), w = threadIdx.x >> 6;
  const int64_t r = window_bound_any(x, xdt, n, xa, xb, w, lane);
  if (lane == 0) range[w] = r;
}

hipError_t launch_window(const void *x, int xdt, int64_t n, int64_t xa, int64_t xb, int64_t *range,
                         hipStream_t st) {
  if (xdt != TS_I32 && xdt != TS_I64 && xdt != TS_U32 && xdt != TS_U64) return hipErrorInvalidValue;
  k_window<<<1, 128, 0, st>>>(x, xdt, n, xa, xb, range);
  return hipGetLastError();
}

// One workgroup of two wavefronts per request.
__global__ void k_windows(WindowBatch wb) {
  const int i = blockIdx.x;
  if (i >= wb.count) return;
  const int lane = lane_id(), w = threadIdx.x >> 6;
  const int64_t r = window_bound_any(wb.x[i], wb.xdt[i], wb.n[i], wb.xa[i], wb.xb[i], w, lane);
  if (lane == 0) {
    wb.ranges[2 * i + w] = r;
    if (wb.host_ranges) wb.host_ranges[2 * i + w] = r;
  }
}

hipError_t launch_windows(const WindowBatch &wb, hipStream_t st) {
  if (wb.count <= 0) return hipSuccess;
  k_windows<<<dim3((unsigned)wb.count), dim3(128), 0, st>>>(wb);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_copy_bytes(char *dst, const char *src, size_t bytes) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (((uintptr_t)dst | (uintptr_t)src) % 8 == 0) {
    const size_t words = bytes / 8;
    for (size_t i = t; i < words; i += stride) ((uint64_t *)dst)[i] = ((const uint64_t *)src)[i];
    for (size_t i = words * 8 + t; i < bytes; i += stride) dst[i] = src[i];
  } else {
    for (size_t i = t; i < bytes; i += stride) dst[i] = src[i];
  }
}

hipError_t launch_copy_bytes(void *dst, const void *src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  size_t blocks = (bytes / 8 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  k_copy_bytes<<<dim3((unsigned)blocks), dim3(256), 0, st>>>((char *)dst, (const char *)src, bytes);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_export_rows(const int64_t *counts, const int64_t *rows, int64_t row,
                                                     int64_t *h_counts, int64_t *h_rows) {
  const int i = blockIdx.x;
  const int64_t c = counts[i];
  for (int64_t j = threadIdx.x; j < c; j += blockDim.x) h_rows[i * row + j] = rows[i * row + j];
  if (threadIdx.x == 0) h_counts[i] = c;
}

hipError_t launch_export_rows(const int64_t *counts, const int64_t *rows, int64_t row, int n, int64_t *h_counts,
                              int64_t *h_rows, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_export_rows<<<dim3((unsigned)n), dim3(256), 0, st>>>(counts, rows, row, h_counts, h_rows);
  return hipGetLastError();
}

}  // namespace tsds

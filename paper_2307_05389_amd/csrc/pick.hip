// pick.hip -- EveryNth and the gather of selected points.
//
// EveryNth (named among the downsamplers in Sec. 1, timed in Table 1) keeps
// every k-th index with k = ceil(n / n_out): it reads no data and writes at
// most n_out indices.  The gather turns selected indices into the values a
// plot draws (the indices retrieve the representative subset, Sec. 2.3): one
// pass that reads the count, the indices and x[i], y[i] and writes both
// outputs, with x and y moved as raw words of their element size.
#include <stdint.h>

#include "common.hpp"
#include "internal.hpp"

namespace tsds {

// ------------------------------------------------------------------ EveryNth

__global__ void __launch_bounds__(256) k_everynth(int64_t k, int64_t m, int64_t *out, int64_t *count) {
  const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = first; i < m; i += stride) out[i] = i * k;
  if (first == 0) *count = m;
}

hipError_t launch_everynth(int64_t k, int64_t m, int64_t *out, int64_t *count, hipStream_t st) {
  const int64_t want = m > 0 ? (m + 255) / 256 : 1;
  const int64_t blocks = want < 4096 ? want : 4096;
  k_everynth<<<(unsigned)blocks, 256, 0, st>>>(k, m, out, count);
  return hipGetLastError();
}

// ------------------------------------------------------------------ gather

// Selected point i (i < min(*count, cap)) -> xo[i] = x[idx[i]], yo[i] = y[idx[i]].
// An index outside [0, n) writes nothing (its outputs keep their contents).
template <typename XW, typename YW>
__global__ void __launch_bounds__(256) k_gather(const XW *__restrict__ x, const YW *__restrict__ y,
                                                int64_t n, const int64_t *__restrict__ idx,
                                                const int64_t *__restrict__ count, int64_t cap,
                                                XW *__restrict__ xo, YW *__restrict__ yo) {
  int64_t m = *count;
  m = m < 0 ? 0 : m > cap ? cap : m;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const int64_t j = idx[i];
    if (j < 0 || j >= n) continue;
    yo[i] = y[j];
    if (xo) xo[i] = x[j];
  }
}

template <typename XW>
static void gather_y(const void *x, const void *y, int ys, int64_t n, const int64_t *idx,
                     const int64_t *count, int64_t cap, void *xo, void *yo, unsigned blocks, hipStream_t st) {
  const XW *xp = (const XW *)x;
  XW *xop = (XW *)xo;
  switch (ys) {
    case 1: k_gather<XW, uint8_t><<<blocks, 256, 0, st>>>(xp, (const uint8_t *)y, n, idx, count, cap, xop, (uint8_t *)yo); break;
    case 2: k_gather<XW, uint16_t><<<blocks, 256, 0, st>>>(xp, (const uint16_t *)y, n, idx, count, cap, xop, (uint16_t *)yo); break;
    case 4: k_gather<XW, uint32_t><<<blocks, 256, 0, st>>>(xp, (const uint32_t *)y, n, idx, count, cap, xop, (uint32_t *)yo); break;
    default: k_gather<XW, uint64_t><<<blocks, 256, 0, st>>>(xp, (const uint64_t *)y, n, idx, count, cap, xop, (uint64_t *)yo); break;
  }
}

hipError_t launch_gather(const void *x, int xs, const void *y, int ys, int64_t n, const int64_t *idx,
                         const int64_t *count, int64_t cap, void *xo, void *yo, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const int64_t want = (cap + 255) / 256;
  const unsigned blocks = (unsigned)(want < 2048 ? want : 2048);
  if (!xo || xs == 0) gather_y<uint64_t>(nullptr, y, ys, n, idx, count, cap, nullptr, yo, blocks, st);
  else if (xs == 4) gather_y<uint32_t>(x, y, ys, n, idx, count, cap, xo, yo, blocks, st);
  else gather_y<uint64_t>(x, y, ys, n, idx, count, cap, xo, yo, blocks, st);
  return hipGetLastError();
}

}  // namespace tsds

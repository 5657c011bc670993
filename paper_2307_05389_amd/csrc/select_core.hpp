// select_core.hpp -- compaction of per-bin selections by one workgroup (the
// step after the per-bin merge: an exclusive scan of the per-bin counts, then
// each bin's indices written at its offset, so the output is strictly
// increasing).
#pragma once

#include "common.hpp"
#include "scan_core.hpp"

namespace tsds {

// Compacts bins [lo, hi) (cnt[b] <= 4 indices in sel[4b .. 4b + cnt[b]) )
// into dst[base ..) with index_offset added; returns the number written to
// every thread.  Thread t takes bins lo + r*T + t for rounds r = 0, 1, ..., so
// a wavefront's loads and stores are contiguous.  Four rounds are scanned at
// once: round q's counts go to bits 16q.. of one 64-bit value per thread (a
// round's block sum is at most 4T <= 4096, so the fields never carry into
// each other), and one block scan gives every round's exclusive prefix and
// total.  All loads of a group of four rounds are issued before the scan (a
// slot beyond a bin's count is read but not used).
__device__ inline int64_t compact_bins(const int64_t *__restrict__ cnt, const int64_t *__restrict__ sel, int64_t lo,
                                       int64_t hi, int64_t *__restrict__ dst, int64_t base, int64_t index_offset,
                                       int64_t *lds) {
  const int64_t T = blockDim.x, t = threadIdx.x;
  const int64_t R = (hi - lo + T - 1) / T;
  int64_t done = 0;  // outputs of the rounds before the current group
  for (int64_t r0 = 0; r0 < R; r0 += 4) {
    int64_t c[4], s[4][4];
    int64_t packed = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      c[q] = 0;
#pragma unroll
      for (int v = 0; v < 4; v++) s[q][v] = 0;
      if (r0 + q < R) {  // uniform: rounds past the last are not loaded
        const int64_t b = lo + (r0 + q) * T + t;
        const bool in = b < hi;
        c[q] = in ? cnt[b] : 0;
        const int64_t bq = in ? b : lo;  // an in-range bin: the loads stay inside sel
#pragma unroll
        for (int v = 0; v < 4; v++) s[q][v] = sel[4 * bq + v];
      }
      packed += c[q] << (16 * q);
    }
    int64_t tot;
    const int64_t ex = block_exclusive_scan(packed, lds, tot);
    int64_t off = base + done;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int64_t o = off + ((ex >> (16 * q)) & 0xffff);
#pragma unroll
      for (int v = 0; v < 4; v++)
        if (v < c[q]) dst[o + v] = s[q][v] + index_offset;
      off += (tot >> (16 * q)) & 0xffff;
    }
    done = off - base;
  }
  return done;
}

}  // namespace tsds

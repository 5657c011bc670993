// select_core.hpp -- compaction of per-bin selections by one workgroup (the
// step after the per-bin merge: an exclusive scan of the per-bin counts, then
// each bin's indices written at its offset, so the output is strictly
// increasing).
#pragma once

#include "common.hpp"
#include "scan_core.hpp"

namespace tsds {

// Bins handled per round trip by one thread.
constexpr int kCompactRun = 8;

// Compacts bins [lo, hi) (cnt[b] indices in sel[4b .. 4b + cnt[b]) ) into
// dst[base ..) with index_offset added; returns the number written to every
// thread.  Each thread takes a contiguous run of bins; the counts of up to
// kCompactRun bins and all four selection slots of each are loaded together
// (a slot beyond a bin's count is read but not used), so a run costs one
// round trip to memory instead of one per bin.
__device__ inline int64_t compact_bins(const int64_t *__restrict__ cnt, const int64_t *__restrict__ sel, int64_t lo,
                                       int64_t hi, int64_t *__restrict__ dst, int64_t base, int64_t index_offset,
                                       int64_t *lds) {
  const int64_t T = blockDim.x;
  const int64_t per = (hi - lo + T - 1) / T;
  const int64_t b0 = lo + (int64_t)threadIdx.x * per;
  const int64_t b1 = b0 + per < hi ? b0 + per : hi;
  int64_t local = 0;
  for (int64_t b = b0; b < b1; b += kCompactRun) {
    int64_t c[kCompactRun];
#pragma unroll
    for (int u = 0; u < kCompactRun; u++) c[u] = b + u < b1 ? cnt[b + u] : 0;
#pragma unroll
    for (int u = 0; u < kCompactRun; u++) local += c[u];
  }
  int64_t total;
  int64_t off = base + block_exclusive_scan(local, lds, total);
  for (int64_t b = b0; b < b1; b += kCompactRun) {
    int64_t c[kCompactRun], s[kCompactRun][4];
#pragma unroll
    for (int u = 0; u < kCompactRun; u++) {
      const bool in = b + u < b1;
      c[u] = in ? cnt[b + u] : 0;
      const int64_t q = in ? b + u : b0;  // an in-range bin: the loads stay inside sel
#pragma unroll
      for (int v = 0; v < 4; v++) s[u][v] = sel[4 * q + v];
    }
#pragma unroll
    for (int u = 0; u < kCompactRun; u++) {
#pragma unroll
      for (int v = 0; v < 4; v++)
        if (v < c[u]) dst[off + v] = s[u][v] + index_offset;
      off += c[u];
    }
  }
  return total;
}

}  // namespace tsds

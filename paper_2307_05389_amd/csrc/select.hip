// select.hip -- per-bin selection and compaction after the argmin/argmax
// scan (scan.hip):
//
//   k_merge         one wavefront per bin: lexicographic merge of the partials
//                   of a straddling bin, then the bin's sorted distinct
//                   selection (k_merge_lanes: one bin per thread).
//   k_bins_direct   one wavefront reduces a whole bin and writes its selection
//                   (replaces the chunked scan and the merge).
//   k_bins_block    the same with a workgroup of four wavefronts per bin.
//   k_compact       one workgroup: exclusive scan of the per-bin counts and
//                   the compaction into strictly increasing indices (many
//                   workgroups above kCompactSingleMax bins).
#include <limits>
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"
#include "scan_core.hpp"
#include "select_core.hpp"

namespace tsds {

// ------------------------------------------------------------------ merge

// Merge + selection of one bin by one wavefront (writes sel/cnt).
__device__ inline void merge_one_bin(const MergeParams &p, int64_t bin, int lane) {
  int64_t s, e;
  bin_range(p, bin, s, e);
  if (s >= e) {
    if (lane == 0) p.cnt[bin] = 0;
    return;
  }
  int64_t imn, imx;
  merged_bin(p, s, e, bin, lane, imn, imx);
  if (imn == INT64_MAX) imn = s;  // only the NaN-aware scan leaves a bin without a value
  if (imx == INT64_MAX) imx = s;
  if (lane == 0) p.cnt[bin] = bin_selection(s, e, imn, imx, p.m4, p.sel + 4 * bin);
}

__global__ __launch_bounds__(256) void k_merge(MergeParams p) {
  const int64_t bin = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (bin < p.nb) merge_one_bin(p, bin, lane_id());
}

// One bin per thread (bins spanning few chunks).
__global__ __launch_bounds__(256) void k_merge_lanes(MergeParams p) {
  const int64_t bin = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (bin >= p.nb) return;
  int64_t s, e;
  bin_range(p, bin, s, e);
  if (s >= e) {
    p.cnt[bin] = 0;
    return;
  }
  int64_t imn, imx;
  merged_bin_lane(p, s, e, bin, imn, imx);
  if (imn == INT64_MAX) imn = s;
  if (imx == INT64_MAX) imx = s;
  p.cnt[bin] = bin_selection(s, e, imn, imx, p.m4, p.sel + 4 * bin);
}

// One wavefront per bin reduces the whole bin (U vectors per lane per tile,
// NB tiles in flight) and writes its selection, so no per-chunk partials and
// no merge launch are needed.
template <typename T, int U, int NB>
__global__ __launch_bounds__(256) void k_bins_direct(ScanParams sp, MergeParams mp) {
  const int64_t bin = uniform((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  if (bin >= mp.nb) return;
  const int lane = lane_id();
  int64_t s, e;
  bin_range(mp, bin, s, e);
  if (s >= e) {
    if (lane == 0) mp.cnt[bin] = 0;
    return;
  }
  const u32x4 *__restrict__ base = (const u32x4 *)((const T *)sp.y - sp.shift);
  u32x4 buf[NB][U];
  SegState<typename Elem<T>::C> st;
  wave_segment<T, U, NB>(base, sp.shift, s, e, lane, buf, 0, st);
  if (lane == 0) mp.cnt[bin] = bin_selection(s, e, st.imn, st.imx, mp.m4, mp.sel + 4 * bin);
}

template <typename T>
static void launch_direct_t(int variant, dim3 grid, dim3 block, const ScanParams &sp, const MergeParams &mp,
                            hipStream_t st) {
  switch (variant) {
    case 1: k_bins_direct<T, 4, 1><<<grid, block, 0, st>>>(sp, mp); break;
    case 2: k_bins_direct<T, 8, 1><<<grid, block, 0, st>>>(sp, mp); break;
    case 3: k_bins_direct<T, 2, 2><<<grid, block, 0, st>>>(sp, mp); break;
    default: k_bins_direct<T, 4, 2><<<grid, block, 0, st>>>(sp, mp); break;
  }
}

// sp.variant picks the tile shape (0 = 4x2, 1 = 4x1, 2 = 8x1, 3 = 2x2).
// Long bins and too few of them for a wavefront each to fill the GPU: a
// workgroup of kBlockWaves wavefronts per bin, wavefront w reducing the w-th
// contiguous part of the bin (the same tile fold), then the first wavefront's
// first lane combining the parts in index order (strict comparisons: an
// equal extreme in a later part never replaces an earlier one) and writing
// the bin's selection.
constexpr int kBlockWaves = 4;

template <typename T, int U, int NB>
__global__ __launch_bounds__(64 * kBlockWaves) void k_bins_block(ScanParams sp, MergeParams mp) {
  using C = typename Elem<T>::C;
  __shared__ C smn[kBlockWaves], smx[kBlockWaves];
  __shared__ int64_t simn[kBlockWaves], simx[kBlockWaves];
  __shared__ int shas[kBlockWaves];
  const int64_t bin = uniform((int64_t)blockIdx.x);
  const int w = uniform((int)(threadIdx.x >> 6));
  const int lane = lane_id();
  int64_t s, e;
  bin_range(mp, bin, s, e);
  if (s >= e) {  // the same for the whole workgroup
    if (threadIdx.x == 0) mp.cnt[bin] = 0;
    return;
  }
  const int64_t len = e - s;
  const int64_t w0 = uniform(s + len * w / kBlockWaves), w1 = uniform(s + len * (w + 1) / kBlockWaves);
  SegState<C> st;
  st.has = false;
  if (w0 < w1) {
    const u32x4 *__restrict__ base = (const u32x4 *)((const T *)sp.y - sp.shift);
    u32x4 buf[NB][U];
    wave_segment<T, U, NB>(base, sp.shift, w0, w1, lane, buf, 0, st);
  }
  if (lane == 0) {
    smn[w] = st.vmn;
    smx[w] = st.vmx;
    simn[w] = st.imn;
    simx[w] = st.imx;
    shas[w] = st.has ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    C vmn = smn[0], vmx = smx[0];
    int64_t imn = simn[0], imx = simx[0];
    bool has = false;
    for (int k = 0; k < kBlockWaves; k++) {
      if (!shas[k]) continue;
      if (!has || smn[k] < vmn) {
        vmn = smn[k];
        imn = simn[k];
      }
      if (!has || vmx < smx[k]) {
        vmx = smx[k];
        imx = simx[k];
      }
      has = true;
    }
    mp.cnt[bin] = bin_selection(s, e, imn, imx, mp.m4, mp.sel + 4 * bin);
  }
}

template <typename T>
static void launch_block_t(int variant, dim3 grid, dim3 block, const ScanParams &sp, const MergeParams &mp,
                           hipStream_t st) {
  switch (variant) {
    case 1: k_bins_block<T, 4, 1><<<grid, block, 0, st>>>(sp, mp); break;
    case 2: k_bins_block<T, 8, 1><<<grid, block, 0, st>>>(sp, mp); break;
    case 3: k_bins_block<T, 2, 2><<<grid, block, 0, st>>>(sp, mp); break;
    default: k_bins_block<T, 4, 2><<<grid, block, 0, st>>>(sp, mp); break;
  }
}

hipError_t launch_bins_block(int ydt, const ScanParams &sp, const MergeParams &mp, hipStream_t st) {
  const dim3 grid((unsigned)mp.nb), block(64 * kBlockWaves);
  const int v = sp.variant;
  switch (ydt) {
    case TS_I8: launch_block_t<int8_t>(v, grid, block, sp, mp, st); break;
    case TS_I16: launch_block_t<int16_t>(v, grid, block, sp, mp, st); break;
    case TS_I32: launch_block_t<int32_t>(v, grid, block, sp, mp, st); break;
    case TS_I64: launch_block_t<int64_t>(v, grid, block, sp, mp, st); break;
    case TS_U8: launch_block_t<uint8_t>(v, grid, block, sp, mp, st); break;
    case TS_U16: launch_block_t<uint16_t>(v, grid, block, sp, mp, st); break;
    case TS_U32: launch_block_t<uint32_t>(v, grid, block, sp, mp, st); break;
    case TS_U64: launch_block_t<uint64_t>(v, grid, block, sp, mp, st); break;
    case TS_F16: launch_block_t<half_t>(v, grid, block, sp, mp, st); break;
    case TS_F32: launch_block_t<float>(v, grid, block, sp, mp, st); break;
    case TS_F64: launch_block_t<double>(v, grid, block, sp, mp, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bins_direct(int ydt, const ScanParams &sp, const MergeParams &mp, hipStream_t st) {
  const dim3 grid((unsigned)((mp.nb + 3) / 4)), block(256);
  const int v = sp.variant;
  switch (ydt) {
    case TS_I8: launch_direct_t<int8_t>(v, grid, block, sp, mp, st); break;
    case TS_I16: launch_direct_t<int16_t>(v, grid, block, sp, mp, st); break;
    case TS_I32: launch_direct_t<int32_t>(v, grid, block, sp, mp, st); break;
    case TS_I64: launch_direct_t<int64_t>(v, grid, block, sp, mp, st); break;
    case TS_U8: launch_direct_t<uint8_t>(v, grid, block, sp, mp, st); break;
    case TS_U16: launch_direct_t<uint16_t>(v, grid, block, sp, mp, st); break;
    case TS_U32: launch_direct_t<uint32_t>(v, grid, block, sp, mp, st); break;
    case TS_U64: launch_direct_t<uint64_t>(v, grid, block, sp, mp, st); break;
    case TS_F16: launch_direct_t<half_t>(v, grid, block, sp, mp, st); break;
    case TS_F32: launch_direct_t<float>(v, grid, block, sp, mp, st); break;
    case TS_F64: launch_direct_t<double>(v, grid, block, sp, mp, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_merge(const MergeParams &p, hipStream_t st) {
  if (p.n / p.nb <= kLaneMergeChunks * p.chunk)
    k_merge_lanes<<<dim3((unsigned)((p.nb + 255) / 256)), dim3(256), 0, st>>>(p);
  else
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

// Compaction by one workgroup of any size: exclusive scan of the per-bin
// counts and the strictly increasing output (or 0..all_n-1).
__device__ void compact_block(const CompactParams &p, int64_t *lds) {
  const int t = threadIdx.x;
  int64_t *out = p.out;
  if (p.all_n >= 0) {
    for (int64_t i = t; i < p.all_n; i += blockDim.x) out[i] = i;
    if (t == 0) *p.out_count = p.all_n;
    return;
  }
  const int64_t total = compact_bins(p.cnt, p.sel, 0, p.nb, out, 0, p.index_offset, lds);
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

__global__ __launch_bounds__(1024) void k_compact(CompactParams p) {
  __shared__ int64_t lds[80];
  compact_block(p, lds);
}

// out[i] = i for i < all_n, many workgroups.
__global__ __launch_bounds__(256) void k_fill_all(CompactParams p) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.all_n; i += stride) p.out[i] = i;
  if (blockIdx.x == 0 && threadIdx.x == 0) *p.out_count = p.all_n;
}

// Multi-workgroup compaction for many bins, in three launches: per-workgroup
// sums of the counts of kCompactBins bins, one workgroup's exclusive scan of
// those sums (plus the count and end points), then every workgroup writes its
// bins' indices from its offset.
__global__ __launch_bounds__(256) void k_compact_sums(CompactParams p) {
  __shared__ int64_t lds[80];
  const int64_t b0 = (int64_t)blockIdx.x * kCompactBins;
  const int64_t b1 = b0 + kCompactBins < p.nb ? b0 + kCompactBins : p.nb;
  int64_t local = 0;
  for (int64_t b = b0 + threadIdx.x; b < b1; b += blockDim.x) local += p.cnt[b];
  int64_t total;
  (void)block_exclusive_scan(local, lds, total);
  if (threadIdx.x == 0) p.bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_compact_offsets(CompactParams p, int64_t nblk) {
  __shared__ int64_t lds[80];
  int64_t carry = 0;
  for (int64_t i0 = 0; i0 < nblk; i0 += blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    const int64_t v = i < nblk ? p.bsum[i] : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan(v, lds, tot);
    if (i < nblk) p.bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    if (p.endpoints_n > 0) {
      p.out[-1] = 0;
      p.out[carry] = p.endpoints_n - 1;
      *p.out_count = carry + 2;
    } else {
      *p.out_count = carry;
    }
  }
}

__global__ __launch_bounds__(256) void k_compact_write(CompactParams p) {
  __shared__ int64_t lds[80];
  const int64_t lo = (int64_t)blockIdx.x * kCompactBins;
  const int64_t hi = lo + kCompactBins < p.nb ? lo + kCompactBins : p.nb;
  (void)compact_bins(p.cnt, p.sel, lo, hi, p.out, p.bsum[blockIdx.x], p.index_offset, lds);
}

// Up to kCompactPrefixBlocks workgroups: the offsets scan is folded into the
// writes (two launches instead of three).  Every workgroup sums the block
// sums in front of it itself (at most that many values, from L2) instead of
// reading them from a separate scan; the last one also writes the count and
// the end points.
constexpr int64_t kCompactPrefixBlocks = 512;

__global__ __launch_bounds__(256) void k_compact_write_prefix(CompactParams p, int64_t nblk) {
  __shared__ int64_t lds[80];
  const int64_t blk = blockIdx.x;
  int64_t part = 0;
  for (int64_t j = threadIdx.x; j < blk; j += blockDim.x) part += p.bsum[j];
  int64_t before;
  (void)block_exclusive_scan(part, lds, before);  // `before` = the block's total: sum of bsum[0, blk)
  __syncthreads();
  const int64_t lo = blk * kCompactBins;
  const int64_t hi = lo + kCompactBins < p.nb ? lo + kCompactBins : p.nb;
  (void)compact_bins(p.cnt, p.sel, lo, hi, p.out, before, p.index_offset, lds);
  if (blk == nblk - 1 && threadIdx.x == 0) {
    const int64_t total = before + p.bsum[blk];
    if (p.endpoints_n > 0) {
      p.out[-1] = 0;
      p.out[total] = p.endpoints_n - 1;
      *p.out_count = total + 2;
    } else {
      *p.out_count = total;
    }
  }
}

hipError_t launch_compact(const CompactParams &p, hipStream_t st) {
  if (p.all_n >= 0) {
    int64_t blocks = (p.all_n + 1023) / 1024;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    k_fill_all<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(p);
    return hipGetLastError();
  }
  if (p.nb <= kCompactSingleMax || !p.bsum) {
    k_compact<<<dim3(1), dim3(1024), 0, st>>>(p);
    return hipGetLastError();
  }
  const int64_t nblk = compact_blocks(p.nb);
  k_compact_sums<<<dim3((unsigned)nblk), dim3(256), 0, st>>>(p);
  if (nblk <= kCompactPrefixBlocks) {
    k_compact_write_prefix<<<dim3((unsigned)nblk), dim3(256), 0, st>>>(p, nblk);
    return hipGetLastError();
  }
  k_compact_offsets<<<dim3(1), dim3(1024), 0, st>>>(p, nblk);
  k_compact_write<<<dim3((unsigned)nblk), dim3(256), 0, st>>>(p);
  return hipGetLastError();
}

}  // namespace tsds

// api.cpp -- the extern "C" entry points of libtsds: argument validation,
// workspace layout and the launch sequence of each downsampler.  Every
// check happens before the first launch, so an error leaves the caller's
// outputs untouched.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "common.hpp"
#include "internal.hpp"
#include "tsds.h"

namespace tsds {

size_t lttb_group_count(int64_t n_out);

static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

static int hip_fail(hipError_t e, const char *what) {
  return fail(TS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t elem_size(int dt) {
  switch (dt) {
    case TS_I8: case TS_U8: return 1;
    case TS_I16: case TS_U16: case TS_F16: return 2;
    case TS_I32: case TS_U32: case TS_F32: return 4;
    case TS_I64: case TS_U64: case TS_F64: return 8;
  }
  return 0;
}

int vec_width(int dt) { return 16 / (int)elem_size(dt); }

static bool x_dtype_ok(int dt) {
  return dt == TS_I32 || dt == TS_I64 || dt == TS_U32 || dt == TS_U64 || dt == TS_F32 || dt == TS_F64;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// ------------------------------------------------------------------ tuning

// Scan launch shape per dtype: tile variant (see launch_scan) and chunk bytes,
// from sweeps on MI355X over 800 MB inputs (each pair is the fastest measured
// for that element type).  Smaller inputs get smaller chunks so that there
// are at least ~4096 chunks (one wavefront each) when possible.
struct ScanShape {
  int32_t variant;
  int64_t chunk_bytes;
  int32_t stage;
  int32_t xclass;  // chunks classified from int64 x, no separate edge search
};

static ScanShape default_shape(int ydt) {
  switch (ydt) {
    case TS_U8: return {1, 16384, 0, 0};
    case TS_I8: return {1, 16384, 0, 0};
    case TS_I16: case TS_U16: return {0, 16384, 0, 0};
    case TS_F16: return {2, 16384, 0, 0};
    case TS_I32: case TS_U32: case TS_F32: return {2, 16384, 0, 0};
    default: return {2, 16384, 0, 0};
  }
}

static int64_t g_chunk_bytes_override = -1;
static int32_t g_small_override = -1;
static int32_t g_variant_override = -1;
static int32_t g_stage_override = -1;
static int32_t g_xclass_override = -1;
static int32_t g_direct_override = -1;

// One wavefront per bin instead of chunks (two launches instead of three, no
// per-chunk partials): series of at most kDirectMaxBytes in at least
// kDirectMinBins bins of at least kDirectMinBin elements (the call is
// launch-bound there), and series without x (equal bins, so every wavefront
// reads the same amount) in at least kDirectWideMinBins bins of
// kDirectWideMinBinBytes..kDirectWideMaxBinBytes.  From kBlockMinBins to
// kDirectWideMinBins bins of at least kBlockMinBinBytes, a wavefront each
// leaves the GPU half empty: a workgroup of four wavefronts per bin instead.
// Sweeps of MinMax over 1 GB series on MI355X (u8, i16, f16, f32, f64; bins
// of 3 KB to 4 MB): from 4 KB to 500 KB bins the per-bin wavefront is the
// fastest path for every type (10 KB u8 bins 3.8 -> 5.8 TB/s, 10 KB f32 bins
// 4.8 -> 6.1 TB/s, 500 KB bins 6.1 -> 6.3-6.6 TB/s); below ~4 KB the
// LDS-staged chunks win; with 500-1,999 bins the workgroup per bin (1,000
// bins: u8 3.9 TB/s with a wavefront per bin, 6.1 with chunks, 6.2 with a
// workgroup per bin; f32 4.4 / 6.1 / 6.4; 500 bins: f32 2.4 / 6.1 / 6.6,
// f64 3.9 / 6.0 / 6.6); with 250 bins (4 MB) the chunks win again except
// for f64 (6.2 with chunks, 6.6 with a workgroup per bin).
static const int64_t kDirectMaxBytes = 8 << 20, kDirectMinBins = 64, kDirectMinBin = 256;
static const int64_t kDirectWideMinBins = 2000, kDirectWideMinBinBytes = 4096, kDirectWideMaxBinBytes = 512 << 10;
static const int64_t kBlockMinBins = 500, kBlockMinBins8 = 250, kBlockMinBinBytes = 256 << 10;

// The per-bin grid has 64 threads per bin: at most 2^25 bins keeps it within
// 2^31 threads; the workgroup-per-bin grid has 256, so at most 2^23 bins.
static const int64_t kDirectMaxBinCount = (int64_t)1 << 25, kBlockMaxBinCount = (int64_t)1 << 23;

// Tile shape of the per-bin kernel (the scan's variant numbering: 0 = 4x2,
// 1 = 4x1, 2 = 8x1, 3 = 2x2) from the same sweeps: bytes 4x1 (their fold
// spreads every byte into a 16-bit lane: with two tiles in flight the
// registers allow three wavefronts per SIMD instead of eight), two-byte
// types 4x2, four- and eight-byte types 2x2 under 8 KB bins, else 4x2, and
// eight-byte types 8x1 from 32 KB bins.
static int32_t direct_variant(int ydt, int64_t bin_bytes) {
  const int64_t es = (int64_t)elem_size(ydt);
  if (es == 1) return 1;
  if (es == 2) return 0;
  if (bin_bytes < 8192) return 3;
  return es == 8 && bin_bytes >= 32768 ? 2 : 0;
}

// 0: chunks (partials, merge); 1: a wavefront per bin; 2: a workgroup of four
// wavefronts per bin (long bins, too few for a wavefront each).
static int direct_mode(int ydt, bool has_x, int64_t n, int64_t nb) {
  if (nb > kDirectMaxBinCount) return 0;
  if (g_direct_override >= 0) return g_direct_override == 2 && nb > kBlockMaxBinCount ? 1 : g_direct_override;
  if (g_chunk_bytes_override >= 0 || g_small_override >= 0 || g_variant_override >= 0 || g_stage_override >= 0)
    return 0;  // explicit chunk tuning: the chunked kernels run
  const int64_t es = (int64_t)elem_size(ydt);
  if (n * es <= kDirectMaxBytes && nb >= kDirectMinBins && n / nb >= kDirectMinBin) return 1;
  const int64_t bin_bytes = n / nb * es;
  if (has_x || bin_bytes < kDirectWideMinBinBytes) return 0;
  if (nb >= (es == 8 ? kBlockMinBins8 : kBlockMinBins) && nb < kDirectWideMinBins && bin_bytes >= kBlockMinBinBytes)
    return 2;
  return nb >= kDirectWideMinBins && bin_bytes <= kDirectWideMaxBinBytes ? 1 : 0;
}

// Tile shape of the workgroup-per-bin kernel: 8x1 for eight-byte types, else
// 4x1 (sweeps over 1 GB series, 500-1,500 bins).
static int32_t block_variant(int ydt) { return elem_size(ydt) == 8 ? 2 : 1; }

// Bins averaging fewer than kStageBin elements go through LDS-staged chunks
// of kStageChunk bytes (one HBM round trip per chunk instead of one per bin).
static const int64_t kStageBin = 4096, kStageChunk = 8192;
// Streamed chunks: chunk bytes, and the bin size (bytes) from which the
// per-bin segments of the default shape take over again.
static const int64_t kStreamChunk = 65536, kStreamMaxBin = 131072;

// Shapes of the scan that classifies chunks from int64 x (sweeps on MI355X
// over 1e8-point series): its per-chunk set-up costs more than the edge
// lookup, so narrow types take longer chunks.
static ScanShape xclass_shape(int ydt) {
  switch (elem_size(ydt)) {
    case 1: return {1, 32768, 0, 1};
    case 2: return {1, 65536, 0, 1};
    case 4: return {0, 16384, 0, 1};
    default: return {2, 16384, 0, 1};
  }
}

// Halves the chunk (down to 4 KB) until the series has min_chunks chunks.
static int64_t fit_chunk(int64_t chunk_bytes, int64_t total, int64_t min_chunks) {
  while (chunk_bytes > 4096 && total / chunk_bytes < min_chunks) chunk_bytes /= 2;
  return chunk_bytes;
}

// Bins averaging at least kXclassChunks chunks are classified from int64 x
// by the scan itself (the edge search would otherwise be a separate pass).
static const int64_t kXclassChunks = 2;

static ScanShape scan_shape(int ydt, int xdt, int64_t n, int64_t nb) {
  const int64_t total = n * (int64_t)elem_size(ydt);
  const int32_t stage = g_stage_override >= 0 ? g_stage_override : (nb > 0 && n / nb < kStageBin ? 1 : 0);
  if (xdt == TS_I64 && !stage && g_xclass_override != 0 && g_direct_override != 1) {
    ScanShape sh = xclass_shape(ydt);
    if (g_variant_override >= 0) sh.variant = g_variant_override;
    sh.chunk_bytes = g_chunk_bytes_override > 0 ? g_chunk_bytes_override : fit_chunk(sh.chunk_bytes, total, 2048);
    const int64_t ce = sh.chunk_bytes / (int64_t)elem_size(ydt);
    if (g_xclass_override == 1 || (nb > 0 && n / nb >= kXclassChunks * ce)) return sh;
  }
  ScanShape sh = default_shape(ydt);
  if (g_variant_override >= 0) sh.variant = g_variant_override;
  sh.stage = stage;
  // Bins of a few chunks or less (2- to 8-byte types): the streamed variant
  // with long chunks walks each chunk's tiles once whatever the bins
  // (sweeps over 1 GB series on MI355X: 10-25% faster than the per-bin
  // segments from 8 KB bins up to kStreamMaxBin, and for 2-byte types from
  // 4 KB bins, where the LDS-staged path took them; bytes stay on the
  // default shape).
  const int64_t es = (int64_t)elem_size(ydt), bin_bytes = nb > 0 ? n / nb * es : 0;
  if (g_variant_override < 0 && g_stage_override != 1 && es >= 2 && bin_bytes < kStreamMaxBin &&
      bin_bytes >= (es == 2 ? 4096 : 8192)) {
    sh.variant = kScanStreamVariant;
    sh.stage = 0;
    sh.chunk_bytes = g_chunk_bytes_override > 0 ? g_chunk_bytes_override : fit_chunk(kStreamChunk, total, 4096);
    return sh;
  }
  if (g_chunk_bytes_override > 0) {
    sh.chunk_bytes = g_chunk_bytes_override;
  } else if (sh.stage) {
    sh.chunk_bytes = kStageChunk;
  } else {
    sh.chunk_bytes = fit_chunk(sh.chunk_bytes, total, 4096);
  }
  if (sh.stage && sh.chunk_bytes > 32768) sh.chunk_bytes = 32768;  // LDS per workgroup
  return sh;
}

static hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

static int32_t small_threshold() { return g_small_override > 0 ? g_small_override : 128; }

// ------------------------------------------------------------------ plans

struct ScanPlan {
  int64_t nb = 0, chunk = 0, nchunks = 0;
  int32_t variant = 0, stage = 0, xclass = 0;
  bool nan = false;  // NaN-aware scan (floating-point y)
  size_t off_edges = 0, off_binres = 0, off_partL = 0, off_partR = 0, off_sel = 0, off_cnt = 0, off_bsum = 0,
         bytes = 0;
};

// Workspace of one argmin/argmax pass over n elements in nb bins.  The chunk
// count allows for the largest possible misalignment of y, so the size does
// not depend on the pointer.
static bool float_dtype(int dt) { return dt == TS_F16 || dt == TS_F32 || dt == TS_F64; }

// Chunk of the NaN-aware scan.
static const int64_t kNanChunk = 32768;

static ScanPlan scan_plan(int ydt, int xdt, int64_t n, int64_t nb, size_t base, bool nan = false) {
  ScanPlan p;
  const bool need_edges = xdt != TS_NONE;
  ScanShape sh = scan_shape(ydt, xdt, n, nb);
  p.nan = nan && float_dtype(ydt);
  if (p.nan) {  // one chunk-major kernel: edges searched first, no staging or streaming
    sh.variant = 0;
    sh.stage = 0;
    sh.xclass = 0;
    sh.chunk_bytes = g_chunk_bytes_override > 0 ? g_chunk_bytes_override
                                                : fit_chunk(kNanChunk, n * (int64_t)elem_size(ydt), 4096);
  }
  p.nb = nb;
  p.chunk = sh.chunk_bytes / (int64_t)elem_size(ydt);
  p.variant = sh.variant;
  p.stage = sh.stage;
  p.xclass = sh.xclass;
  p.nchunks = (n + vec_width(ydt) - 1 + p.chunk - 1) / p.chunk;
  if (p.nchunks < 1) p.nchunks = 1;
  size_t o = base;
  p.off_edges = o;
  if (need_edges) o = align256(o + sizeof(int64_t) * (size_t)(nb + 1));
  p.off_binres = o;
  o = align256(o + sizeof(int64_t) * 2 * (size_t)nb);
  p.off_partL = o;
  o = align256(o + sizeof(Partial) * (size_t)p.nchunks);
  p.off_partR = o;
  o = align256(o + sizeof(Partial) * (size_t)p.nchunks);
  p.off_sel = o;
  o = align256(o + sizeof(int64_t) * 4 * (size_t)nb);
  p.off_cnt = o;
  o = align256(o + sizeof(int64_t) * (size_t)nb);
  p.off_bsum = o;
  if (nb > kCompactSingleMax) o = align256(o + sizeof(int64_t) * (size_t)compact_blocks(nb));
  p.bytes = o;
  return p;
}

// LTTB walk variants: buckets of a few points (transition map over all
// anchors), long buckets of a plain series (hull candidates), else one
// workgroup walking every point.
enum LttbMode { kLttbSeq = 0, kLttbSmall = 1, kLttbHull = 2 };

static LttbMode lttb_mode(bool has_sel, int64_t m_max, int64_t n_out) {
  const int64_t nb = n_out - 2;
  const int64_t maxb = (m_max - 2 + nb - 1) / nb, minb = (m_max - 2) / nb;
  if (maxb <= 32 && m_max <= (int64_t)1 << 30) return kLttbSmall;
  if (!has_sel && minb >= kHullMinBucket && maxb < ((int64_t)1 << 30)) return kLttbHull;
  return kLttbSeq;
}

struct LttbPlan {
  LttbMode mode = kLttbSeq;
  size_t off_cx = 0, off_cy = 0, off_next = 0, off_entry = 0, off_ccnt = 0, off_cidx = 0, off_ccx = 0,
         off_ccy = 0, off_hnext = 0, off_hjump = 0, off_hflag = 0, off_gx = 0, off_gy = 0, bytes = 0;
};

static LttbPlan lttb_plan(int64_t m_max, int64_t n_out, bool has_sel, size_t base) {
  LttbPlan p;
  p.mode = lttb_mode(has_sel, m_max, n_out);
  size_t o = base;
  const size_t nb = (size_t)(n_out - 2);
  p.off_cx = o;
  o = align256(o + sizeof(double) * nb);
  p.off_cy = o;
  o = align256(o + sizeof(double) * nb);
  if (p.mode == kLttbSmall) {
    p.off_next = o;
    o = align256(o + sizeof(int32_t) * 2 * (size_t)m_max);
    p.off_entry = o;
    o = align256(o + sizeof(int32_t) * (lttb_group_count(n_out) + 1));
  } else if (p.mode == kLttbHull) {
    p.off_ccnt = o;
    o = align256(o + sizeof(int32_t) * nb);
    p.off_cidx = o;
    o = align256(o + sizeof(int64_t) * nb * kHullCand);
    p.off_ccx = o;
    o = align256(o + sizeof(double) * nb * kHullCand);
    p.off_ccy = o;
    o = align256(o + sizeof(double) * nb * kHullCand);
    p.off_hnext = o;
    o = align256(o + nb * kHullCand);
    p.off_hjump = o;
    o = align256(o + (size_t)lttb_hull_group((int64_t)nb) * kHullCand);
    p.off_hflag = o;
    o = align256(o + sizeof(int32_t));
  }
  if (has_sel) {  // the candidates' coordinates, gathered once
    p.off_gx = o;
    o = align256(o + sizeof(uint64_t) * (size_t)m_max);
    p.off_gy = o;
    o = align256(o + sizeof(uint64_t) * (size_t)m_max);
  }
  p.bytes = o;
  return p;
}

// ------------------------------------------------------------------ checks

static int check_series(const ts_series *s) {
  if (!s) return fail(TS_ERR_NULL, "series descriptor is NULL");
  if (s->n < 0) return fail(TS_ERR_ARG, "n = %lld < 0", (long long)s->n);
  if (elem_size(s->y_dtype) == 0) return fail(TS_ERR_DTYPE, "y dtype %d is not a ts dtype", s->y_dtype);
  if (s->n > 0 && !s->y) return fail(TS_ERR_NULL, "y is NULL");
  if ((s->x == nullptr) != (s->x_dtype == TS_NONE))
    return fail(TS_ERR_NULL, "x is %s but x_dtype is %d", s->x ? "set" : "NULL", s->x_dtype);
  if (s->x && !x_dtype_ok(s->x_dtype))
    return fail(TS_ERR_DTYPE, "x dtype %d unsupported (int32/int64/uint32/uint64/float32/float64)", s->x_dtype);
  if (s->y && ((uintptr_t)s->y % elem_size(s->y_dtype)))
    return fail(TS_ERR_ALIGN, "y is not aligned to its element size");
  if (s->x && ((uintptr_t)s->x % elem_size(s->x_dtype)))
    return fail(TS_ERR_ALIGN, "x is not aligned to its element size");
  if (s->n > ((int64_t)1 << 48)) return fail(TS_ERR_ARG, "n = %lld exceeds 2^48", (long long)s->n);
  return TS_OK;
}

// nb bins over n points: the closed-form edges multiply b by n-1.
static int check_bins(int64_t n, int64_t nb) {
  if (nb < 1) return fail(TS_ERR_ARG, "need at least one bin");
  if (nb >= ((int64_t)1 << 31)) return fail(TS_ERR_ARG, "too many bins (%lld)", (long long)nb);
  if (n > 0 && (unsigned __int128)(n - 1) * (unsigned __int128)nb >= ((unsigned __int128)1 << 62))
    return fail(TS_ERR_ARG, "n * bins too large");
  return TS_OK;
}

static int check_out(const int64_t *out_idx, const int64_t *out_count) {
  if (!out_idx || !out_count) return fail(TS_ERR_NULL, "out_idx / out_count is NULL");
  return TS_OK;
}

static int check_ws(void *ws, size_t ws_bytes, size_t need) {
  if (need == 0) return TS_OK;
  if (!ws) return fail(TS_ERR_WORKSPACE, "workspace is NULL (%zu bytes needed)", need);
  if ((uintptr_t)ws % 256) return fail(TS_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (ws_bytes < need) return fail(TS_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, need);
  return TS_OK;
}

static int check_nout(int algo, int64_t n_out, int64_t ratio) {
  switch (algo) {
    case TS_NAN_MINMAX:
    case TS_MINMAX:
      if (n_out < 2 || n_out % 2) return fail(TS_ERR_ARG, "MinMax n_out must be even and >= 2 (got %lld)", (long long)n_out);
      return check_bins(2, n_out / 2);
    case TS_NAN_M4:
    case TS_M4:
      if (n_out < 4 || n_out % 4) return fail(TS_ERR_ARG, "M4 n_out must be a multiple of 4 (got %lld)", (long long)n_out);
      return check_bins(2, n_out / 4);
    case TS_LTTB:
      if (n_out < 3) return fail(TS_ERR_ARG, "LTTB n_out must be >= 3 (got %lld)", (long long)n_out);
      if (n_out >= ((int64_t)1 << 31)) return fail(TS_ERR_ARG, "n_out too large");
      return TS_OK;
    case TS_MINMAXLTTB:
      if (n_out < 3) return fail(TS_ERR_ARG, "MinMaxLTTB n_out must be >= 3 (got %lld)", (long long)n_out);
      if (ratio < 1) return fail(TS_ERR_ARG, "minmax_ratio must be >= 1 (got %lld)", (long long)ratio);
      if (n_out >= ((int64_t)1 << 28) || ratio >= ((int64_t)1 << 16) || (n_out * ratio) % 2)
        return fail(TS_ERR_ARG, "n_out * minmax_ratio must be even and < 2^44");
      return check_bins(2, n_out * ratio / 2);
  }
  return fail(TS_ERR_ARG, "unknown algorithm %d", algo);
}

// ------------------------------------------------------------------ pieces

static char *wsp(void *ws, size_t off) { return (char *)ws + off; }

static int64_t y_shift(const ts_series &s) {
  const size_t esz = elem_size(s.y_dtype);
  return (int64_t)(((uintptr_t)s.y & 15) / esz);
}

// Argmin/argmax pass + per-bin selection + compaction for MinMax / M4 / the
// preselection.  `out` receives the indices (+ index_offset).
static int run_scan(const ts_series &s, int64_t nb, int m4, const ScanPlan &pl, void *ws, int64_t *out,
                    int64_t *out_count, int64_t index_offset, int64_t endpoints_n, hipStream_t st) {
  const int64_t *edges = nullptr;
  int64_t *ed = nullptr;
  hipError_t e;
  if (s.x) {
    ed = (int64_t *)wsp(ws, pl.off_edges);
    if (!pl.xclass && (e = launch_edges_x(s.x, s.x_dtype, s.n, nb, ed, st)) != hipSuccess)
      return hip_fail(e, "edges");
    edges = ed;
  }
  ScanParams sp;
  sp.y = s.y;
  sp.n = s.n;
  sp.shift = y_shift(s);
  sp.chunk = pl.chunk;
  sp.nchunks = (s.n + sp.shift + pl.chunk - 1) / pl.chunk;
  sp.edges = edges;
  sp.nb = nb;
  sp.binres = (int64_t *)wsp(ws, pl.off_binres);
  sp.partL = (Partial *)wsp(ws, pl.off_partL);
  sp.partR = (Partial *)wsp(ws, pl.off_partR);
  sp.small = small_threshold();
  sp.variant = pl.variant;
  sp.stage = pl.stage;
  sp.xclass = pl.xclass;
  sp.x = pl.xclass ? s.x : nullptr;
  sp.xedges = pl.xclass ? ed : nullptr;
  if (pl.xclass) sp.edges = nullptr;
  // one wavefront per bin, no merge (not while the scan kernel is being timed)
  const int dmode = !pl.nan && !pl.xclass && !g_ev_start ? direct_mode(s.y_dtype, s.x != nullptr, s.n, nb) : 0;
  const bool direct = dmode > 0;
  if (pl.nan) {
    if ((e = launch_scan_nan(s.y_dtype, sp, st)) != hipSuccess) return hip_fail(e, "nan scan");
  } else if (!direct && (e = launch_scan(s.y_dtype, sp, st, g_ev_start, g_ev_stop)) != hipSuccess) {
    return hip_fail(e, "scan");
  }
  MergeParams mp;
  mp.n = s.n;
  mp.shift = sp.shift;
  mp.chunk = sp.chunk;
  mp.edges = edges;
  mp.nb = nb;
  mp.binres = sp.binres;
  mp.partL = sp.partL;
  mp.partR = sp.partR;
  mp.m4 = m4;
  mp.sel = (int64_t *)wsp(ws, pl.off_sel);
  mp.cnt = (int64_t *)wsp(ws, pl.off_cnt);
  CompactParams cp;
  cp.nb = nb;
  cp.sel = mp.sel;
  cp.cnt = mp.cnt;
  cp.out = out;
  cp.out_count = out_count;
  cp.index_offset = index_offset;
  cp.endpoints_n = endpoints_n;
  cp.all_n = -1;
  cp.bsum = nb > kCompactSingleMax ? (int64_t *)wsp(ws, pl.off_bsum) : nullptr;
  if (direct) {
    ScanParams dp = sp;
    dp.variant = g_variant_override >= 0 && g_variant_override < kScanStreamVariant ? g_variant_override
                 : dmode == 2 ? block_variant(s.y_dtype)
                              : direct_variant(s.y_dtype, s.n / nb * (int64_t)elem_size(s.y_dtype));
    e = dmode == 2 ? launch_bins_block(s.y_dtype, dp, mp, st) : launch_bins_direct(s.y_dtype, dp, mp, st);
    if (e != hipSuccess) return hip_fail(e, "bins");
  } else if ((e = launch_merge(mp, st)) != hipSuccess) {
    return hip_fail(e, "merge");
  }
  if ((e = launch_compact(cp, st)) != hipSuccess) return hip_fail(e, "compact");
  return TS_OK;
}

static int write_all(int64_t n, int64_t *out, int64_t *out_count, hipStream_t st) {
  CompactParams cp{};
  cp.out = out;
  cp.out_count = out_count;
  cp.all_n = n;
  hipError_t e = launch_compact(cp, st);
  if (e != hipSuccess) return hip_fail(e, "arange");
  return TS_OK;
}

// MinMaxLTTB preselection sizes: interior of n-2 points, n_out*ratio outputs.
struct MmlPlan {
  bool presel_all = false;  // the interior is not reduced: candidates = all points
  ScanPlan scan;
  size_t off_cand = 0, off_m = 0;
  LttbPlan lt;
  int64_t m_max = 0;
  size_t bytes = 0;
};

static MmlPlan mml_plan(const ts_series &s, int64_t n_out, int64_t ratio) {
  MmlPlan p;
  const int64_t npre = n_out * ratio, ni = s.n - 2;
  p.presel_all = ni <= npre;
  size_t o = 0;
  if (!p.presel_all) {
    p.scan = scan_plan(s.y_dtype, s.x_dtype, ni, npre / 2, 0);
    o = p.scan.bytes;
    p.off_cand = o;
    o = align256(o + sizeof(int64_t) * (size_t)(npre + 2));
    p.off_m = o;
    o = align256(o + sizeof(int64_t));
    p.m_max = npre + 2;
  } else {
    p.m_max = s.n;
  }
  p.lt = lttb_plan(p.m_max, n_out, !p.presel_all, o);
  p.bytes = p.lt.bytes;
  return p;
}

// A side stream (default priority) and fork/join events per host thread and
// device, created on first use: the LTTB centres of a plain series run there
// beside the hull kernel (the hulls use the VALU and most of the LDS, the
// centres stream the series from HBM; neither reads the other's output).
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  bool tried = false;
};
static thread_local SideStream g_side[64];

static SideStream *side_stream(hipStream_t st) {
  int dev = -1;
  if ((st ? hipStreamGetDevice(st, &dev) : hipGetDevice(&dev)) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  SideStream &ss = g_side[dev];
  if (!ss.tried) {
    // not created while the caller's stream is being captured (stream
    // creation is not a capturable operation); later calls create it
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (st && (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)) return nullptr;
    ss.tried = true;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
    const bool ok = hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking) == hipSuccess &&
                    hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming) == hipSuccess &&
                    hipEventCreateWithFlags(&ss.join, hipEventDisableTiming) == hipSuccess;
    if (cur != dev) (void)hipSetDevice(cur);
    if (!ok) ss.s = nullptr;
  }
  return ss.s ? &ss : nullptr;
}

// Average candidates per bucket up to which the small-bucket map computes its
// own centres (each anchor then re-reads at most a few points).
static const int64_t kOwnCentresPerBucket = 8;

static int run_lttb(const ts_series &s, const int64_t *sel, int64_t m, const int64_t *m_dev, int64_t m_max,
                    int64_t n_out, const LttbPlan &lp, void *ws, int64_t *out, int64_t *out_count, hipStream_t st) {
  LttbParams p{};
  p.x = s.x;
  p.x_dtype = s.x_dtype;
  p.y = s.y;
  p.y_dtype = s.y_dtype;
  p.sel = sel;
  p.m = m;
  p.m_dev = m_dev;
  p.m_max = m_max;
  p.n_out = n_out;
  p.cx = (double *)wsp(ws, lp.off_cx);
  p.cy = (double *)wsp(ws, lp.off_cy);
  if (lp.mode == kLttbSmall) {
    p.next = (int32_t *)wsp(ws, lp.off_next);
    p.entry = (int32_t *)wsp(ws, lp.off_entry);
  }
  if (lp.mode == kLttbHull) {
    p.cand_cnt = (int32_t *)wsp(ws, lp.off_ccnt);
    p.cand_idx = (int64_t *)wsp(ws, lp.off_cidx);
    p.cand_x = (double *)wsp(ws, lp.off_ccx);
    p.cand_y = (double *)wsp(ws, lp.off_ccy);
    p.hnext = (uint8_t *)wsp(ws, lp.off_hnext);
    p.hjump = (uint8_t *)wsp(ws, lp.off_hjump);
    p.hflag = (int32_t *)wsp(ws, lp.off_hflag);
  }
  p.out = out;
  p.out_count = out_count;
  hipError_t e;
  // Buckets of a few points (MinMaxLTTB's candidates): the map computes the
  // centres it needs from the candidates directly, so neither the gather nor
  // the centre pass runs first (two launches instead of four).
  const bool own = lp.mode == kLttbSmall && m_max <= kOwnCentresPerBucket * (n_out - 2) + 2;
  if (sel && !own) {
    p.gx = (uint64_t *)wsp(ws, lp.off_gx);
    p.gy = (uint64_t *)wsp(ws, lp.off_gy);
    if ((e = launch_lttb_gather(p, st)) != hipSuccess) return hip_fail(e, "lttb candidate gather");
  }
  SideStream *ss = lp.mode == kLttbHull ? side_stream(st) : nullptr;
  if (ss) {  // centres on the side stream, beside the hulls
    if ((e = hipEventRecord(ss->fork, st)) != hipSuccess || (e = hipStreamWaitEvent(ss->s, ss->fork, 0)) != hipSuccess)
      return hip_fail(e, "lttb fork");
    if ((e = launch_lttb_centres(p, ss->s)) != hipSuccess) return hip_fail(e, "lttb centres");
    if ((e = hipEventRecord(ss->join, ss->s)) != hipSuccess) return hip_fail(e, "lttb join");
  } else if (!own && (e = launch_lttb_centres(p, st)) != hipSuccess) {
    return hip_fail(e, "lttb centres");
  }
  switch (lp.mode) {
    case kLttbSmall: e = launch_lttb_small(p, own, st); break;
    case kLttbHull:
      if ((e = launch_lttb_hull(p, st)) != hipSuccess) return hip_fail(e, "lttb hulls");
      if (ss && (e = hipStreamWaitEvent(st, ss->join, 0)) != hipSuccess) return hip_fail(e, "lttb join");
      e = launch_lttb_hull_walk(p, st);
      break;
    default: e = launch_lttb_seq(p, st); break;
  }
  if (e != hipSuccess) return hip_fail(e, "lttb walk");
  return TS_OK;
}

int api_fail(int code, const char *msg) { return fail(code, "%s", msg); }
int api_check_series(const ts_series *s) { return check_series(s); }
int api_check_nout(int algo, int64_t n_out, int64_t ratio) { return check_nout(algo, n_out, ratio); }

}  // namespace tsds

using namespace tsds;

extern "C" {

int ts_version(void) { return 10000; }

const char *ts_last_error(void) { return g_err.c_str(); }

size_t ts_workspace_bytes(int algo, const ts_series *s, int64_t n_out, int64_t minmax_ratio) {
  if (check_series(s) || check_nout(algo, n_out, minmax_ratio)) return 0;
  if (s->n <= n_out) return 0;
  switch (algo) {
    case TS_MINMAX: return scan_plan(s->y_dtype, s->x_dtype, s->n, n_out / 2, 0).bytes;
    case TS_M4: return scan_plan(s->y_dtype, s->x_dtype, s->n, n_out / 4, 0).bytes;
    case TS_NAN_MINMAX: return scan_plan(s->y_dtype, s->x_dtype, s->n, n_out / 2, 0, true).bytes;
    case TS_NAN_M4: return scan_plan(s->y_dtype, s->x_dtype, s->n, n_out / 4, 0, true).bytes;
    case TS_LTTB: return lttb_plan(s->n, n_out, false, 0).bytes;
    case TS_MINMAXLTTB: return mml_plan(*s, n_out, minmax_ratio).bytes;
  }
  return 0;
}

static int minmax_m4(int algo, const ts_series *s, int64_t n_out, int64_t *out_idx, int64_t *out_count,
                     void *ws, size_t ws_bytes, void *stream) {
  int rc;
  if ((rc = check_series(s)) || (rc = check_nout(algo, n_out, 0)) || (rc = check_out(out_idx, out_count)))
    return rc;
  hipStream_t st = (hipStream_t)stream;
  if (s->n <= n_out) return write_all(s->n, out_idx, out_count, st);
  const bool m4 = algo == TS_M4 || algo == TS_NAN_M4;
  const int64_t nb = m4 ? n_out / 4 : n_out / 2;
  if ((rc = check_bins(s->n, nb))) return rc;
  const ScanPlan pl = scan_plan(s->y_dtype, s->x_dtype, s->n, nb, 0, algo == TS_NAN_MINMAX || algo == TS_NAN_M4);
  if ((rc = check_ws(ws, ws_bytes, pl.bytes))) return rc;
  return run_scan(*s, nb, m4, pl, ws, out_idx, out_count, 0, 0, st);
}

int ts_minmax(const ts_series *s, int64_t n_out, int64_t *out_idx, int64_t *out_count, void *ws,
              size_t ws_bytes, void *stream) {
  return minmax_m4(TS_MINMAX, s, n_out, out_idx, out_count, ws, ws_bytes, stream);
}

int ts_m4(const ts_series *s, int64_t n_out, int64_t *out_idx, int64_t *out_count, void *ws, size_t ws_bytes,
          void *stream) {
  return minmax_m4(TS_M4, s, n_out, out_idx, out_count, ws, ws_bytes, stream);
}

int ts_nan_minmax(const ts_series *s, int64_t n_out, int64_t *out_idx, int64_t *out_count, void *ws,
                  size_t ws_bytes, void *stream) {
  return minmax_m4(TS_NAN_MINMAX, s, n_out, out_idx, out_count, ws, ws_bytes, stream);
}

int ts_nan_m4(const ts_series *s, int64_t n_out, int64_t *out_idx, int64_t *out_count, void *ws, size_t ws_bytes,
              void *stream) {
  return minmax_m4(TS_NAN_M4, s, n_out, out_idx, out_count, ws, ws_bytes, stream);
}

int ts_lttb(const ts_series *s, int64_t n_out, int64_t *out_idx, int64_t *out_count, void *ws, size_t ws_bytes,
            void *stream) {
  int rc;
  if ((rc = check_series(s)) || (rc = check_nout(TS_LTTB, n_out, 0)) || (rc = check_out(out_idx, out_count)))
    return rc;
  hipStream_t st = (hipStream_t)stream;
  if (s->n <= n_out) return write_all(s->n, out_idx, out_count, st);
  if ((unsigned __int128)s->n * (unsigned __int128)n_out >= ((unsigned __int128)1 << 62))
    return fail(TS_ERR_ARG, "n * n_out too large");
  const LttbPlan lp = lttb_plan(s->n, n_out, false, 0);
  if ((rc = check_ws(ws, ws_bytes, lp.bytes))) return rc;
  return run_lttb(*s, nullptr, s->n, nullptr, s->n, n_out, lp, ws, out_idx, out_count, st);
}

int ts_minmaxlttb(const ts_series *s, int64_t n_out, int64_t minmax_ratio, int64_t *out_idx, int64_t *out_count,
                  void *ws, size_t ws_bytes, void *stream) {
  int rc;
  if ((rc = check_series(s)) || (rc = check_nout(TS_MINMAXLTTB, n_out, minmax_ratio)) ||
      (rc = check_out(out_idx, out_count)))
    return rc;
  hipStream_t st = (hipStream_t)stream;
  if (s->n <= n_out) return write_all(s->n, out_idx, out_count, st);
  const MmlPlan pl = mml_plan(*s, n_out, minmax_ratio);
  if ((rc = check_ws(ws, ws_bytes, pl.bytes))) return rc;
  if ((unsigned __int128)pl.m_max * (unsigned __int128)n_out >= ((unsigned __int128)1 << 62))
    return fail(TS_ERR_ARG, "n * n_out too large");
  if (pl.presel_all) {
    return run_lttb(*s, nullptr, s->n, nullptr, s->n, n_out, pl.lt, ws, out_idx, out_count, st);
  }
  // Preselection over the interior points 1..n-2.
  ts_series in = *s;
  in.n = s->n - 2;
  in.y = (const char *)s->y + elem_size(s->y_dtype);
  if (s->x) in.x = (const char *)s->x + elem_size(s->x_dtype);
  const int64_t npre = n_out * minmax_ratio;
  if ((rc = check_bins(in.n, npre / 2))) return rc;
  int64_t *cand = (int64_t *)wsp(ws, pl.off_cand);
  int64_t *m_dev = (int64_t *)wsp(ws, pl.off_m);
  if ((rc = run_scan(in, npre / 2, 0, pl.scan, ws, cand + 1, m_dev, 1, s->n, st))) return rc;
  return run_lttb(*s, cand, -1, m_dev, pl.m_max, n_out, pl.lt, ws, out_idx, out_count, st);
}

int ts_bin_edges(const ts_series *s, int64_t nb, int64_t *edges, void *stream) {
  int rc;
  if ((rc = check_series(s)) || (rc = check_bins(s->n, nb))) return rc;
  if (!edges) return fail(TS_ERR_NULL, "edges is NULL");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (s->x && s->n > 0) e = launch_edges_x(s->x, s->x_dtype, s->n, nb, edges, st);
  else e = launch_edges_nox(s->n, nb, edges, st);
  if (e != hipSuccess) return hip_fail(e, "edges");
  return TS_OK;
}

size_t ts_argminmax_workspace_bytes(const ts_series *s, int64_t nb) {
  if (check_series(s) || nb < 1) return 0;
  return scan_plan(s->y_dtype, TS_NONE, s->n, nb, 0).bytes;
}

int ts_bin_argminmax(const ts_series *s, const int64_t *edges, int64_t nb, int64_t *imin, int64_t *imax, void *ws,
                     size_t ws_bytes, void *stream) {
  int rc;
  if ((rc = check_series(s)) || (rc = check_bins(s->n, nb))) return rc;
  if (!edges || !imin || !imax) return fail(TS_ERR_NULL, "edges / imin / imax is NULL");
  if (s->n == 0) return fail(TS_ERR_ARG, "empty series");
  const ScanPlan pl = scan_plan(s->y_dtype, TS_NONE, s->n, nb, 0);
  if ((rc = check_ws(ws, ws_bytes, pl.bytes))) return rc;
  hipStream_t st = (hipStream_t)stream;
  ScanParams sp;
  sp.y = s->y;
  sp.n = s->n;
  sp.shift = y_shift(*s);
  sp.chunk = pl.chunk;
  sp.nchunks = (s->n + sp.shift + pl.chunk - 1) / pl.chunk;
  sp.edges = edges;
  sp.nb = nb;
  sp.binres = (int64_t *)wsp(ws, pl.off_binres);
  sp.partL = (Partial *)wsp(ws, pl.off_partL);
  sp.partR = (Partial *)wsp(ws, pl.off_partR);
  sp.small = small_threshold();
  sp.variant = pl.variant;
  sp.stage = pl.stage;
  sp.x = nullptr;
  sp.xedges = nullptr;
  sp.xclass = 0;
  hipError_t e;
  if ((e = launch_scan(s->y_dtype, sp, st, g_ev_start, g_ev_stop)) != hipSuccess) return hip_fail(e, "scan");
  MergeParams mp{};
  mp.n = s->n;
  mp.shift = sp.shift;
  mp.chunk = sp.chunk;
  mp.edges = edges;
  mp.nb = nb;
  mp.binres = sp.binres;
  mp.partL = sp.partL;
  mp.partR = sp.partR;
  if ((e = launch_binres_to_outputs(mp, imin, imax, st)) != hipSuccess) return hip_fail(e, "bin outputs");
  return TS_OK;
}

int ts_lttb_centres(const ts_series *s, const int64_t *sel, int64_t m, int64_t n_out, double *cx, double *cy,
                    void *stream) {
  int rc;
  if ((rc = check_series(s))) return rc;
  if (n_out < 3 || m <= n_out) return fail(TS_ERR_ARG, "need m > n_out >= 3");
  if (!sel && m != s->n) return fail(TS_ERR_ARG, "without sel, m must equal n");
  if (!cx || !cy) return fail(TS_ERR_NULL, "cx / cy is NULL");
  LttbParams p{};
  p.x = s->x;
  p.x_dtype = s->x_dtype;
  p.y = s->y;
  p.y_dtype = s->y_dtype;
  p.sel = sel;
  p.m = m;
  p.m_max = m;
  p.n_out = n_out;
  p.cx = cx;
  p.cy = cy;
  hipError_t e = launch_lttb_centres(p, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "lttb centres");
  return TS_OK;
}

int ts_window(const ts_series *s, int64_t xa, int64_t xb, int64_t *range, void *stream) {
  int rc;
  if ((rc = check_series(s))) return rc;
  if (!s->x) return fail(TS_ERR_NULL, "window needs x");
  if (s->x_dtype == TS_F32 || s->x_dtype == TS_F64) return fail(TS_ERR_DTYPE, "window needs integer x");
  if (!range) return fail(TS_ERR_NULL, "range is NULL");
  hipError_t e = launch_window(s->x, s->x_dtype, s->n, xa, xb, range, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "window");
  return TS_OK;
}

int ts_everynth(const ts_series *s, int64_t n_out, int64_t *out_idx, int64_t *out_count, void *stream) {
  int rc;
  if ((rc = check_series(s))) return rc;
  if (n_out < 1) return fail(TS_ERR_ARG, "EveryNth needs n_out >= 1 (got %lld)", (long long)n_out);
  if (!out_idx || !out_count) return fail(TS_ERR_NULL, "out_idx / out_count is NULL");
  const int64_t n = s->n;
  const int64_t k = n <= n_out ? 1 : n / n_out + (n % n_out != 0);
  const int64_t m = n <= n_out ? n : (n + k - 1) / k;
  hipError_t e = launch_everynth(k, m, out_idx, out_count, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "everynth");
  return TS_OK;
}

int ts_gather(const ts_series *s, const int64_t *idx, const int64_t *count, int64_t cap, void *x_out,
              void *y_out, void *stream) {
  int rc;
  if ((rc = check_series(s))) return rc;
  if (cap < 0) return fail(TS_ERR_ARG, "cap = %lld < 0", (long long)cap);
  if (cap == 0) return TS_OK;
  if (!idx || !count || !y_out) return fail(TS_ERR_NULL, "idx / count / y_out is NULL");
  if (x_out && !s->x) return fail(TS_ERR_NULL, "x_out given for a series without x");
  const int ys = (int)elem_size(s->y_dtype), xs = s->x ? (int)elem_size(s->x_dtype) : 0;
  if ((uintptr_t)y_out % ys) return fail(TS_ERR_ALIGN, "y_out is not aligned to y's element size");
  if (x_out && ((uintptr_t)x_out % xs)) return fail(TS_ERR_ALIGN, "x_out is not aligned to x's element size");
  if (((uintptr_t)idx | (uintptr_t)count) % 8) return fail(TS_ERR_ALIGN, "idx / count is not 8-byte aligned");
  hipError_t e = launch_gather(s->x, xs, s->y, ys, s->n, idx, count, cap, x_out, y_out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gather");
  return TS_OK;
}

// Tuning knobs (tests use them to show that results do not depend on them).
int ts_set_tuning(int64_t chunk_bytes, int32_t small_bin, int32_t scan_variant, int32_t stage, int32_t xclass,
                  int32_t direct) {
  if (chunk_bytes > 0 && (chunk_bytes < 4096 || (chunk_bytes & (chunk_bytes - 1))))
    return fail(TS_ERR_ARG, "chunk_bytes must be a power of two >= 4096");
  if (scan_variant > kScanStreamVariant) return fail(TS_ERR_ARG, "scan_variant must be -1..4");
  if (stage > 1) return fail(TS_ERR_ARG, "stage must be -1, 0 or 1");
  if (xclass > 1) return fail(TS_ERR_ARG, "xclass must be -1, 0 or 1");
  if (direct > 2) return fail(TS_ERR_ARG, "direct must be -1, 0, 1 or 2");
  g_direct_override = direct < 0 ? -1 : direct;
  g_chunk_bytes_override = chunk_bytes;
  g_small_override = small_bin;
  g_variant_override = scan_variant;
  g_stage_override = stage;
  g_xclass_override = xclass;
  return TS_OK;
}

int ts_scan_config(int y_dtype, int x_dtype, int64_t n, int64_t nb, int32_t *variant, int64_t *chunk_bytes,
                   int32_t *kind) {
  if (elem_size(y_dtype) == 0) return fail(TS_ERR_DTYPE, "y dtype %d is not a ts dtype", y_dtype);
  if (x_dtype != TS_NONE && elem_size(x_dtype) == 0) return fail(TS_ERR_DTYPE, "x dtype %d is not a ts dtype", x_dtype);
  if (!variant || !chunk_bytes || !kind) return fail(TS_ERR_NULL, "variant / chunk_bytes / kind is NULL");
  if (nb < 1) return fail(TS_ERR_ARG, "need at least one bin");
  const ScanShape sh = scan_shape(y_dtype, x_dtype, n, nb);
  *variant = sh.variant;
  *chunk_bytes = sh.chunk_bytes;
  *kind = sh.stage ? 1 : sh.xclass ? 2 : sh.variant == kScanStreamVariant ? 3 : 0;
  const int dmode = sh.xclass ? 0 : direct_mode(y_dtype, x_dtype != TS_NONE, n, nb);
  if (dmode) {
    *kind = dmode == 2 ? 5 : 4;
    *variant = g_variant_override >= 0 && g_variant_override < kScanStreamVariant ? g_variant_override
               : dmode == 2 ? block_variant(y_dtype)
                            : direct_variant(y_dtype, n / nb * (int64_t)elem_size(y_dtype));
  }
  return TS_OK;
}

int ts_profile_scan_events(void *start, void *stop) {
  if ((start == nullptr) != (stop == nullptr)) return fail(TS_ERR_NULL, "give both events or neither");
  g_ev_start = (hipEvent_t)start;
  g_ev_stop = (hipEvent_t)stop;
  return TS_OK;
}

}  // extern "C"

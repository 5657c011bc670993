// internal.hpp -- host-side interface between the C-ABI layer (api.cpp) and
// the kernel translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tsds.h"

namespace tsds {

struct Partial;

// Binning of one series for the argmin/argmax scan.  Without x the bins are
// equal index ranges given in closed form; with x (or caller-given edges) the
// starts live in `edges` (device, nb + 1 entries).
struct ScanParams {
  const void *y;          // first element of the series
  int64_t n;              // series length
  int64_t shift;          // elements between the 16-byte aligned base and y
  int64_t chunk;          // elements per chunk (multiple of the vector width)
  int64_t nchunks;
  const int64_t *edges;   // NULL: closed-form equal index bins
  int64_t nb;
  int64_t *binres;        // [2*nb] argmin, argmax of bins inside one chunk
  Partial *partL;         // [nchunks] bin that started before the chunk
  Partial *partR;         // [nchunks] bin that continues after the chunk
  int32_t small;          // segments shorter than this: one lane per bin
  int32_t variant;        // tile shape (see launch_scan); kScanStreamVariant: tiles streamed over the chunk's bins
  int32_t stage;          // 1: chunks go through LDS (many small bins per chunk)
  const void *x;          // int64 x when the chunks are classified from x (xclass), else NULL
  int64_t *xedges;        // edge array the x-classified scan writes (nb + 1 entries)
  int32_t xclass;
};

// Scan variant that walks each chunk's tiles once, in order, folding every
// tile into the bin segments it overlaps (bins of a few kilobytes).
constexpr int32_t kScanStreamVariant = 4;

struct MergeParams {
  int64_t n;
  int64_t shift;
  int64_t chunk;
  const int64_t *edges;   // NULL: closed form
  int64_t nb;
  const int64_t *binres;
  const Partial *partL;
  const Partial *partR;
  int32_t m4;             // 0: MinMax {argmin, argmax}; 1: M4 adds first/last
  int64_t *sel;           // [4*nb] selected indices per bin (sorted, distinct)
  int64_t *cnt;           // [nb]   how many
};

// The merge takes a bin per thread while bins average at most this many
// chunks, a wavefront per bin above.
constexpr int64_t kLaneMergeChunks = 4;

struct CompactParams {
  int64_t nb;
  const int64_t *sel;
  const int64_t *cnt;
  int64_t *out;           // output indices
  int64_t *out_count;     // device scalar
  int64_t index_offset;   // added to every index (interior preselection)
  int64_t endpoints_n;    // > 0: also write out[-1] = 0 and out[count] = endpoints_n - 1
  int64_t all_n;          // >= 0: ignore bins, write out[i] = i for i < all_n
  int64_t *bsum;          // [compact_blocks(nb)] scratch of the multi-workgroup compaction (NULL: one workgroup)
};

// Bins per workgroup of the multi-workgroup compaction, and the bin count
// from which it is used (below it one workgroup scans every bin).
constexpr int64_t kCompactBins = 1024;
constexpr int64_t kCompactSingleMax = 4096;
inline int64_t compact_blocks(int64_t nb) { return (nb + kCompactBins - 1) / kCompactBins; }

size_t elem_size(int dtype);
int vec_width(int dtype);

hipError_t launch_edges_x(const void *x, int x_dtype, int64_t n, int64_t nb, int64_t *edges,
                          hipStream_t st);
hipError_t launch_edges_nox(int64_t n, int64_t nb, int64_t *edges, hipStream_t st);
// e0/e1 (optional): events stamped with the scan dispatch's start and end.
hipError_t launch_scan(int y_dtype, const ScanParams &p, hipStream_t st, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
hipError_t launch_merge(const MergeParams &p, hipStream_t st);
// Small series: one wavefront per bin, selection written directly (replaces
// the scan and the merge).
hipError_t launch_bins_direct(int y_dtype, const ScanParams &sp, const MergeParams &mp, hipStream_t st);
hipError_t launch_bins_block(int y_dtype, const ScanParams &sp, const MergeParams &mp, hipStream_t st);
hipError_t launch_compact(const CompactParams &p, hipStream_t st);
hipError_t launch_binres_to_outputs(const MergeParams &p, int64_t *imin, int64_t *imax,
                                    hipStream_t st);
hipError_t launch_window(const void *x, int x_dtype, int64_t n, int64_t xa, int64_t xb,
                         int64_t *range, hipStream_t st);

// LTTB over m points taken through `sel` (NULL = the series itself).
struct LttbParams {
  const void *x;
  int32_t x_dtype;        // TS_NONE: X is the index
  const void *y;
  int32_t y_dtype;
  const int64_t *sel;     // NULL or device [m_max]
  int64_t m;              // number of points, or -1: read *m_dev
  const int64_t *m_dev;
  int64_t m_max;
  int64_t n_out;
  double *cx;             // [n_out - 2] centres (workspace)
  double *cy;
  int32_t *next;          // [m_max] transition map (workspace)
  int32_t *entry;         // [groups + 1] workspace
  int64_t *out;
  int64_t *out_count;
  // candidate coordinates gathered after the preselection (NULL: read the
  // series through sel): one 64-bit word per candidate, the exact integer
  // (int64, or uint64 bits) for integer dtypes and the index without x, the
  // double for float dtypes
  uint64_t *gx;
  uint64_t *gy;
  // hull-pruned walk of plain LTTB (long buckets); NULL when unused
  int32_t *cand_cnt;      // [nb] candidates of bucket k, 0: walk every point of it
  int64_t *cand_idx;      // [nb * kHullCand]
  double *cand_x;         // [nb * kHullCand]
  double *cand_y;         // [nb * kHullCand]
  uint8_t *hnext;         // [nb * kHullCand] pick in bucket k for each candidate anchor of bucket k-1
  uint8_t *hjump;         // [groups * kHullCand] exit of each group for each entry anchor
  int32_t *hflag;         // [1] 1 when the map walk has written the result
};

// LDS of the small-bucket walk: its own tables (19 KB) plus the map next[]
// and jump[] (8 bytes per point, at most kWalkMapLds), within 144 KB per
// workgroup; larger maps stay in the workspace.
constexpr int64_t kWalkMapLds = 124 * 1024;

// Hull-pruned plain LTTB: used for buckets of at least kHullMinBucket points;
// at most kHullCand candidates are kept per bucket (else the bucket is walked
// in full) and kHullLane hull points per lane segment.
constexpr int64_t kHullMinBucket = 512;
constexpr int kHullCand = 64;
constexpr int kHullLane = 24;

hipError_t launch_lttb_centres(const LttbParams &p, hipStream_t st);
hipError_t launch_lttb_gather(const LttbParams &p, hipStream_t st);
hipError_t launch_lttb_hull(const LttbParams &p, hipStream_t st);
hipError_t launch_lttb_hull_walk(const LttbParams &p, hipStream_t st);
int64_t lttb_hull_group(int64_t nb);
// own_centres: the map computes each centre where it needs it (no centre
// pass before it).
hipError_t launch_lttb_small(const LttbParams &p, bool own_centres, hipStream_t st);
hipError_t launch_lttb_seq(const LttbParams &p, hipStream_t st);

}  // namespace tsds

namespace tsds {

// One task of a batched launch (device table entry).  Offsets (o_*) are
// byte offsets into the workspace; out_offset indexes the output array.
struct BatchTask {
  const void *y;        // scanned series (the interior for MinMaxLTTB)
  const void *x;        // NULL if no x
  int64_t n;
  int32_t ydt, xdt;
  int32_t algo;         // TS_MINMAX, TS_M4, TS_MINMAXLTTB, TS_NAN_MINMAX, TS_NAN_M4 (NaN-aware only for float y)
  int32_t mode;         // 0: scan; 1: n <= n_out (all indices); 2: MinMaxLTTB without preselection
  int32_t stage;        // 1: staged chunks (many small bins); 2: a wavefront per bin (no chunks, no merge)
  int32_t pad_;
  int64_t shift, chunk, nchunks, nb;
  int64_t chunk_begin;  // first work item (chunk, or bin when stage == 2) of this task in its group's list
  int64_t slot_begin;   // first global bin slot (nb + 1 slots per task)
  int64_t n_out, out_offset;
  int64_t o_edges, o_binres, o_partL, o_partR, o_sel, o_cnt;
  int64_t o_cand, o_m, o_cx, o_cy, o_next, o_entry, o_gx, o_gy;
  const void *yf;       // full series (MinMaxLTTB's LTTB step)
  const void *xf;
  int64_t nf;
  int64_t m_max;        // candidates capacity
};

struct BatchArgs {
  const BatchTask *tasks;
  const int32_t *slot_task;  // [total_slots] task of each global bin slot
  const int32_t *lttb_tasks; // [n_lttb] indices of MinMaxLTTB tasks
  int64_t ntasks, total_chunks, total_slots, n_lttb;
  int64_t wave_slots;        // slots [0, wave_slots): tasks merged a wavefront per bin
  char *ws;
  int64_t *out;
  int64_t *counts;
  int32_t small;
  int32_t lds_ok;            // LTTB maps fit in LDS for every task
  int64_t lds_m;             // m capacity of the LDS maps
  int64_t max_m;             // largest candidate capacity of a MinMaxLTTB task
};

hipError_t launch_batch_edges(const BatchArgs &a, hipStream_t st);
// Work list of one dtype group: the group's tasks in order (tix) and the
// first work item of each (cb, non-decreasing), total items.
struct BatchGroup {
  const int64_t *cb;
  const int32_t *tix;
  int64_t ntasks;
  int64_t total;
  int32_t ydt;
  int32_t stage;
  int32_t nan;     // NaN-aware tasks (floating-point y)
};

hipError_t launch_batch_scan(const BatchArgs &a, const BatchGroup &g, int64_t grid_blocks, hipStream_t st);
hipError_t launch_batch_scan_nan(const BatchArgs &a, const BatchGroup &g, int64_t grid_blocks, hipStream_t st);
hipError_t launch_batch_merge(const BatchArgs &a, hipStream_t st);
hipError_t launch_batch_compact(const BatchArgs &a, hipStream_t st);
hipError_t launch_batch_lttb(const BatchArgs &a, hipStream_t st);

}  // namespace tsds

namespace tsds {

// Zoom windows of up to kMaxWindows requests: ranges[2i], ranges[2i+1] =
// [i0, i1) of the points of request i with xa <= x <= xb (integer x).
constexpr int kMaxWindows = 32;
struct WindowBatch {
  const void *x[kMaxWindows];
  int64_t n[kMaxWindows];
  int64_t xa[kMaxWindows];
  int64_t xb[kMaxWindows];
  int32_t xdt[kMaxWindows];
  int32_t count;
  int64_t *ranges;
  int64_t *host_ranges;  // host-mapped copy of ranges (NULL: none)
};

hipError_t launch_windows(const WindowBatch &wb, hipStream_t st);

// Copies bytes with a kernel between device memory and host-mapped pinned
// memory (the serving loop avoids memcpy calls, which can hold the calling
// thread for milliseconds while other streams are busy).
hipError_t launch_copy_bytes(void *dst, const void *src, size_t bytes, hipStream_t st);
// Serving results to host-mapped memory: h_counts[i] = counts[i] and the
// first counts[i] entries of row i (rows of `row` int64) into h_rows.
hipError_t launch_export_rows(const int64_t *counts, const int64_t *rows, int64_t row, int n, int64_t *h_counts,
                              int64_t *h_rows, hipStream_t st);

// NaN-aware argmin/argmax scan (f16, f32, f64 y): NaN skipped, chunk-major
// like launch_scan, results in the same binres / partial slots.
hipError_t launch_scan_nan(int y_dtype, const ScanParams &p, hipStream_t st);

// EveryNth: out[i] = i*k for i < m, *count = m.
hipError_t launch_everynth(int64_t k, int64_t m, int64_t *out, int64_t *count, hipStream_t st);
// Gather of selected points, moved as raw words: xs, ys are the element sizes
// (xs = 0 or xo = NULL: y only).  Indices outside [0, n) are skipped.
hipError_t launch_gather(const void *x, int xs, const void *y, int ys, int64_t n, const int64_t *idx,
                         const int64_t *count, int64_t cap, void *xo, void *yo, hipStream_t st);

// Host-side argument checks and the thread-local error message of the C ABI
// (api.cpp), shared by the batched, served and allocation-free entry points.
int api_fail(int code, const char *msg);
int api_check_series(const ts_series *s);
int api_check_nout(int algo, int64_t n_out, int64_t ratio);

}  // namespace tsds

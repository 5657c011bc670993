/*
 * tsds.h -- C ABI of the MI355X (gfx950) time-series downsampling library
 * (libtsds.so).
 *
 * The library computes the data-parallel hot path of the downsamplers in
 * "tsdownsample: high-performance time series downsampling for scalable
 * visualization" (arXiv 2307.05389): the per-bin argmin/argmax scan behind
 * MinMax, M4 and the MinMax preselection of MinMaxLTTB (Sec. 2.1, Listing 1;
 * Sec. 2.2), and the bucketed triangle-area argmax of LTTB (Sec. 4, LTTB and
 * MinMaxLTTB rows of Table 1).  The user-facing operation the paper defines is
 *     downsample([x], y, n_out) -> indices                        (Sec. 2.3)
 * x optional (absent = equally sampled without gaps), y mandatory, n_out the
 * number of output points, fewer returned when x has gaps (empty bins).
 *
 * Conventions shared by every entry point
 *   - All data pointers (x, y, outputs, workspace) are DEVICE pointers
 *     (hipMalloc'ed or equivalent) unless the comment says "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call only enqueues work on that stream and returns; results are
 *     valid once the stream has reached that point.  Nothing is allocated
 *     on the device by the compute calls; the caller owns every buffer, and
 *     the library keeps no pointer after a call returns.
 *   - Indices are int64, into the caller's series, strictly increasing.
 *   - x must be sorted non-decreasing and finite; y must hold no NaN.
 *     These preconditions are not checked (checking would cost a pass over
 *     the data); violating them gives unspecified but in-bounds indices.
 *   - Every element pointer must be aligned to its element size.
 *   - Return value: TS_OK (0) or a negative TS_ERR_* code.  All argument
 *     checks happen before anything is enqueued, so an error leaves every
 *     output untouched.  ts_last_error() gives a thread-local message.
 *
 * Workspace: each compute call takes a scratch buffer `ws` of at least
 * ts_workspace_bytes(...) bytes (device memory, any content, 256-byte
 * aligned).  Calls that overlap in time must not share a workspace.
 */
#ifndef TSDS_H
#define TSDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element types (the dtypes the paper's argminmax supports, Sec. 2.1). */
enum {
  TS_NONE = -1, /* x absent */
  TS_I8 = 0, TS_I16 = 1, TS_I32 = 2, TS_I64 = 3,
  TS_U8 = 4, TS_U16 = 5, TS_U32 = 6, TS_U64 = 7,
  TS_F16 = 8, TS_F32 = 9, TS_F64 = 10
};

/* Status codes. */
enum {
  TS_OK = 0,
  TS_ERR_ARG = -1,        /* bad size, n_out or ratio */
  TS_ERR_DTYPE = -2,      /* unsupported dtype for that argument */
  TS_ERR_NULL = -3,       /* required pointer is NULL, or x/x_dtype mismatch */
  TS_ERR_WORKSPACE = -4,  /* ws_bytes smaller than required, or ws misaligned */
  TS_ERR_HIP = -5,        /* a HIP runtime call or kernel launch failed */
  TS_ERR_ALIGN = -6,      /* an element pointer is not aligned to its size */
  TS_ERR_CANCELLED = -7,  /* serving: the request was cancelled before it ran */
  TS_ERR_TIMEOUT = -8     /* serving: the request waited longer than the server's timeout */
};

/* Algorithms. */
enum { TS_MINMAX = 0, TS_M4 = 1, TS_LTTB = 2, TS_MINMAXLTTB = 3, TS_NAN_MINMAX = 4, TS_NAN_M4 = 5 };

/* One series.  y: n elements of y_dtype (any of the 11 types).
 * x: NULL (x_dtype = TS_NONE) or n sorted elements of x_dtype in
 * {TS_I32, TS_I64, TS_U32, TS_U64, TS_F32, TS_F64}. */
typedef struct {
  const void *x;
  int32_t x_dtype;
  const void *y;
  int32_t y_dtype;
  int64_t n;
} ts_series;

/* Library version (major*10000 + minor*100 + patch). */
int ts_version(void);

/* Message describing the last error returned on this host thread. */
const char *ts_last_error(void);

/* Bytes of workspace `algo` needs for this series and n_out (minmax_ratio is
 * read for TS_MINMAXLTTB only).  Returns 0 if the arguments are invalid;
 * a valid call may also need 0 bytes only if n <= n_out. */
size_t ts_workspace_bytes(int algo, const ts_series *s, int64_t n_out, int64_t minmax_ratio);

/* MinMax (Sec. 2.1, Sec. 2.2): n_out/2 bins; each non-empty bin keeps the
 * first index of its minimum and the first index of its maximum.
 * Bins: without x, bin b = [ceil(b(n-1)/nb), ceil((b+1)(n-1)/nb)) with the
 * last bin ending at n (equal index ranges, identical to x = 0..n-1); with
 * x, nb equal-width bins over [x[0], x[n-1]] located by search-sorted, the
 * last bin closed on both sides.  n_out must be even and >= 2.
 * n <= n_out returns 0..n-1.  out_idx: device int64[n_out] (written up to
 * *out_count); out_count: device int64[1]. */
int ts_minmax(const ts_series *s, int64_t n_out, int64_t *out_idx, int64_t *out_count,
              void *ws, size_t ws_bytes, void *stream);

/* M4 (Jugel et al., cited in Sec. 1): n_out/4 bins, same bins as MinMax;
 * each non-empty bin keeps its first index, argmin, argmax and last index,
 * de-duplicated.  n_out must be a multiple of 4 and >= 4. */
int ts_m4(const ts_series *s, int64_t n_out, int64_t *out_idx, int64_t *out_count,
          void *ws, size_t ws_bytes, void *stream);

/* LTTB (Steinarsson, cited in Sec. 1; Sec. 4): first and last point kept;
 * the n-2 interior points split into n_out-2 buckets by count
 * (bucket k = [1+floor(k(n-2)/(n_out-2)), 1+floor((k+1)(n-2)/(n_out-2))));
 * walking the buckets in order, each keeps the first point of largest
 * triangle area with the previous pick and the mean (x, y) of the next
 * bucket (the last bucket uses the last point).  Coordinates are x (or the
 * index) and y, widened to double; means use exact integer sums for integer
 * coordinates; the area is |(XA-Cx)(Yb-YA) - (XA-Xb)(Cy-YA)| in double with
 * no fused multiply-add.  n_out >= 3; *out_count = min(n, n_out). */
int ts_lttb(const ts_series *s, int64_t n_out, int64_t *out_idx, int64_t *out_count,
            void *ws, size_t ws_bytes, void *stream);

/* MinMaxLTTB (Van Der Donckt et al., cited in Sec. 1; Sec. 4): MinMax with
 * n_out*minmax_ratio outputs over the interior points 1..n-2 (x-range bins
 * over the interior when x is given) plus the first and last point form the
 * candidates; LTTB with n_out outputs runs on the candidates with their
 * original coordinates.  minmax_ratio >= 1, n_out*minmax_ratio even. */
int ts_minmaxlttb(const ts_series *s, int64_t n_out, int64_t minmax_ratio, int64_t *out_idx,
                  int64_t *out_count, void *ws, size_t ws_bytes, void *stream);

/* ts_minmaxlttb without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc).  The library brings its own
 * scratch: one static device array of ts_noalloc_scratch_bytes() = 64 MiB per
 * GPU, reserved when the library's code is loaded on that GPU and held until
 * the process ends; its device address is looked up once per GPU, on the
 * first call there.  Arguments, outputs and results are those of
 * ts_minmaxlttb on the stream's device (NULL stream: the current device).
 * Errors: TS_ERR_WORKSPACE, before anything touches the GPU, when
 * ts_workspace_bytes(TS_MINMAXLTTB, s, n_out, minmax_ratio) exceeds the
 * scratch (n_out of a few thousand: up to ~16 GB of y; n_out ~200,000: a
 * few GB); otherwise ts_minmaxlttb's checks and codes.
 * The scratch needs no initial content, and every call on a GPU reuses that
 * GPU's one array: calls whose work overlaps in time on the same GPU (two
 * streams, two host threads) race on it and must be serialised by the
 * caller. */
size_t ts_noalloc_scratch_bytes(void);
int ts_minmaxlttb_noalloc(const ts_series *s, int64_t n_out, int64_t minmax_ratio, int64_t *out_idx,
                          int64_t *out_count, void *stream);

/* NaN-aware MinMax and M4 (the paper flags NaN as needing a different
 * initial value, Sec. 2.1, Listing 1, and defines no more).  Reading: NaN
 * values of y are skipped; a bin holding only NaN keeps its first index as
 * both argmin and argmax (so MinMax returns that one index and M4 its first
 * and last).  Everything else (bins, ties, +-0, de-duplication, n <= n_out,
 * n_out rules, workspace via ts_workspace_bytes(TS_NAN_MINMAX / TS_NAN_M4))
 * is as for ts_minmax / ts_m4, and these are the only calls for which y may
 * hold NaN.  Integer y holds no NaN: the result equals ts_minmax / ts_m4. */
int ts_nan_minmax(const ts_series *s, int64_t n_out, int64_t *out_idx, int64_t *out_count,
                  void *ws, size_t ws_bytes, void *stream);
int ts_nan_m4(const ts_series *s, int64_t n_out, int64_t *out_idx, int64_t *out_count,
              void *ws, size_t ws_bytes, void *stream);

/* ---- Single steps of the path, exposed so each can be checked alone ---- */

/* Bin starts edges[0..nb] (edges[nb] = n) as used by ts_minmax / ts_m4 for
 * nb bins (search-sorted binning, Sec. 2.2).  edges: device int64[nb+1]. */
int ts_bin_edges(const ts_series *s, int64_t nb, int64_t *edges, void *stream);

/* Per-bin argmin/argmax over the bins given by edges[0..nb] (device int64,
 * non-decreasing, edges[0] >= 0, edges[nb] <= n): imin[b], imax[b] (device
 * int64[nb]) receive the first index of the bin's minimum / maximum, or -1
 * for an empty bin (Sec. 2.1, Listing 1).  ws: ts_argminmax_workspace_bytes. */
size_t ts_argminmax_workspace_bytes(const ts_series *s, int64_t nb);
int ts_bin_argminmax(const ts_series *s, const int64_t *edges, int64_t nb, int64_t *imin,
                     int64_t *imax, void *ws, size_t ws_bytes, void *stream);

/* LTTB centres for m points taken through `sel` (device int64[m] indices
 * into the series, or NULL for all n points): cx[k], cy[k] (device
 * double[n_out-2]) = mean x and y of bucket k+1, or the last point for the
 * last bucket.  Requires m > n_out >= 3. */
int ts_lttb_centres(const ts_series *s, const int64_t *sel, int64_t m, int64_t n_out,
                    double *cx, double *cy, void *stream);

/* Zoom window: [i0, i1) = the points with xa <= x <= xb, written to the
 * device int64[2] `range` (integer x only). */
int ts_window(const ts_series *s, int64_t xa, int64_t xb, int64_t *range, void *stream);

/* ---- EveryNth and the gather of selected points ------------------------ */

/* EveryNth (listed among the downsamplers in Sec. 1; Table 1): the indices
 * 0, k, 2k, ... below n with k = ceil(n / n_out), the smallest stride whose
 * output fits n_out, so *out_count = ceil(n / k) <= n_out.  Only the index
 * list is written; x and y are not read (the series gives n and is checked
 * like every other call).  n <= n_out returns 0..n-1.  n_out >= 1.
 * out_idx: device int64[min(n, n_out)]; out_count: device int64[1].  No
 * workspace. */
int ts_everynth(const ts_series *s, int64_t n_out, int64_t *out_idx, int64_t *out_count, void *stream);

/* The selected points themselves (the indices retrieve the representative
 * subset that is drawn, Sec. 2.3): for i < min(*count, cap),
 * y_out[i] = y[idx[i]] and, when x_out is not NULL, x_out[i] = x[idx[i]],
 * in the series' own element types.  idx, count: device int64 (typically a
 * downsampler's out_idx / out_count, read on the device, so no host sync is
 * needed); idx holds at least min(*count, cap) entries (a negative count
 * gathers nothing); y_out, x_out: device buffers of cap elements aligned to their
 * element size.  x_out must be NULL when the series has no x.  An index
 * outside [0, n) writes nothing at its position.  cap = 0 enqueues nothing. */
int ts_gather(const ts_series *s, const int64_t *idx, const int64_t *count, int64_t cap, void *x_out,
              void *y_out, void *stream);

/* ---- Batched mode: many series in one pass ---------------------------- */

/* One task: a series, its algorithm (TS_MINMAX, TS_M4, TS_MINMAXLTTB, or the
 * NaN-aware TS_NAN_MINMAX / TS_NAN_M4 with ts_nan_minmax's semantics),
 * n_out, minmax_ratio (MinMaxLTTB only, 1..30) and the first slot of its
 * output in the batch's out_idx array (it writes up to n_out indices there
 * and its count to counts[task]). */
typedef struct {
  int32_t algo;
  ts_series series;
  int64_t n_out;
  int64_t minmax_ratio;
  int64_t out_offset;
} ts_task;

typedef struct ts_plan ts_plan;

/* Validates every task (same rules as the single-series calls) and builds
 * the per-series offset tables: every series is cut into equal-byte chunks
 * of one global work list and its bins into one global list of bin slots.
 * The plan keeps the series pointers (they must stay valid while the plan is
 * used) and owns a small device table (about 160 B per task + 4 B per bin)
 * that it allocates here and frees in ts_plan_free.  *plan = NULL on error. */
int ts_batch_plan(const ts_task *tasks, int64_t n_tasks, ts_plan **plan);

/* Workspace bytes ts_batch_run needs (any tuning), and the length out_idx
 * must have (max over tasks of out_offset + n_out). */
size_t ts_batch_workspace_bytes(const ts_plan *plan);
int64_t ts_batch_out_size(const ts_plan *plan);

/* Runs every task: one persistent argmin/argmax launch per element type
 * present (and per chunk kind: plain or LDS-staged), one merge launch over
 * all bins (a wavefront per bin for long bins, a thread per bin for short
 * ones), one compaction launch (one workgroup per task) and, if there are
 * MinMaxLTTB tasks, one LTTB launch (one workgroup per task).  The scans of
 * different element types run concurrently on up to three side streams
 * (default priority) owned by the plan, forked from `stream` by an event and
 * joined back to it before the merge, so the caller sees one ordered
 * sequence on `stream`.  Outputs are identical to one single-series call per
 * task.  use_graph != 0: the launches are captured once into a hipGraph
 * (re-captured when out_idx, counts or ws change) and replayed with one
 * hipGraphLaunch on `stream`.  out_idx: device int64 [ts_batch_out_size];
 * counts: device int64[n_tasks]; ws: device, 256-byte aligned, >=
 * ts_batch_workspace_bytes.  Calls on one plan must not overlap (the side
 * streams and the graph belong to the plan). */
int ts_batch_run(ts_plan *plan, int64_t *out_idx, int64_t *counts, void *ws, size_t ws_bytes, void *stream,
                 int use_graph);

/* Tuning of a plan: chunk_bytes (power of two, 4 KiB..4 MiB) per work item,
 * small_bin (segments shorter than this are reduced one bin per lane, i.e.
 * up to 64 bins per wavefront) and the persistent grid size in workgroups of
 * four wavefronts.  Results do not depend on them. */
int ts_batch_set_tuning(ts_plan *plan, int64_t chunk_bytes, int32_t small_bin, int64_t grid_blocks);
int ts_batch_get_tuning(const ts_plan *plan, int64_t *chunk_bytes, int32_t *small_bin, int64_t *grid_blocks);

/* Autotuner: times every candidate (chunk 8..64 KiB x small_bin 32/128/512 x
 * grid 4/6/8 workgroups per CU) on the caller's buffers, keeps the fastest,
 * and synchronises `stream`.  With cache_path (a text file), the choice is
 * stored per batch signature (the dtype / algorithm / size-class mix) and
 * reused without timing.  Results never change. */
int ts_batch_autotune(ts_plan *plan, int64_t *out_idx, int64_t *counts, void *ws, size_t ws_bytes, void *stream,
                      const char *cache_path);

void ts_plan_free(ts_plan *plan);

/* ---- Serving: zoom/pan requests over series resident in HBM ------------ */

typedef struct {
  int32_t n_streams;     /* concurrent batches in flight (1..16), one HIP stream each */
  int32_t max_batch;     /* requests per batch (1..32) */
  int64_t max_nout;      /* largest n_out a request may ask for */
  int64_t minmax_ratio;  /* MinMaxLTTB preselection ratio (1..30) */
  int32_t plain;         /* 1: no batching -- each request alone, in arrival order, with
                            ts_window + ts_minmaxlttb on one stream (baseline) */
  size_t arena_bytes;    /* device workspace per stream (0: max_batch worst-case requests);
                            raised to at least one worst-case request */
  double timeout_s;      /* a request still pending this many seconds after submission is
                            dropped with status TS_ERR_TIMEOUT (0: never) */
} ts_server_config;

/* One finished request.  Its indices (into the full series, strictly
 * increasing) are idx[offset .. offset+count) of the poll buffer. */
typedef struct {
  int64_t id;
  int32_t series;
  int32_t status;       /* TS_OK, the error of the batch it ran in, or TS_ERR_CANCELLED /
                           TS_ERR_TIMEOUT for a request that never ran (count 0) */
  int64_t count;
  int64_t offset;
  int64_t i0, i1;       /* the request's window [i0, i1) */
  double t_submit;      /* ts_server_now() at submission */
  double t_done;        /* ts_server_now() when the indices were in host memory */
  int64_t batch_size;   /* requests in the batch it ran in */
  double t_admit;       /* its batch was admitted to a slot (window search enqueued) */
  double t_run;         /* the windows had arrived and the downsampling was enqueued */
} ts_result;

typedef struct ts_server ts_server;

/* Starts a server over n_series resident series (device x, int32/int64/
 * uint32/uint64, and y of any dtype; they must stay valid until
 * ts_server_free).  A request (series, xa, xb, n_out) is MinMaxLTTB with
 * cfg->minmax_ratio on the points with xa <= x <= xb, indices into the full
 * series (the zoom/pan use of Sec. 1).  One scheduler thread admits pending
 * requests oldest-first into free streams -- at most max_batch per batch and
 * only while their worst-case workspace fits the stream's arena -- resolves
 * their windows on the device, runs them as one batch (ts_batch_run's
 * kernels) and copies the results back; batches on different streams overlap
 * on the GPU, and requests that arrive meanwhile join the next free stream.
 * A batch of one request runs the single-series kernels.  Every result
 * equals ts_minmaxlttb on its window alone.  Allocates the
 * arenas and pinned buffers here; ts_server_free releases them. */
int ts_server_create(const ts_series *series, int32_t n_series, const ts_server_config *cfg, ts_server **server);

/* Queues a request; *req_id receives its id.  Thread-safe. */
int ts_server_submit(ts_server *server, int32_t series, int64_t xa, int64_t xb, int64_t n_out, int64_t *req_id);

/* Cancels a request that is still pending (not yet admitted to a stream):
 * it comes back from ts_server_poll with status TS_ERR_CANCELLED and no
 * indices.  TS_ERR_ARG if the request is unknown, already running or
 * finished (a running batch always completes).  Thread-safe. */
int ts_server_cancel(ts_server *server, int64_t req_id);

/* Moves up to max_results finished requests out of the server: metadata to
 * res[], indices to the host buffer idx (capacity idx_cap); *n_results =
 * how many.  Thread-safe. */
int ts_server_poll(ts_server *server, ts_result *res, int32_t max_results, int64_t *idx, int64_t idx_cap,
                   int32_t *n_results);

/* Counters; returns the last batch error (TS_OK if none). */
int ts_server_stats(ts_server *server, int64_t *batches, int64_t *max_batch, int64_t *requests_done,
                    int64_t *pending);

/* Seconds on the server's monotonic clock (the clock of t_submit/t_done). */
double ts_server_now(void);

/* Finishes every queued request, joins the scheduler, frees everything. */
void ts_server_free(ts_server *server);

/* Tuning knobs of the argmin/argmax pass, process-wide: chunk_bytes (a power
 * of two >= 4096; -1 = automatic) is the slice of y one wavefront reduces;
 * bin segments shorter than small_bin elements (-1 = default 128) are reduced
 * one bin per lane instead of one bin per wavefront; scan_variant (-1 =
 * default, 0..4) picks the tile shape (16-byte vectors per lane per tile and
 * tiles in flight: 0 = 4x2, 1 = 4x1, 2 = 8x1, 3 = 2x2; 4 = each chunk's
 * tiles walked once in order, every tile folded into the bins it overlaps); stage (-1 = automatic:
 * on when bins average < 4096 elements, 0 = off, 1 = on) copies each chunk to
 * LDS first and reduces its bins from there (chunk_bytes <= 32768 when on);
 * xclass (-1 = automatic: on for int64 x when bins average at least two
 * chunks, 0 = off, 1 = on; int64 x and unstaged scans only) lets each chunk
 * find its bins from x directly, so that the edge array is written by the scan
 * instead of a separate edge search; direct (-1 = automatic: series up to
 * 8 MB in at least 64 bins of at least 256 elements, and series without x
 * in at least 2,000 bins of 4-512 KB, get a wavefront per bin; series
 * without x in 500-1,999 bins (eight-byte types 250-1,999) of at least
 * 256 KB get a workgroup per bin;
 * 0 = off, 1 = a wavefront per bin, 2 = a workgroup of four wavefronts per
 * bin (a wavefront per bin above 2^23 bins), for every MinMax / M4 call and
 * preselection; neither above 2^25 bins) gives each bin one
 * wavefront or workgroup that reduces the whole bin and writes its
 * selection (no chunks, partials or merge; any other override set switches
 * the automatic choice off).
 * Results never depend on them; workspace sizes do, so query
 * ts_workspace_bytes after a change.  Not thread-safe with concurrent
 * compute calls. */
int ts_set_tuning(int64_t chunk_bytes, int32_t small_bin, int32_t scan_variant, int32_t stage, int32_t xclass,
                  int32_t direct);

/* Host-side query: the scan's tile variant, chunk size (bytes) and kind
 * (0 = chunks with an edge array or closed-form bins, 1 = LDS-staged,
 * 2 = classified from int64 x, 3 = chunks streamed tile by tile over their
 * bins, 4 = one wavefront per bin, no chunks, 5 = one workgroup of four
 * wavefronts per bin, no chunks) for n elements of y_dtype in nb
 * bins, x of x_dtype (TS_NONE: no x), under the current tuning. */
int ts_scan_config(int y_dtype, int x_dtype, int64_t n, int64_t nb, int32_t *variant, int64_t *chunk_bytes,
                   int32_t *kind);

/* Timing hook: when both are non-NULL, the next single-series compute calls
 * launch the argmin/argmax scan kernel with hipExtLaunchKernel, which stamps
 * the hipEvent_t `start` and `stop` (created by the caller) with that
 * dispatch's own start and end times, so hipEventElapsedTime gives the
 * kernel's duration alone.  Pass NULL, NULL to switch it off.  Process-wide. */
int ts_profile_scan_events(void *start, void *stop);

#ifdef __cplusplus
}
#endif

#endif /* TSDS_H */

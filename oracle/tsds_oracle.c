/*
 * tsds_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU oracle for the downsampling hot path
 * of "tsdownsample: high-performance time series downsampling for scalable
 * visualization" (Van Der Donckt, Van Der Donckt, Van Hoecke; arXiv 2307.05389).
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code, header, table or constant with
 * the GPU library; it is compiled with gcc -O2 -ffp-contract=off so that every
 * floating-point expression is evaluated exactly as written (no FMA).
 *
 * What the paper fixes, and what this file therefore computes:
 *   - MinMax, M4 and MinMaxLTTB take, inside every bin, the index of the
 *     minimum and of the maximum in one pass (Sec. 2.1, Listing 1: strict
 *     less-than / greater-than compares that keep the earlier index on ties).
 *   - Bins are local and independent; their boundaries come from a
 *     search-sorted over x (Sec. 2.2).
 *   - x is optional; without x the series is equally sampled with no gaps,
 *     and an equally sampled x must give the same result as no x
 *     (Sec. 2.2 unit-test remark, Sec. 2.3).
 *   - Empty bins (gaps in x) select nothing, so fewer than n_out indices may
 *     be returned (Sec. 2.3, footnote on n_out).
 *   - The result is an array of indices into the series (Sec. 2.3).
 *   - f16 is ordered by its numeric value; unsigned integers by their
 *     unsigned value (Sec. 2.1.2: the i16ord and XOR maps only preserve that
 *     order).  Here every value is compared by exact widening to a common type.
 * Where the paper is silent (bin-edge formulas, tie-break across lanes, +-0,
 * LTTB bucketing, mean precision, MinMaxLTTB composition) the readings are the
 * ones documented beside each function below.
 *
 * Every entry point returns 0 on success and a negative value on a bad
 * argument; indices are int64.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* dtype codes of this oracle (independent of the GPU library's codes) */
enum {
  OR_I8 = 0, OR_I16 = 1, OR_I32 = 2, OR_I64 = 3,
  OR_U8 = 4, OR_U16 = 5, OR_U32 = 6, OR_U64 = 7,
  OR_F16 = 8, OR_F32 = 9, OR_F64 = 10
};

typedef __int128 i128;

/* ------------------------------------------------------------------ */
/* Values: every element is widened exactly to one of three classes.   */
/* ------------------------------------------------------------------ */

enum { CLS_SIGNED = 0, CLS_UNSIGNED = 1, CLS_FLOAT = 2 };

typedef struct {
  int cls;
  int64_t s;
  uint64_t u;
  double f;
} oval;

/* IEEE 754 binary16 -> double, written from the format's definition:
 * 1 sign bit, 5 exponent bits (bias 15), 10 fraction bits.  Exact. */
static double half_to_double(uint16_t h) {
  int sign = (h >> 15) & 1;
  int e = (h >> 10) & 0x1f;
  int frac = h & 0x3ff;
  double mag;
  if (e == 0) {
    mag = ldexp((double)frac, -24);               /* subnormal: frac * 2^-24 */
  } else if (e == 31) {
    mag = frac ? NAN : INFINITY;
  } else {
    mag = ldexp((double)(1024 + frac), e - 25);   /* (1 + frac/1024) * 2^(e-15) */
  }
  return sign ? -mag : mag;
}

static int dtype_valid(int dt) { return dt >= OR_I8 && dt <= OR_F64; }

static int dtype_class(int dt) {
  if (dt <= OR_I64) return CLS_SIGNED;
  if (dt <= OR_U64) return CLS_UNSIGNED;
  return CLS_FLOAT;
}

static oval load(const void *p, int dt, int64_t i) {
  oval v;
  v.cls = dtype_class(dt);
  v.s = 0; v.u = 0; v.f = 0.0;
  switch (dt) {
    case OR_I8:  v.s = ((const int8_t *)p)[i]; break;
    case OR_I16: v.s = ((const int16_t *)p)[i]; break;
    case OR_I32: v.s = ((const int32_t *)p)[i]; break;
    case OR_I64: v.s = ((const int64_t *)p)[i]; break;
    case OR_U8:  v.u = ((const uint8_t *)p)[i]; break;
    case OR_U16: v.u = ((const uint16_t *)p)[i]; break;
    case OR_U32: v.u = ((const uint32_t *)p)[i]; break;
    case OR_U64: v.u = ((const uint64_t *)p)[i]; break;
    case OR_F16: v.f = half_to_double(((const uint16_t *)p)[i]); break;
    case OR_F32: v.f = (double)((const float *)p)[i]; break;
    case OR_F64: v.f = ((const double *)p)[i]; break;
  }
  return v;
}

/* Natural numeric order; IEEE compares for floats, so -0 == +0. */
static int less(oval a, oval b) {
  if (a.cls == CLS_SIGNED) return a.s < b.s;
  if (a.cls == CLS_UNSIGNED) return a.u < b.u;
  return a.f < b.f;
}

static int greater(oval a, oval b) { return less(b, a); }

/* Value as a double (round to nearest for 64-bit integers beyond 2^53). */
static double as_double(oval v) {
  if (v.cls == CLS_SIGNED) return (double)v.s;
  if (v.cls == CLS_UNSIGNED) return (double)v.u;
  return v.f;
}

/* ------------------------------------------------------------------ */
/* Argmin / argmax of one bin (Sec. 2.1, Listing 1).                   */
/* ------------------------------------------------------------------ */

/* Scan y[lo..hi) in index order.  The running minimum and maximum start at
 * the bin's first element; an element replaces them only when it is strictly
 * smaller (resp. strictly larger), so both results are the FIRST index at
 * which the extreme value occurs.  Requires lo < hi. */
int oracle_argminmax(const void *y, int ydt, int64_t lo, int64_t hi,
                     int64_t *imin, int64_t *imax) {
  if (!y || !imin || !imax || !dtype_valid(ydt) || lo < 0 || hi <= lo) return -1;
  oval vmin = load(y, ydt, lo), vmax = vmin;
  int64_t amin = lo, amax = lo;
  for (int64_t i = lo + 1; i < hi; i++) {
    oval v = load(y, ydt, i);
    if (less(v, vmin)) { vmin = v; amin = i; }
    if (greater(v, vmax)) { vmax = v; amax = i; }
  }
  *imin = amin;
  *imax = amax;
  return 0;
}

/* ------------------------------------------------------------------ */
/* Bin edges (Sec. 2.2 search-sorted binning; Sec. 2.3 optional x).    */
/* ------------------------------------------------------------------ */

/* No x: the series is equally sampled, i.e. x = 0, 1, ..., n-1.  Applying
 * the integer-x rule below to that x gives s_b = ceil(b (n-1) / nb), which is
 * what makes "equally sampled x == no x" hold exactly.  edges[nb] = n. */
int oracle_edges_nox(int64_t n, int64_t nb, int64_t *edges) {
  if (n < 0 || nb < 1 || !edges) return -1;
  for (int64_t b = 0; b < nb; b++) {
    i128 num = (i128)b * (i128)(n > 0 ? n - 1 : 0);
    i128 q = num / nb;
    if (q * nb < num) q += 1;              /* ceiling of a non-negative ratio */
    edges[b] = (int64_t)q;
  }
  edges[nb] = n;
  if (n == 0) for (int64_t b = 0; b <= nb; b++) edges[b] = 0;
  return 0;
}

/* Bin edge value E_b for integer x: x0 + ceil(b * R / nb), R = x_last - x0,
 * all exact in 128-bit integers. */
static i128 int_edge_value(i128 x0, i128 R, int64_t b, int64_t nb) {
  i128 num = (i128)b * R;
  i128 q = num / nb;
  if (q * nb < num) q += 1;
  return x0 + q;
}

static i128 int_x(const void *x, int xdt, int64_t i) {
  oval v = load(x, xdt, i);
  return v.cls == CLS_SIGNED ? (i128)v.s : (i128)v.u;
}

/* With x: nb bins of equal width over [x[0], x[n-1]], left-closed, the last
 * one closed on both ends.  s_b is the first index whose x is >= E_b (a
 * left search-sorted of the edge values into the sorted x).
 *   integer x: E_b = x0 + ceil(b R / nb), exact;
 *   float x:   E_b = x0 + ((double)b * R) / (double)nb, each operation
 *              rounded to nearest, with x widened exactly to double.
 * The search is one forward sweep (edges are non-decreasing). */
int oracle_edges_x(const void *x, int xdt, int64_t n, int64_t nb, int64_t *edges) {
  if (!x || !edges || n < 0 || nb < 1) return -1;
  if (xdt == OR_I8 || xdt == OR_I16 || xdt == OR_U8 || xdt == OR_U16 || xdt == OR_F16 ||
      !dtype_valid(xdt))
    return -2;
  if (n == 0) {
    for (int64_t b = 0; b <= nb; b++) edges[b] = 0;
    return 0;
  }
  int64_t i = 0;
  if (dtype_class(xdt) != CLS_FLOAT) {
    i128 x0 = int_x(x, xdt, 0), R = int_x(x, xdt, n - 1) - x0;
    for (int64_t b = 0; b < nb; b++) {
      i128 E = int_edge_value(x0, R, b, nb);
      while (i < n && int_x(x, xdt, i) < E) i++;
      edges[b] = i;
    }
  } else {
    double x0 = load(x, xdt, 0).f, R = load(x, xdt, n - 1).f - x0;
    for (int64_t b = 0; b < nb; b++) {
      double E = x0 + ((double)b * R) / (double)nb;
      while (i < n && load(x, xdt, i).f < E) i++;
      edges[b] = i;
    }
  }
  edges[nb] = n;
  return 0;
}

static int make_edges(const void *x, int xdt, int64_t n, int64_t nb, int64_t *edges) {
  return x ? oracle_edges_x(x, xdt, n, nb, edges) : oracle_edges_nox(n, nb, edges);
}

/* ------------------------------------------------------------------ */
/* Emit: sorted distinct indices per bin, concatenated in bin order.    */
/* ------------------------------------------------------------------ */

static int64_t emit_sorted_distinct(int64_t *v, int k, int64_t *out) {
  for (int a = 1; a < k; a++)                     /* insertion sort, k <= 4 */
    for (int c = a; c > 0 && v[c - 1] > v[c]; c--) {
      int64_t t = v[c]; v[c] = v[c - 1]; v[c - 1] = t;
    }
  int64_t m = 0;
  for (int a = 0; a < k; a++)
    if (a == 0 || v[a] != v[a - 1]) out[m++] = v[a];
  return m;
}

static int64_t emit_all(int64_t n, int64_t *out) {
  for (int64_t i = 0; i < n; i++) out[i] = i;
  return n;
}

/* MinMax: nb = n_out / 2 bins; each non-empty bin contributes its argmin and
 * argmax (Sec. 2.1: the inner loop of MinMax).  n <= n_out returns every
 * index.  n_out must be even and >= 2. */
int oracle_minmax(const void *x, int xdt, const void *y, int ydt, int64_t n,
                  int64_t n_out, int64_t *out, int64_t *count) {
  if (!y || !out || !count || !dtype_valid(ydt) || n < 0) return -1;
  if (n_out < 2 || n_out % 2) return -1;
  if (n <= n_out) { *count = emit_all(n, out); return 0; }
  int64_t nb = n_out / 2;
  int64_t *edges = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb + 1));
  if (!edges) return -3;
  int rc = make_edges(x, xdt, n, nb, edges);
  if (rc) { free(edges); return rc; }
  int64_t m = 0;
  for (int64_t b = 0; b < nb; b++) {
    if (edges[b] >= edges[b + 1]) continue;       /* empty bin: nothing */
    int64_t v[2];
    oracle_argminmax(y, ydt, edges[b], edges[b + 1], &v[0], &v[1]);
    m += emit_sorted_distinct(v, 2, out + m);
  }
  free(edges);
  *count = m;
  return 0;
}

/* EveryNth (Sec. 1 lists it among the downsamplers; Sec. 4 and Table 1
 * report its constant time): every k-th index 0, k, 2k, ... below n.  The
 * paper does not give k; the reading here is the smallest stride whose output
 * fits n_out, k = ceil(n / n_out), so the count is ceil(n / k) <= n_out.
 * x plays no part (the points are taken by index).  n <= n_out returns every
 * index; n_out must be >= 1. */
int oracle_everynth(int64_t n, int64_t n_out, int64_t *out, int64_t *count) {
  if (!out || !count || n < 0 || n_out < 1) return -1;
  if (n <= n_out) { *count = emit_all(n, out); return 0; }
  int64_t k = n / n_out + (n % n_out != 0);
  int64_t m = 0;
  for (int64_t i = 0; i < n; i += k) out[m++] = i;
  *count = m;
  return 0;
}

/* M4 (Jugel et al., cited by the paper): nb = n_out / 4 bins; each non-empty
 * bin contributes its first index, argmin, argmax and last index. */
int oracle_m4(const void *x, int xdt, const void *y, int ydt, int64_t n,
              int64_t n_out, int64_t *out, int64_t *count) {
  if (!y || !out || !count || !dtype_valid(ydt) || n < 0) return -1;
  if (n_out < 4 || n_out % 4) return -1;
  if (n <= n_out) { *count = emit_all(n, out); return 0; }
  int64_t nb = n_out / 4;
  int64_t *edges = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb + 1));
  if (!edges) return -3;
  int rc = make_edges(x, xdt, n, nb, edges);
  if (rc) { free(edges); return rc; }
  int64_t m = 0;
  for (int64_t b = 0; b < nb; b++) {
    if (edges[b] >= edges[b + 1]) continue;
    int64_t v[4];
    v[0] = edges[b];
    oracle_argminmax(y, ydt, edges[b], edges[b + 1], &v[1], &v[2]);
    v[3] = edges[b + 1] - 1;
    m += emit_sorted_distinct(v, 4, out + m);
  }
  free(edges);
  *count = m;
  return 0;
}

/* ------------------------------------------------------------------ */
/* Bin-parallel driver (CPU baseline only: Sec. 2.2 runs bins on all    */
/* cores).  The same per-bin scalar loop as oracle_minmax / oracle_m4,  */
/* with the bins split into contiguous ranges, one per thread; the      */
/* result is identical because bins are independent.                   */
/* ------------------------------------------------------------------ */

/* First index in [0, n) whose x is >= E (integer x, exact). */
static int64_t lower_bound_int(const void *x, int xdt, int64_t n, i128 E) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (int_x(x, xdt, mid) < E) lo = mid + 1; else hi = mid;
  }
  return lo;
}

/* First index in [0, n) whose (double)x is >= E (float x). */
static int64_t lower_bound_flt(const void *x, int xdt, int64_t n, double E) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (load(x, xdt, mid).f < E) lo = mid + 1; else hi = mid;
  }
  return lo;
}

typedef struct {
  const void *x; int xdt; const void *y; int ydt; int64_t n, nb; int m4;
  int64_t b0, b1;
  int64_t *edges, *sel, *cnt;
} par_job;

/* Edge b as oracle_edges_x / oracle_edges_nox define it (the first index at
 * or above the edge value), found by bisection instead of the sweep. */
static int64_t par_edge(const par_job *J, int64_t b) {
  if (!J->x) {
    i128 num = (i128)b * (i128)(J->n - 1);
    i128 q = num / J->nb;
    if (q * J->nb < num) q += 1;
    return (int64_t)q;
  }
  if (dtype_class(J->xdt) != CLS_FLOAT) {
    i128 x0 = int_x(J->x, J->xdt, 0), R = int_x(J->x, J->xdt, J->n - 1) - x0;
    return lower_bound_int(J->x, J->xdt, J->n, int_edge_value(x0, R, b, J->nb));
  }
  double x0 = load(J->x, J->xdt, 0).f, R = load(J->x, J->xdt, J->n - 1).f - x0;
  return lower_bound_flt(J->x, J->xdt, J->n, x0 + ((double)b * R) / (double)J->nb);
}

static void *par_edges(void *arg) {
  par_job *J = (par_job *)arg;
  for (int64_t b = J->b0; b < J->b1; b++) J->edges[b] = par_edge(J, b);
  return NULL;
}

static void *par_bins(void *arg) {
  par_job *J = (par_job *)arg;
  for (int64_t b = J->b0; b < J->b1; b++) {
    int64_t lo = J->edges[b], hi = J->edges[b + 1];
    J->cnt[b] = 0;
    if (lo >= hi) continue;
    int64_t v[4];
    int k = 0;
    if (J->m4) v[k++] = lo;
    oracle_argminmax(J->y, J->ydt, lo, hi, &v[k], &v[k + 1]);
    k += 2;
    if (J->m4) v[k++] = hi - 1;
    J->cnt[b] = emit_sorted_distinct(v, k, J->sel + 4 * b);
  }
  return NULL;
}

/* MinMax (m4 = 0) or M4 (m4 = 1) over `threads` threads; same arguments and
 * result as oracle_minmax / oracle_m4. */
int oracle_binned_parallel(const void *x, int xdt, const void *y, int ydt, int64_t n, int64_t n_out, int m4,
                           int threads, int64_t *out, int64_t *count) {
  if (!y || !out || !count || !dtype_valid(ydt) || n < 0 || threads < 1 || threads > 1024) return -1;
  const int64_t per = m4 ? 4 : 2;
  if (n_out < per || n_out % per) return -1;
  if (x && (xdt == OR_I8 || xdt == OR_I16 || xdt == OR_U8 || xdt == OR_U16 || xdt == OR_F16 ||
            !dtype_valid(xdt)))
    return -2;
  if (n <= n_out) { *count = emit_all(n, out); return 0; }
  const int64_t nb = n_out / per;
  int64_t *edges = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb + 1));
  int64_t *sel = (int64_t *)malloc(sizeof(int64_t) * 4 * (size_t)nb);
  int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
  par_job *jobs = (par_job *)malloc(sizeof(par_job) * (size_t)threads);
  pthread_t *tid = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
  int rc = 0;
  if (!edges || !sel || !cnt || !jobs || !tid) { rc = -3; goto done; }
  edges[nb] = n;
  for (int phase = 0; phase < 2; phase++) {
    int started = 0;
    for (int t = 0; t < threads; t++) {
      par_job *J = &jobs[t];
      J->x = x; J->xdt = xdt; J->y = y; J->ydt = ydt; J->n = n; J->nb = nb; J->m4 = m4;
      J->b0 = (int64_t)(((i128)nb * t) / threads);
      J->b1 = (int64_t)(((i128)nb * (t + 1)) / threads);
      J->edges = edges; J->sel = sel; J->cnt = cnt;
      if (pthread_create(&tid[t], NULL, phase == 0 ? par_edges : par_bins, J) != 0) { rc = -3; break; }
      started++;
    }
    for (int t = 0; t < started; t++) pthread_join(tid[t], NULL);
    if (rc) goto done;
  }
  int64_t m = 0;
  for (int64_t b = 0; b < nb; b++)
    for (int64_t j = 0; j < cnt[b]; j++) out[m++] = sel[4 * b + j];
  *count = m;
done:
  free(edges); free(sel); free(cnt); free(jobs); free(tid);
  return rc;
}

/* ------------------------------------------------------------------ */
/* NaN-aware MinMax and M4.  The paper only remarks that floats need a   */
/* different initial value once NaN is handled (Sec. 2.1, Listing 1);   */
/* the reading here: NaN values are passed over, and a bin holding only  */
/* NaN keeps its first index as both argmin and argmax.                  */
/* ------------------------------------------------------------------ */

static int is_nan(oval v) { return v.cls == CLS_FLOAT && v.f != v.f; }

/* Scan y[lo..hi) in index order; the first non-NaN value starts both running
 * extremes and later ones replace them only when strictly smaller (larger).
 * With no non-NaN value both results are lo.  Requires lo < hi. */
int oracle_nan_argminmax(const void *y, int ydt, int64_t lo, int64_t hi,
                         int64_t *imin, int64_t *imax) {
  if (!y || !imin || !imax || !dtype_valid(ydt) || lo < 0 || hi <= lo) return -1;
  int64_t amin = -1, amax = -1;
  oval vmin, vmax;
  for (int64_t i = lo; i < hi; i++) {
    oval v = load(y, ydt, i);
    if (is_nan(v)) continue;
    if (amin < 0 || less(v, vmin)) { vmin = v; amin = i; }
    if (amax < 0 || greater(v, vmax)) { vmax = v; amax = i; }
  }
  *imin = amin < 0 ? lo : amin;
  *imax = amax < 0 ? lo : amax;
  return 0;
}

/* The MinMax (m4 = 0) or M4 (m4 = 1) selection over the same bins as
 * oracle_minmax / oracle_m4, per bin with oracle_nan_argminmax. */
static int nan_binned(const void *x, int xdt, const void *y, int ydt, int64_t n,
                      int64_t n_out, int m4, int64_t *out, int64_t *count) {
  if (!y || !out || !count || !dtype_valid(ydt) || n < 0) return -1;
  const int64_t per = m4 ? 4 : 2;
  if (n_out < per || n_out % per) return -1;
  if (n <= n_out) { *count = emit_all(n, out); return 0; }
  int64_t nb = n_out / per;
  int64_t *edges = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb + 1));
  if (!edges) return -3;
  int rc = make_edges(x, xdt, n, nb, edges);
  if (rc) { free(edges); return rc; }
  int64_t m = 0;
  for (int64_t b = 0; b < nb; b++) {
    if (edges[b] >= edges[b + 1]) continue;
    int64_t v[4];
    int k = 0;
    if (m4) v[k++] = edges[b];
    oracle_nan_argminmax(y, ydt, edges[b], edges[b + 1], &v[k], &v[k + 1]);
    k += 2;
    if (m4) v[k++] = edges[b + 1] - 1;
    m += emit_sorted_distinct(v, k, out + m);
  }
  free(edges);
  *count = m;
  return 0;
}

int oracle_nan_minmax(const void *x, int xdt, const void *y, int ydt, int64_t n,
                      int64_t n_out, int64_t *out, int64_t *count) {
  return nan_binned(x, xdt, y, ydt, n, n_out, 0, out, count);
}

int oracle_nan_m4(const void *x, int xdt, const void *y, int ydt, int64_t n,
                  int64_t n_out, int64_t *out, int64_t *count) {
  return nan_binned(x, xdt, y, ydt, n, n_out, 1, out, count);
}

/* ------------------------------------------------------------------ */
/* LTTB (Steinarsson 2013, cited by the paper as the algorithm whose     */
/* bucket walk cannot be parallelised; Sec. 4).                         */
/* ------------------------------------------------------------------ */

/* The LTTB points are P_j = (X_j, Y_j), j = 0..m-1, taken through an optional
 * index list `sel` (MinMaxLTTB's candidates): source index s_j = sel ? sel[j] : j.
 * X_j = s_j when there is no x, else x[s_j]; Y_j = y[s_j]. */
typedef struct {
  const void *x; int xdt;
  const void *y; int ydt;
  const int64_t *sel;
} points;

static int64_t src_index(const points *P, int64_t j) { return P->sel ? P->sel[j] : j; }

static double X_of(const points *P, int64_t j) {
  int64_t s = src_index(P, j);
  return P->x ? as_double(load(P->x, P->xdt, s)) : (double)s;
}

static double Y_of(const points *P, int64_t j) {
  return as_double(load(P->y, P->ydt, src_index(P, j)));
}

/* Mean over points j in [lo, hi) of X (which = 0) or Y (which = 1).
 * Integer-valued coordinates (the index, integer x, integer y) are summed
 * exactly in 128-bit integers and the sum is rounded once; float coordinates
 * are widened to double and summed in index order.  Then sum / count. */
static double mean_of(const points *P, int which, int64_t lo, int64_t hi) {
  const void *p = which == 0 ? P->x : P->y;
  int dt = which == 0 ? P->xdt : P->ydt;
  double cnt = (double)(hi - lo);
  if (which == 0 && !p) {
    i128 s = 0;
    for (int64_t j = lo; j < hi; j++) s += src_index(P, j);
    return (double)s / cnt;
  }
  if (dtype_class(dt) != CLS_FLOAT) {
    i128 s = 0;
    for (int64_t j = lo; j < hi; j++) s += int_x(p, dt, src_index(P, j));
    return (double)s / cnt;
  }
  double s = 0.0;
  for (int64_t j = lo; j < hi; j++) s += load(p, dt, src_index(P, j)).f;
  return s / cnt;
}

/* Interior bucket k of nb covers points [1 + floor(k (m-2) / nb),
 * 1 + floor((k+1) (m-2) / nb)); the first and last point stand alone. */
static int64_t bucket_start(int64_t k, int64_t m, int64_t nb) {
  return 1 + (int64_t)(((i128)k * (i128)(m - 2)) / nb);
}

/* Doubled triangle area of anchor A, candidate b and next-bucket centre C,
 * evaluated exactly in this order with no fused multiply-add:
 *   | (XA - Cx) * (Yb - YA) - (XA - Xb) * (Cy - YA) |                   */
double oracle_lttb_area2(double XA, double YA, double Xb, double Yb, double Cx, double Cy) {
  return fabs((XA - Cx) * (Yb - YA) - (XA - Xb) * (Cy - YA));
}

/* One LTTB step: among points [lo, hi) pick the first b with the largest
 * doubled area against anchor A and centre (cx, cy). */
static int64_t lttb_pick(const points *P, int64_t lo, int64_t hi, int64_t A,
                         double cx, double cy, double *best_area) {
  double XA = X_of(P, A), YA = Y_of(P, A);
  double best = -1.0;
  int64_t arg = lo;
  for (int64_t b = lo; b < hi; b++) {
    double a = oracle_lttb_area2(XA, YA, X_of(P, b), Y_of(P, b), cx, cy);
    if (a > best) { best = a; arg = b; }
  }
  if (best_area) *best_area = best;
  return arg;
}

/* Centre C_k used while choosing in interior bucket k: the mean of bucket k+1,
 * or the last point itself for the last bucket. */
static void lttb_centre(const points *P, int64_t k, int64_t m, int64_t nb, double *cx, double *cy) {
  if (k == nb - 1) {
    *cx = X_of(P, m - 1);
    *cy = Y_of(P, m - 1);
  } else {
    int64_t lo = bucket_start(k + 1, m, nb), hi = bucket_start(k + 2, m, nb);
    *cx = mean_of(P, 0, lo, hi);
    *cy = mean_of(P, 1, lo, hi);
  }
}

static int lttb_points(const points *P, int64_t m, int64_t n_out, int64_t *out, int64_t *count) {
  if (m <= n_out) {
    for (int64_t j = 0; j < m; j++) out[j] = src_index(P, j);
    *count = m;
    return 0;
  }
  int64_t nb = n_out - 2;
  int64_t A = 0;
  out[0] = src_index(P, 0);
  for (int64_t k = 0; k < nb; k++) {
    double cx, cy;
    lttb_centre(P, k, m, nb, &cx, &cy);
    A = lttb_pick(P, bucket_start(k, m, nb), bucket_start(k + 1, m, nb), A, cx, cy, NULL);
    out[k + 1] = src_index(P, A);
  }
  out[n_out - 1] = src_index(P, m - 1);
  *count = n_out;
  return 0;
}

/* LTTB over the whole series: n_out - 2 interior buckets by point count, the
 * first and last point always kept, one pick per bucket (the point forming the
 * largest triangle with the previous pick and the next bucket's mean). */
int oracle_lttb(const void *x, int xdt, const void *y, int ydt, int64_t n,
                int64_t n_out, int64_t *out, int64_t *count) {
  if (!y || !out || !count || !dtype_valid(ydt) || n < 0 || n_out < 3) return -1;
  if (x && !dtype_valid(xdt)) return -2;
  points P = {x, xdt, y, ydt, NULL};
  return lttb_points(&P, n, n_out, out, count);
}

/* MinMaxLTTB (Van Der Donckt et al., cited by the paper): MinMax with
 * n_out * ratio output points over the interior points 1..n-2 (bins over
 * their x-range when x is given), plus the first and last point, form the
 * candidate set; LTTB then runs on the candidates with their original
 * coordinates.  Indices are into the full series. */
int oracle_minmaxlttb(const void *x, int xdt, const void *y, int ydt, int64_t n,
                      int64_t n_out, int64_t ratio, int64_t *out, int64_t *count) {
  if (!y || !out || !count || !dtype_valid(ydt) || n < 0 || n_out < 3 || ratio < 1) return -1;
  if ((n_out * ratio) % 2) return -1;
  if (x && !dtype_valid(xdt)) return -2;
  if (n <= n_out) { *count = emit_all(n, out); return 0; }
  int64_t npre = n_out * ratio;
  int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)(npre + 2));
  if (!cand) return -3;
  int64_t szx = 0, szy = 0;
  switch (ydt) {
    case OR_I8: case OR_U8: szy = 1; break;
    case OR_I16: case OR_U16: case OR_F16: szy = 2; break;
    case OR_I32: case OR_U32: case OR_F32: szy = 4; break;
    default: szy = 8;
  }
  if (x) {
    switch (xdt) {
      case OR_I32: case OR_U32: case OR_F32: szx = 4; break;
      case OR_I64: case OR_U64: case OR_F64: szx = 8; break;
      default: free(cand); return -2;
    }
  }
  int64_t cnt = 0;
  int rc = oracle_minmax(x ? (const char *)x + szx : NULL, xdt, (const char *)y + szy, ydt,
                         n - 2, npre, cand + 1, &cnt);
  if (rc) { free(cand); return rc; }
  cand[0] = 0;
  for (int64_t j = 1; j <= cnt; j++) cand[j] += 1;
  cand[cnt + 1] = n - 1;
  points P = {x, xdt, y, ydt, cand};
  rc = lttb_points(&P, cnt + 2, n_out, out, count);
  free(cand);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Helpers exposed for the step-wise LTTB checker and for the means.    */
/* ------------------------------------------------------------------ */

/* Centres C_k (k = 0..nb-1) for LTTB over m points through `sel` (may be NULL). */
int oracle_lttb_centres(const void *x, int xdt, const void *y, int ydt, const int64_t *sel,
                        int64_t m, int64_t n_out, double *cx, double *cy) {
  if (!y || !cx || !cy || n_out < 3 || m <= n_out) return -1;
  points P = {x, xdt, y, ydt, sel};
  int64_t nb = n_out - 2;
  for (int64_t k = 0; k < nb; k++) lttb_centre(&P, k, m, nb, &cx[k], &cy[k]);
  return 0;
}

/* Step k of LTTB over m points through `sel`, from anchor point j = A (a point
 * position, not a source index): writes the oracle's pick (point position),
 * its doubled area, and the doubled area of `other` (a point position in the
 * same bucket) against the same anchor and centre. */
int oracle_lttb_step(const void *x, int xdt, const void *y, int ydt, const int64_t *sel,
                     int64_t m, int64_t n_out, int64_t k, int64_t A, int64_t other,
                     int64_t *pick, double *pick_area, double *other_area) {
  if (!y || n_out < 3 || m <= n_out || k < 0 || k >= n_out - 2) return -1;
  points P = {x, xdt, y, ydt, sel};
  int64_t nb = n_out - 2;
  double cx, cy;
  lttb_centre(&P, k, m, nb, &cx, &cy);
  int64_t lo = bucket_start(k, m, nb), hi = bucket_start(k + 1, m, nb);
  *pick = lttb_pick(&P, lo, hi, A, cx, cy, pick_area);
  if (other_area) {
    if (other < lo || other >= hi) return -4;
    *other_area = oracle_lttb_area2(X_of(&P, A), Y_of(&P, A), X_of(&P, other), Y_of(&P, other), cx, cy);
  }
  return 0;
}

/* Candidate set of MinMaxLTTB (first point, interior MinMax preselection,
 * last point); returns its size in *count.  cand must hold n_out*ratio + 2. */
int oracle_minmaxlttb_candidates(const void *x, int xdt, const void *y, int ydt, int64_t n,
                                 int64_t n_out, int64_t ratio, int64_t *cand, int64_t *count) {
  if (!y || !cand || !count || n <= n_out || n_out < 3 || ratio < 1 || (n_out * ratio) % 2)
    return -1;
  int64_t szy, szx = 0;
  switch (ydt) {
    case OR_I8: case OR_U8: szy = 1; break;
    case OR_I16: case OR_U16: case OR_F16: szy = 2; break;
    case OR_I32: case OR_U32: case OR_F32: szy = 4; break;
    default: szy = 8;
  }
  if (x) szx = (xdt == OR_I32 || xdt == OR_U32 || xdt == OR_F32) ? 4 : 8;
  int64_t cnt = 0;
  int rc = oracle_minmax(x ? (const char *)x + szx : NULL, xdt, (const char *)y + szy, ydt,
                         n - 2, n_out * ratio, cand + 1, &cnt);
  if (rc) return rc;
  cand[0] = 0;
  for (int64_t j = 1; j <= cnt; j++) cand[j] += 1;
  cand[cnt + 1] = n - 1;
  *count = cnt + 2;
  return 0;
}

/* Zoom window (serving): the points with xa <= x <= xb, i.e. [i0, i1) with
 * i0 = left search-sorted of xa and i1 = right search-sorted of xb.  Integer
 * x only (the resident series carry int64 timestamps). */
int oracle_window(const void *x, int xdt, int64_t n, int64_t xa, int64_t xb,
                  int64_t *i0, int64_t *i1) {
  if (!x || !i0 || !i1 || n < 0 || dtype_class(xdt) == CLS_FLOAT) return -1;
  int64_t lo = 0, hi = n;                 /* first index with x >= xa */
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (int_x(x, xdt, mid) < (i128)xa) lo = mid + 1; else hi = mid;
  }
  *i0 = lo;
  lo = 0; hi = n;                         /* first index with x > xb */
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (int_x(x, xdt, mid) <= (i128)xb) lo = mid + 1; else hi = mid;
  }
  *i1 = lo;
  return 0;
}

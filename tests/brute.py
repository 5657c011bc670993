"""Brute-force pins for the oracle, written independently of it.

Each function states the operation from its definition in a different form
than the oracle uses (per-point bin ids instead of edge searches, numpy's
argmin/argmax instead of a running scan, exact rational arithmetic for LTTB
areas), so that a slip in the oracle's arithmetic shows up as a mismatch.
Tiny inputs only.
"""
from fractions import Fraction

import numpy as np


def bin_ids_nox(n, nb):
    """Equally sampled series = x = 0..n-1 binned into nb equal-width bins
    over [0, n-1]: point i lies in bin floor(i*nb/(n-1)), the last point in
    the last bin (Sec. 2.2 / 2.3: no x is the same as an equally sampled x)."""
    if n == 1:
        return np.zeros(1, np.int64)
    return np.array([min(i * nb // (n - 1), nb - 1) for i in range(n)], np.int64)


def bin_ids_int_x(x, nb):
    """Integer x: nb bins of equal width R/nb over [x0, x_last]; point i lies
    in bin floor((x_i - x0) * nb / R) (clamped to nb-1); R = 0 puts every point
    in the last bin."""
    x0, xl = int(x[0]), int(x[-1])
    R = xl - x0
    if R == 0:
        return np.full(len(x), nb - 1, np.int64)
    return np.array([min((int(v) - x0) * nb // R, nb - 1) for v in x], np.int64)


def per_bin(y, ids, nb, kind):
    """Concatenate, bin by bin, the sorted distinct selected indices."""
    out = []
    for b in range(nb):
        idx = np.nonzero(ids == b)[0]
        if len(idx) == 0:
            continue
        seg = y[idx[0]: idx[-1] + 1]
        assert len(seg) == len(idx), "bins must be contiguous"
        amin = idx[0] + int(np.argmin(seg))
        amax = idx[0] + int(np.argmax(seg))
        pick = {amin, amax}
        if kind == "m4":
            pick |= {int(idx[0]), int(idx[-1])}
        out.extend(sorted(pick))
    return np.array(out, np.int64)


def per_bin_nan(y, ids, nb, kind):
    """per_bin with NaN ignored: numpy's argmin / argmax over the bin's
    non-NaN values only (first occurrence), mapped back to their positions
    (numpy's nanargmin / nanargmax would not do: they stand NaN in for +-inf,
    so a NaN can tie with an infinity); a bin of NaN only gives its first
    index for both."""
    out = []
    for b in range(nb):
        idx = np.nonzero(ids == b)[0]
        if len(idx) == 0:
            continue
        seg = y[idx[0]: idx[-1] + 1].astype(np.float64)
        if np.isnan(seg).all():
            pick = {int(idx[0])}
        else:
            keep = np.nonzero(~np.isnan(seg))[0]
            vals = seg[keep]
            pick = {idx[0] + int(keep[np.argmin(vals)]), idx[0] + int(keep[np.argmax(vals)])}
        if kind == "m4":
            pick |= {int(idx[0]), int(idx[-1])}
        out.extend(sorted(pick))
    return np.array(out, np.int64)


def nan_binned(y, n_out, kind, x=None):
    n = len(y)
    if n <= n_out:
        return np.arange(n, dtype=np.int64)
    nb = n_out // (2 if kind == "minmax" else 4)
    ids = bin_ids_nox(n, nb) if x is None else bin_ids_int_x(x, nb)
    return per_bin_nan(y, ids, nb, kind)


def minmax(y, n_out, x=None):
    n = len(y)
    if n <= n_out:
        return np.arange(n, dtype=np.int64)
    nb = n_out // 2
    ids = bin_ids_nox(n, nb) if x is None else bin_ids_int_x(x, nb)
    return per_bin(y, ids, nb, "minmax")


def m4(y, n_out, x=None):
    n = len(y)
    if n <= n_out:
        return np.arange(n, dtype=np.int64)
    nb = n_out // 4
    ids = bin_ids_nox(n, nb) if x is None else bin_ids_int_x(x, nb)
    return per_bin(y, ids, nb, "m4")


def _exact(v):
    if isinstance(v, (np.floating, float)):
        return Fraction(float(v))
    return Fraction(int(v))


def lttb_exact(y, n_out, x=None, rel_tie=1e-9):
    """LTTB with exact rational coordinates, means and areas.  Returns the
    picks and, per step, whether the exact best and second-best areas are
    closer than rel_tie (a near tie, where a double-precision evaluation may
    legitimately choose the other point)."""
    m = len(y)
    if m <= n_out:
        return np.arange(m, dtype=np.int64), []
    X = [Fraction(i) for i in range(m)] if x is None else [_exact(v) for v in x]
    Y = [_exact(v) for v in y]
    nb = n_out - 2
    bounds = [1 + (k * (m - 2)) // nb for k in range(nb + 1)]
    sel = [0]
    near = []
    A = 0
    for k in range(nb):
        if k == nb - 1:
            cx, cy = X[m - 1], Y[m - 1]
        else:
            lo, hi = bounds[k + 1], bounds[k + 2]
            cx = sum(X[lo:hi], Fraction(0)) / (hi - lo)
            cy = sum(Y[lo:hi], Fraction(0)) / (hi - lo)
        areas = []
        for b in range(bounds[k], bounds[k + 1]):
            # twice the triangle area = |cross(P_b - A, C - A)|
            areas.append(abs((X[b] - X[A]) * (cy - Y[A]) - (Y[b] - Y[A]) * (cx - X[A])))
        best = max(areas)
        j = areas.index(best)
        srt = sorted(areas, reverse=True)
        second = srt[1] if len(srt) > 1 else None
        near.append(second is not None and best - second <= Fraction(rel_tie) * best)
        A = bounds[k] + j
        sel.append(A)
    sel.append(m - 1)
    return np.array(sel, np.int64), near

"""CPU oracle for the downsampling hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``tsds_oracle.c`` (plain C,
host arrays, fp64 where floating point is involved) through ctypes and shares
nothing with the GPU library.  See ``tsds_oracle.c`` for the definitions and
the passages of the paper each function follows.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_CODES = {
    np.dtype(np.int8): 0, np.dtype(np.int16): 1, np.dtype(np.int32): 2, np.dtype(np.int64): 3,
    np.dtype(np.uint8): 4, np.dtype(np.uint16): 5, np.dtype(np.uint32): 6, np.dtype(np.uint64): 7,
    np.dtype(np.float16): 8, np.dtype(np.float32): 9, np.dtype(np.float64): 10,
}

_lib = None
_I64P = ctypes.POINTER(ctypes.c_int64)
_F64P = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False, sanitize=_build.sanitize_requested())
        lib = ctypes.CDLL(path)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.oracle_argminmax.argtypes = [vp, i32, i64, i64, _I64P, _I64P]
        lib.oracle_edges_nox.argtypes = [i64, i64, _I64P]
        lib.oracle_edges_x.argtypes = [vp, i32, i64, i64, _I64P]
        lib.oracle_nan_argminmax.argtypes = [vp, i32, i64, i64, _I64P, _I64P]
        for f in (lib.oracle_minmax, lib.oracle_m4, lib.oracle_lttb, lib.oracle_nan_minmax, lib.oracle_nan_m4):
            f.argtypes = [vp, i32, vp, i32, i64, i64, _I64P, _I64P]
        lib.oracle_minmaxlttb.argtypes = [vp, i32, vp, i32, i64, i64, i64, _I64P, _I64P]
        lib.oracle_minmaxlttb_candidates.argtypes = [vp, i32, vp, i32, i64, i64, i64, _I64P, _I64P]
        lib.oracle_lttb_centres.argtypes = [vp, i32, vp, i32, _I64P, i64, i64, _F64P, _F64P]
        lib.oracle_lttb_step.argtypes = [vp, i32, vp, i32, _I64P, i64, i64, i64, i64, i64,
                                         _I64P, _F64P, _F64P]
        lib.oracle_lttb_area2.argtypes = [ctypes.c_double] * 6
        lib.oracle_lttb_area2.restype = ctypes.c_double
        lib.oracle_window.argtypes = [vp, i32, i64, i64, i64, _I64P, _I64P]
        lib.oracle_everynth.argtypes = [i64, i64, _I64P, _I64P]
        lib.oracle_binned_parallel.argtypes = [vp, i32, vp, i32, i64, i64, i32, i32, _I64P, _I64P]
        lib.oracle_binned_parallel.restype = ctypes.c_int
        for f in (lib.oracle_argminmax, lib.oracle_edges_nox, lib.oracle_edges_x, lib.oracle_minmax,
                  lib.oracle_m4, lib.oracle_lttb, lib.oracle_minmaxlttb,
                  lib.oracle_minmaxlttb_candidates, lib.oracle_lttb_centres, lib.oracle_lttb_step,
                  lib.oracle_window, lib.oracle_everynth, lib.oracle_nan_argminmax, lib.oracle_nan_minmax,
                  lib.oracle_nan_m4):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _arr(a):
    a = np.ascontiguousarray(a)
    if a.dtype not in _CODES:
        raise TypeError(f"oracle: unsupported dtype {a.dtype}")
    return a, a.ctypes.data_as(ctypes.c_void_p), _CODES[a.dtype]


def _x(x):
    if x is None:
        return None, None, -1
    return _arr(x)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what}: status {rc}")


def _i64(a):
    return a.ctypes.data_as(_I64P)


def argminmax(y, lo=0, hi=None):
    """First index of the minimum and of the maximum of y[lo:hi]."""
    y, yp, yd = _arr(y)
    hi = len(y) if hi is None else hi
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(_load().oracle_argminmax(yp, yd, lo, hi, ctypes.byref(a), ctypes.byref(b)), "argminmax")
    return a.value, b.value


def edges(n, nb, x=None):
    """Bin starts s_0..s_nb (s_nb = n) for nb bins, with or without x."""
    out = np.empty(nb + 1, np.int64)
    if x is None:
        _check(_load().oracle_edges_nox(n, nb, _i64(out)), "edges")
    else:
        x, xp, xd = _arr(x)
        _check(_load().oracle_edges_x(xp, xd, len(x), nb, _i64(out)), "edges")
    return out


def _run(fn, y, n_out, x, cap, *extra):
    y, yp, yd = _arr(y)
    x, xp, xd = _x(x)
    out = np.empty(max(cap, 1), np.int64)
    cnt = ctypes.c_int64()
    rc = fn(xp, xd, yp, yd, len(y), n_out, *extra, _i64(out), ctypes.byref(cnt))
    _check(rc, fn.__name__)
    return out[: cnt.value].copy()


def everynth(n, n_out):
    """EveryNth over n points: every k-th index, k = ceil(n / n_out)."""
    out = np.empty(max(min(n, n_out), 1), np.int64)
    cnt = ctypes.c_int64()
    _check(_load().oracle_everynth(n, n_out, _i64(out), ctypes.byref(cnt)), "everynth")
    return out[: cnt.value].copy()


def minmax(y, n_out, x=None):
    return _run(_load().oracle_minmax, y, n_out, x, max(n_out, len(y) if len(y) <= n_out else 0))


def m4(y, n_out, x=None):
    return _run(_load().oracle_m4, y, n_out, x, max(n_out, len(y) if len(y) <= n_out else 0))


def nan_minmax(y, n_out, x=None):
    """NaN-aware MinMax: NaN skipped; an all-NaN bin keeps its first index."""
    return _run(_load().oracle_nan_minmax, y, n_out, x, max(n_out, len(y) if len(y) <= n_out else 0))


def nan_m4(y, n_out, x=None):
    """NaN-aware M4: NaN skipped in the argmin/argmax; first and last kept."""
    return _run(_load().oracle_nan_m4, y, n_out, x, max(n_out, len(y) if len(y) <= n_out else 0))


def binned_parallel(algo, y, n_out, x=None, threads=1):
    """MinMax or M4 (algo) with the bins split over `threads` host threads
    (the CPU baseline's all-cores mode); the same result as minmax / m4."""
    if algo not in ("minmax", "m4"):
        raise ValueError(algo)
    y, yp, yd = _arr(y)
    x, xp, xd = _x(x)
    cap = max(n_out, len(y) if len(y) <= n_out else 0)
    out = np.empty(max(cap, 1), np.int64)
    cnt = ctypes.c_int64()
    rc = _load().oracle_binned_parallel(xp, xd, yp, yd, len(y), n_out, 1 if algo == "m4" else 0, int(threads),
                                        _i64(out), ctypes.byref(cnt))
    _check(rc, "binned_parallel")
    return out[: cnt.value].copy()


def lttb(y, n_out, x=None):
    return _run(_load().oracle_lttb, y, n_out, x, max(n_out, len(y) if len(y) <= n_out else 0))


def minmaxlttb(y, n_out, ratio=4, x=None):
    return _run(_load().oracle_minmaxlttb, y, n_out, x,
                max(n_out, len(y) if len(y) <= n_out else 0), ratio)


def minmaxlttb_candidates(y, n_out, ratio=4, x=None):
    y, yp, yd = _arr(y)
    x, xp, xd = _x(x)
    out = np.empty(n_out * ratio + 2, np.int64)
    cnt = ctypes.c_int64()
    _check(_load().oracle_minmaxlttb_candidates(xp, xd, yp, yd, len(y), n_out, ratio, _i64(out),
                                                ctypes.byref(cnt)), "candidates")
    return out[: cnt.value].copy()


def lttb_centres(y, n_out, x=None, sel=None):
    """Centres (mean X, mean Y of the next bucket; the last point for the
    last bucket) used at each of the n_out - 2 LTTB steps."""
    y, yp, yd = _arr(y)
    x, xp, xd = _x(x)
    selp = None
    m = len(y)
    if sel is not None:
        sel = np.ascontiguousarray(sel, np.int64)
        selp = _i64(sel)
        m = len(sel)
    cx = np.empty(n_out - 2, np.float64)
    cy = np.empty(n_out - 2, np.float64)
    _check(_load().oracle_lttb_centres(xp, xd, yp, yd, selp, m, n_out, cx.ctypes.data_as(_F64P),
                                       cy.ctypes.data_as(_F64P)), "centres")
    return cx, cy


def lttb_step(y, n_out, k, anchor, other, x=None, sel=None):
    """Oracle's LTTB step k from point position `anchor`: returns
    (pick, pick_area2, area2 of point position `other`)."""
    y, yp, yd = _arr(y)
    x, xp, xd = _x(x)
    selp = None
    m = len(y)
    if sel is not None:
        sel = np.ascontiguousarray(sel, np.int64)
        selp = _i64(sel)
        m = len(sel)
    pick = ctypes.c_int64()
    pa, oa = ctypes.c_double(), ctypes.c_double()
    _check(_load().oracle_lttb_step(xp, xd, yp, yd, selp, m, n_out, k, anchor, other,
                                    ctypes.byref(pick), ctypes.byref(pa), ctypes.byref(oa)), "step")
    return pick.value, pa.value, oa.value


def lttb_area2(XA, YA, Xb, Yb, Cx, Cy):
    return _load().oracle_lttb_area2(XA, YA, Xb, Yb, Cx, Cy)


def window(x, xa, xb):
    """[i0, i1) of the points with xa <= x <= xb (integer x)."""
    x, xp, xd = _arr(x)
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(_load().oracle_window(xp, xd, len(x), int(xa), int(xb), ctypes.byref(a), ctypes.byref(b)),
           "window")
    return a.value, b.value

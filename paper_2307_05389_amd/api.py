"""Torch-facing wrappers over the C ABI (marshalling only)."""
import ctypes

import torch

from . import _lib as L


def workspace_bytes(algo, y, n_out, x=None, minmax_ratio=4):
    s = L.series(y, x)
    return int(L.lib().ts_workspace_bytes(L.ALGO[algo], ctypes.byref(s), n_out, minmax_ratio))


def downsample_into(algo, y, n_out, out, count, x=None, minmax_ratio=4, workspace=None, stream=None):
    """Enqueue one downsampling call; `out` (int64, >= n_out) and `count`
    (int64, 1 element) are device tensors the caller owns.  No host sync."""
    s = L.series(y, x)
    lib = L.lib()
    st = stream if stream is not None else torch.cuda.current_stream(y.device)
    need = int(lib.ts_workspace_bytes(L.ALGO[algo], ctypes.byref(s), n_out, minmax_ratio))
    if workspace is None:
        workspace = L.WS.get(need, y.device, st)
    wsp = ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else ctypes.c_void_p(None)
    wsb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    if out.numel() < min(n_out, y.numel()) or out.dtype != torch.int64 or count.dtype != torch.int64:
        raise ValueError("out must hold n_out int64 values and count one int64")
    sp = ctypes.c_void_p(st.cuda_stream)
    if algo == "minmaxlttb":
        rc = lib.ts_minmaxlttb(ctypes.byref(s), n_out, minmax_ratio, L._ptr(out), L._ptr(count), wsp, wsb, sp)
    else:
        f = {"minmax": lib.ts_minmax, "m4": lib.ts_m4, "lttb": lib.ts_lttb, "nan_minmax": lib.ts_nan_minmax,
             "nan_m4": lib.ts_nan_m4}[algo]
        rc = f(ctypes.byref(s), n_out, L._ptr(out), L._ptr(count), wsp, wsb, sp)
    L.check(rc)
    return out, count


def minmaxlttb_noalloc(y, n_out, out, count, x=None, minmax_ratio=4, stream=None):
    """ts_minmaxlttb_noalloc: MinMaxLTTB into the caller's `out` (int64,
    >= n_out) and `count` (int64, 1 element) over the library's static
    device scratch; neither this wrapper nor the library allocates device
    memory.  Calls overlapping on one GPU share that scratch and must be
    serialised by the caller."""
    s = L.series(y, x)
    if out.numel() < min(n_out, y.numel()) or out.dtype != torch.int64 or count.dtype != torch.int64:
        raise ValueError("out must hold n_out int64 values and count one int64")
    st = stream if stream is not None else torch.cuda.current_stream(y.device)
    L.check(L.lib().ts_minmaxlttb_noalloc(ctypes.byref(s), n_out, minmax_ratio, L._ptr(out), L._ptr(count),
                                          ctypes.c_void_p(st.cuda_stream)))
    return out, count


def _run(algo, y, n_out, x, minmax_ratio):
    out = torch.empty(max(n_out, 1), dtype=torch.int64, device=y.device)
    count = torch.zeros(1, dtype=torch.int64, device=y.device)
    downsample_into(algo, y, n_out, out, count, x=x, minmax_ratio=minmax_ratio)
    return out[: int(count.item())]


def minmax(y, n_out, x=None):
    """MinMax: per bin the first argmin and first argmax (n_out/2 bins)."""
    return _run("minmax", y, n_out, x, 0)


def m4(y, n_out, x=None):
    """M4: per bin the first, argmin, argmax and last index (n_out/4 bins)."""
    return _run("m4", y, n_out, x, 0)


def nan_minmax(y, n_out, x=None):
    """NaN-aware MinMax: NaN values skipped; an all-NaN bin keeps its first index."""
    return _run("nan_minmax", y, n_out, x, 0)


def nan_m4(y, n_out, x=None):
    """NaN-aware M4: NaN values skipped in the argmin/argmax; first and last kept."""
    return _run("nan_m4", y, n_out, x, 0)


def lttb(y, n_out, x=None):
    """LTTB: largest-triangle-three-buckets over all points."""
    return _run("lttb", y, n_out, x, 0)


def minmaxlttb(y, n_out, x=None, minmax_ratio=4):
    """MinMaxLTTB: MinMax preselection of n_out*minmax_ratio interior points,
    then LTTB over them and the two end points."""
    return _run("minmaxlttb", y, n_out, x, minmax_ratio)


def everynth(y, n_out, x=None):
    """EveryNth: indices 0, k, 2k, ... below len(y), k = ceil(len(y) / n_out)."""
    s = L.series(y, x)
    out = torch.empty(max(min(n_out, y.numel()), 1), dtype=torch.int64, device=y.device)
    count = torch.zeros(1, dtype=torch.int64, device=y.device)
    L.check(L.lib().ts_everynth(ctypes.byref(s), n_out, L._ptr(out), L._ptr(count),
                                L.stream_ptr(device=y.device)))
    return out[: int(count.item())]


def gather(y, idx, x=None, count=None):
    """The selected points: y[idx] (and x[idx] when x is given), gathered in
    one kernel.  idx: device int64; count: optional device int64[1] giving
    how many of idx to take (read on the device).  Returns y_sel, or
    (x_sel, y_sel) when x is given."""
    s = L.series(y, x)
    if idx.dtype != torch.int64 or idx.device != y.device or idx.dim() != 1 or not idx.is_contiguous():
        raise ValueError("idx must be a contiguous 1-D int64 tensor on y's device")
    cap = idx.numel()
    if count is None:
        count = torch.full((1,), cap, dtype=torch.int64, device=y.device)
    ys = torch.empty(cap, dtype=y.dtype, device=y.device)
    xs = torch.empty(cap, dtype=x.dtype, device=y.device) if x is not None else None
    if cap:
        L.check(L.lib().ts_gather(ctypes.byref(s), L._ptr(idx), L._ptr(count), cap, L._ptr(xs), L._ptr(ys),
                                  L.stream_ptr(device=y.device)))
    return ys if x is None else (xs, ys)


def bin_edges(y, nb, x=None):
    """Bin starts edges[0..nb] (edges[nb] = n) used by MinMax / M4."""
    s = L.series(y, x)
    edges = torch.empty(nb + 1, dtype=torch.int64, device=y.device)
    L.check(L.lib().ts_bin_edges(ctypes.byref(s), nb, L._ptr(edges), L.stream_ptr(device=y.device)))
    return edges


def bin_argminmax(y, edges):
    """Per-bin first argmin / argmax (-1 for empty bins) over caller edges."""
    s = L.series(y)
    nb = edges.numel() - 1
    lib = L.lib()
    need = int(lib.ts_argminmax_workspace_bytes(ctypes.byref(s), nb))
    st = torch.cuda.current_stream(y.device)
    ws = L.WS.get(need, y.device, st)
    imin = torch.empty(nb, dtype=torch.int64, device=y.device)
    imax = torch.empty(nb, dtype=torch.int64, device=y.device)
    L.check(lib.ts_bin_argminmax(ctypes.byref(s), L._ptr(edges), nb, L._ptr(imin), L._ptr(imax),
                                 L._ptr(ws), ws.numel() if ws is not None else 0,
                                 ctypes.c_void_p(st.cuda_stream)))
    return imin, imax


def lttb_centres(y, n_out, x=None, sel=None):
    """LTTB centres (mean x, mean y of the next bucket; the last point for
    the last bucket) for the points y (or y[sel])."""
    s = L.series(y, x)
    m = y.numel() if sel is None else sel.numel()
    cx = torch.empty(n_out - 2, dtype=torch.float64, device=y.device)
    cy = torch.empty(n_out - 2, dtype=torch.float64, device=y.device)
    L.check(L.lib().ts_lttb_centres(ctypes.byref(s), L._ptr(sel), m, n_out, L._ptr(cx), L._ptr(cy),
                                    L.stream_ptr(device=y.device)))
    return cx, cy


def window(x, xa, xb, y=None):
    """[i0, i1) of the points with xa <= x <= xb (integer x)."""
    yy = y if y is not None else x
    s = L.series(yy, x)
    r = torch.empty(2, dtype=torch.int64, device=x.device)
    L.check(L.lib().ts_window(ctypes.byref(s), int(xa), int(xb), L._ptr(r), L.stream_ptr(device=x.device)))
    return r


def set_tuning(chunk_bytes=-1, small_bin=-1, scan_variant=-1, stage=-1, xclass=-1, direct=-1):
    """Override the scan's chunk size (power of two >= 4096 bytes), the
    segment length below which one lane handles a whole bin, the tile shape
    variant, LDS staging, the classification of chunks from int64 x and the
    per-bin paths (direct: 0 = chunks, 1 = a wavefront per bin, 2 = a
    workgroup of four wavefronts per bin); -1 restores the defaults.  Results
    do not depend on them."""
    L.check(L.lib().ts_set_tuning(int(chunk_bytes), int(small_bin), int(scan_variant), int(stage), int(xclass),
                                  int(direct)))

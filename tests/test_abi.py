"""CPU-side checks of the C ABI: the library loads, exports every function
that include/tsds.h declares, and rejects bad arguments before it touches the
GPU (validation is host logic; no kernel is launched in these tests)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsds.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ts_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2307_05389_amd import _lib
    return _lib.lib()


def test_header_declares_the_paths_entry_points():
    names = _declared()
    for f in ("ts_minmax", "ts_m4", "ts_lttb", "ts_minmaxlttb", "ts_workspace_bytes", "ts_bin_edges",
              "ts_bin_argminmax", "ts_lttb_centres", "ts_window", "ts_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name


def _series(n, ydt=9, y=0x1000, x=None, xdt=-1):
    from paper_2307_05389_amd._lib import TsSeries
    return TsSeries(x, xdt, y, ydt, n)


def test_workspace_bytes_host_logic(L):
    s = _series(10**8, ydt=10, x=0x2000, xdt=3)
    ws = L.ts_workspace_bytes(1, ctypes.byref(s), 4000, 0)
    assert ws > 0 and ws % 256 == 0
    assert L.ts_workspace_bytes(1, ctypes.byref(s), 4001, 0) == 0       # M4 needs n_out % 4 == 0
    assert L.ts_workspace_bytes(0, ctypes.byref(_series(100)), 1000, 0) == 0  # n <= n_out
    assert L.ts_workspace_bytes(3, ctypes.byref(_series(10**7)), 1000, 4) > 0
    assert L.ts_workspace_bytes(3, ctypes.byref(_series(10**7)), 1001, 1) == 0  # odd n_out*ratio
    # NaN-aware MinMax / M4 (algos 4, 5): same n_out rules, their own chunking
    for algo, ok, bad in ((4, 1000, 1001), (5, 4000, 4002)):
        w = L.ts_workspace_bytes(algo, ctypes.byref(_series(10**8, ydt=10)), ok, 0)
        assert w > 0 and w % 256 == 0
        assert L.ts_workspace_bytes(algo, ctypes.byref(_series(10**8, ydt=10)), bad, 0) == 0


@pytest.mark.parametrize("call,code", [
    ("minmax_odd", -1), ("m4_bad", -1), ("lttb_small", -1), ("ratio0", -1), ("bad_dtype", -2),
    ("x_mismatch", -3), ("null_out", -3), ("misaligned", -6), ("no_ws", -4), ("neg_n", -1),
    ("everynth_n_out0", -1), ("everynth_null_out", -3), ("gather_x_out_no_x", -3),
    ("gather_misaligned", -6), ("gather_neg_cap", -1), ("gather_null_idx", -3),
])
def test_validation_errors_without_launch(L, call, code):
    out = ctypes.c_void_p(0x10000)
    cnt = ctypes.c_void_p(0x20000)
    ws = ctypes.c_void_p(0x100000)
    s = _series(10**6)
    args = None
    if call == "minmax_odd":
        rc = L.ts_minmax(ctypes.byref(s), 1001, out, cnt, ws, 1 << 30, None)
    elif call == "m4_bad":
        rc = L.ts_m4(ctypes.byref(s), 1002, out, cnt, ws, 1 << 30, None)
    elif call == "lttb_small":
        rc = L.ts_lttb(ctypes.byref(s), 2, out, cnt, ws, 1 << 30, None)
    elif call == "ratio0":
        rc = L.ts_minmaxlttb(ctypes.byref(s), 1000, 0, out, cnt, ws, 1 << 30, None)
    elif call == "bad_dtype":
        rc = L.ts_minmax(ctypes.byref(_series(10**6, ydt=11)), 1000, out, cnt, ws, 1 << 30, None)
    elif call == "x_mismatch":
        rc = L.ts_minmax(ctypes.byref(_series(10**6, x=0x3000, xdt=-1)), 1000, out, cnt, ws, 1 << 30, None)
    elif call == "null_out":
        rc = L.ts_minmax(ctypes.byref(s), 1000, None, cnt, ws, 1 << 30, None)
    elif call == "misaligned":
        rc = L.ts_minmax(ctypes.byref(_series(10**6, y=0x1001)), 1000, out, cnt, ws, 1 << 30, None)
    elif call == "no_ws":
        rc = L.ts_minmax(ctypes.byref(s), 1000, out, cnt, ws, 16, None)
    elif call == "neg_n":
        rc = L.ts_minmax(ctypes.byref(_series(-5)), 1000, out, cnt, ws, 1 << 30, None)
    elif call == "everynth_n_out0":
        rc = L.ts_everynth(ctypes.byref(s), 0, out, cnt, None)
    elif call == "everynth_null_out":
        rc = L.ts_everynth(ctypes.byref(s), 10, None, cnt, None)
    elif call == "gather_x_out_no_x":
        rc = L.ts_gather(ctypes.byref(s), out, cnt, 10, ctypes.c_void_p(0x30000), ctypes.c_void_p(0x40000), None)
    elif call == "gather_misaligned":
        rc = L.ts_gather(ctypes.byref(s), out, cnt, 10, None, ctypes.c_void_p(0x40002), None)
    elif call == "gather_neg_cap":
        rc = L.ts_gather(ctypes.byref(s), out, cnt, -1, None, ctypes.c_void_p(0x40000), None)
    elif call == "gather_null_idx":
        rc = L.ts_gather(ctypes.byref(s), None, cnt, 10, None, ctypes.c_void_p(0x40000), None)
    assert rc == code, (call, rc, L.ts_last_error())
    assert L.ts_last_error()


def test_noalloc_rejects_before_touching_the_gpu(L):
    """ts_minmaxlttb_noalloc: the static scratch holds 64 MiB; a series whose
    workspace exceeds it, and invalid arguments, are rejected on the host
    (no device is needed to get these codes)."""
    assert L.ts_noalloc_scratch_bytes() == 64 << 20
    out, cnt = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000)
    big = _series(10**10)
    assert L.ts_workspace_bytes(3, ctypes.byref(big), 2000, 4) > L.ts_noalloc_scratch_bytes()
    assert L.ts_minmaxlttb_noalloc(ctypes.byref(big), 2000, 4, out, cnt, None) == -4
    assert b"scratch" in L.ts_last_error()
    s = _series(10**6)
    assert L.ts_minmaxlttb_noalloc(ctypes.byref(s), 1000, 0, out, cnt, None) == -1       # ratio 0
    assert L.ts_minmaxlttb_noalloc(ctypes.byref(s), 1001, 1, out, cnt, None) == -1       # odd n_out * ratio
    assert L.ts_minmaxlttb_noalloc(ctypes.byref(s), 1000, 4, None, cnt, None) == -3      # no output
    assert L.ts_minmaxlttb_noalloc(ctypes.byref(_series(10**6, y=0x1001)), 1000, 4, out, cnt, None) == -6


def test_no_cpu_fallback_in_product_package():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2307_05389_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".cpp", ".hip", ".hpp")):
                txt = open(os.path.join(dp, f)).read()
                assert "oracle" not in txt.replace("the oracle", ""), f


def test_downsampler_argument_parsing_before_any_device_work():
    import numpy as np
    import paper_2307_05389_amd as t
    y = np.zeros(10, np.float32)
    with pytest.raises(TypeError):
        t.MinMaxDownsampler().downsample(y)                      # no n_out
    with pytest.raises(TypeError):
        t.M4Downsampler().downsample(y, n_out=8, minmax_ratio=2)  # MinMaxLTTB-only keyword
    with pytest.raises(TypeError):
        t.LTTBDownsampler().downsample(y, y, y, 4)               # too many arrays


def test_per_bin_mode_host_logic():
    """Which kernel reduces the bins (host logic, no launch): a wavefront per
    bin for many few-kilobyte bins, a workgroup per bin for 500-1,999 long
    bins (eight-byte types from 250), chunks otherwise; the forced modes fall
    back where their grid would exceed 2^31 threads."""
    import torch
    from paper_2307_05389_amd import _lib
    from paper_2307_05389_amd.api import set_tuning
    sc = lambda *a, **k: _lib.scan_config(*a, **k)[2]
    n = 1 << 28                                                          # 1 GB of f32
    assert sc(torch.float32, n, 1000).startswith("tsds::k_bins_block<")      # 1 MB bins
    assert sc(torch.float32, n, 100000).startswith("tsds::k_bins_direct<")   # 10 KB bins
    assert not sc(torch.float32, n, 250).startswith("tsds::k_bins")         # 4 MB bins: chunks
    assert sc(torch.float64, n // 2, 250).startswith("tsds::k_bins_block<")
    assert not sc(torch.float32, n, 1000, x_dtype=torch.int64).startswith("tsds::k_bins")  # with x: chunks
    try:
        set_tuning(direct=2)
        assert sc(torch.float32, n, 1 << 23).startswith("tsds::k_bins_block<")
        assert sc(torch.float32, n, (1 << 23) + 1).startswith("tsds::k_bins_direct<")
        assert not sc(torch.float32, 1 << 30, (1 << 25) + 1).startswith("tsds::k_bins")
        with pytest.raises(Exception):
            set_tuning(direct=3)
    finally:
        set_tuning()

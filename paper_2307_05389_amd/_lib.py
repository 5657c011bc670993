"""ctypes binding of libtsds.so (argument marshalling only).

Every step of the downsampling path runs in the library's HIP kernels; this
module only turns torch tensors into device pointers, sizes workspaces and
maps status codes to exceptions.  It refuses to work without the compiled
library: there is no CPU fallback.
"""
import ctypes
import os

import torch

# TSDS_SANITIZE=1 selects the build with ASan/UBSan on the host code (CPU
# test runs; needs the sanitizer runtime preloaded)
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "libtsds_san.so" if os.environ.get("TSDS_SANITIZE", "") == "1" else "libtsds.so")

TS_NONE = -1
DTYPE_CODES = {
    torch.int8: 0, torch.int16: 1, torch.int32: 2, torch.int64: 3,
    torch.uint8: 4, torch.uint16: 5, torch.uint32: 6, torch.uint64: 7,
    torch.float16: 8, torch.float32: 9, torch.float64: 10,
}
ALGO = {"minmax": 0, "m4": 1, "lttb": 2, "minmaxlttb": 3, "nan_minmax": 4, "nan_m4": 5}
ERRORS = {-1: "TS_ERR_ARG", -2: "TS_ERR_DTYPE", -3: "TS_ERR_NULL", -4: "TS_ERR_WORKSPACE",
          -5: "TS_ERR_HIP", -6: "TS_ERR_ALIGN", -7: "TS_ERR_CANCELLED", -8: "TS_ERR_TIMEOUT"}


class TsSeries(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("x_dtype", ctypes.c_int32),
                ("y", ctypes.c_void_p), ("y_dtype", ctypes.c_int32), ("n", ctypes.c_int64)]


class TsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class TsArgError(TsError, ValueError):
    pass


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        SP = ctypes.POINTER(TsSeries)
        L.ts_version.restype = ctypes.c_int
        L.ts_last_error.restype = ctypes.c_char_p
        L.ts_workspace_bytes.argtypes = [ctypes.c_int, SP, i64, i64]
        L.ts_workspace_bytes.restype = sz
        for f in (L.ts_minmax, L.ts_m4, L.ts_lttb, L.ts_nan_minmax, L.ts_nan_m4):
            f.argtypes = [SP, i64, vp, vp, vp, sz, vp]
            f.restype = ctypes.c_int
        L.ts_minmaxlttb.argtypes = [SP, i64, i64, vp, vp, vp, sz, vp]
        L.ts_minmaxlttb.restype = ctypes.c_int
        L.ts_minmaxlttb_noalloc.argtypes = [SP, i64, i64, vp, vp, vp]
        L.ts_minmaxlttb_noalloc.restype = ctypes.c_int
        L.ts_noalloc_scratch_bytes.argtypes = []
        L.ts_noalloc_scratch_bytes.restype = sz
        L.ts_bin_edges.argtypes = [SP, i64, vp, vp]
        L.ts_bin_edges.restype = ctypes.c_int
        L.ts_argminmax_workspace_bytes.argtypes = [SP, i64]
        L.ts_argminmax_workspace_bytes.restype = sz
        L.ts_bin_argminmax.argtypes = [SP, vp, i64, vp, vp, vp, sz, vp]
        L.ts_bin_argminmax.restype = ctypes.c_int
        L.ts_lttb_centres.argtypes = [SP, vp, i64, i64, vp, vp, vp]
        L.ts_lttb_centres.restype = ctypes.c_int
        L.ts_window.argtypes = [SP, i64, i64, vp, vp]
        L.ts_window.restype = ctypes.c_int
        L.ts_everynth.argtypes = [SP, i64, vp, vp, vp]
        L.ts_everynth.restype = ctypes.c_int
        L.ts_gather.argtypes = [SP, vp, vp, i64, vp, vp, vp]
        L.ts_gather.restype = ctypes.c_int
        L.ts_set_tuning.argtypes = [i64, i32, i32, i32, i32, i32]
        L.ts_set_tuning.restype = ctypes.c_int
        L.ts_scan_config.argtypes = [ctypes.c_int, ctypes.c_int, i64, i64, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
        L.ts_scan_config.restype = ctypes.c_int
        L.ts_profile_scan_events.argtypes = [vp, vp]
        L.ts_profile_scan_events.restype = ctypes.c_int
        _lib = L
    return _lib


VARIANT_SHAPE = {0: (4, 2), 1: (4, 1), 2: (8, 1), 3: (2, 2)}
CTYPE_NAME = {0: "signed char", 1: "short", 2: "int", 3: "long", 4: "unsigned char", 5: "unsigned short",
              6: "unsigned int", 7: "unsigned long", 8: "tsds::half_t", 9: "float", 10: "double"}


SCAN_KINDS = {0: "k_scan", 1: "k_scan_staged", 2: "k_scan_xc", 3: "k_scan_stream"}


def scan_config(dtype, n, nb=1, x_dtype=None):
    """(variant, chunk_bytes, kernel name) the scan uses for n elements of
    dtype in nb bins with x of x_dtype (None: no x)."""
    v, c, k = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
    xd = TS_NONE if x_dtype is None else DTYPE_CODES[x_dtype]
    check(lib().ts_scan_config(DTYPE_CODES[dtype], xd, int(n), int(nb), ctypes.byref(v), ctypes.byref(c),
                               ctypes.byref(k)))
    ct = CTYPE_NAME[DTYPE_CODES[dtype]]
    if k.value in (4, 5):
        u, nbuf = VARIANT_SHAPE[v.value]
        name = "k_bins_direct" if k.value == 4 else "k_bins_block"
        return v.value, c.value, f"tsds::{name}<{ct}, {u}, {nbuf}>"
    if k.value == 1:
        return v.value, c.value, f"tsds::k_scan_staged<{ct}>"
    if k.value == 3:
        es = torch.empty((), dtype=dtype).element_size()
        u = 8 if es >= 4 else 4 if es == 2 else 2
        return v.value, c.value, f"tsds::k_scan_stream<{ct}, {u}>"
    u, nbuf = VARIANT_SHAPE[v.value]
    return v.value, c.value, f"tsds::{SCAN_KINDS[k.value]}<{ct}, {u}, {nbuf}>"


def check(rc):
    if rc != 0:
        msg = lib().ts_last_error().decode()
        if rc in (-1, -2, -3, -6):
            raise TsArgError(rc, msg)
        raise TsError(rc, msg)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def series(y, x=None):
    """TsSeries for device tensors y (and x); both 1-D and contiguous."""
    if not isinstance(y, torch.Tensor) or y.device.type != "cuda":
        raise ValueError("y must be a CUDA (HIP) tensor")
    if y.dim() != 1 or not y.is_contiguous():
        raise ValueError("y must be 1-D and contiguous")
    if y.dtype not in DTYPE_CODES:
        raise ValueError(f"unsupported y dtype {y.dtype}")
    s = TsSeries(None, TS_NONE, y.data_ptr() if y.numel() else None, DTYPE_CODES[y.dtype], y.numel())
    if x is not None:
        if x.device != y.device or x.dim() != 1 or not x.is_contiguous() or x.numel() != y.numel():
            raise ValueError("x must be a contiguous 1-D tensor on y's device with y's length")
        if x.dtype not in DTYPE_CODES:
            raise ValueError(f"unsupported x dtype {x.dtype}")
        s.x = x.data_ptr() if x.numel() else None
        s.x_dtype = DTYPE_CODES[x.dtype] if x.numel() else TS_NONE
    return s


def stream_ptr(stream=None, device=None):
    st = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(st.cuda_stream)


class Workspace:
    """Grow-only device scratch buffer (one per stream: calls on one stream
    are ordered, so they may share it)."""

    def __init__(self):
        self.buf = {}

    def get(self, nbytes, device, stream):
        key = (str(device), stream.cuda_stream)
        b = self.buf.get(key)
        if nbytes == 0:
            return None
        if b is None or b.numel() < nbytes:
            b = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device=device)
            self.buf[key] = b
        return b


WS = Workspace()

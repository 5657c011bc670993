"""Serving engine binding: zoom/pan MinMaxLTTB requests over series resident
in HBM, continuously batched by libtsds's scheduler thread (marshalling only).

    srv = Server([(x0, y0), (x1, y1)], n_streams=4, max_batch=32)
    rid = srv.submit(series=0, xa=1000, xb=90000, n_out=2000)
    srv.cancel(rid)        # only while it is still pending
    for r in srv.poll():   # dicts with id, indices (numpy), t_submit, t_done ...
        ...
    srv.close()
"""
import ctypes

import numpy as np

from . import _lib as L


class TsServerConfig(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("max_nout", ctypes.c_int64),
                ("minmax_ratio", ctypes.c_int64), ("plain", ctypes.c_int32), ("arena_bytes", ctypes.c_size_t),
                ("timeout_s", ctypes.c_double)]


class TsResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("series", ctypes.c_int32), ("status", ctypes.c_int32),
                ("count", ctypes.c_int64), ("offset", ctypes.c_int64), ("i0", ctypes.c_int64),
                ("i1", ctypes.c_int64), ("t_submit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("batch_size", ctypes.c_int64), ("t_admit", ctypes.c_double), ("t_run", ctypes.c_double)]


def _setup(lib):
    if getattr(lib, "_serve_ready", False):
        return
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.ts_server_create.argtypes = [ctypes.POINTER(L.TsSeries), i32, ctypes.POINTER(TsServerConfig),
                                     ctypes.POINTER(vp)]
    lib.ts_server_create.restype = ctypes.c_int
    lib.ts_server_submit.argtypes = [vp, i32, i64, i64, i64, ctypes.POINTER(i64)]
    lib.ts_server_submit.restype = ctypes.c_int
    lib.ts_server_poll.argtypes = [vp, ctypes.POINTER(TsResult), i32, ctypes.POINTER(i64), i64,
                                   ctypes.POINTER(i32)]
    lib.ts_server_poll.restype = ctypes.c_int
    lib.ts_server_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                    ctypes.POINTER(i64)]
    lib.ts_server_stats.restype = ctypes.c_int
    lib.ts_server_cancel.argtypes = [vp, i64]
    lib.ts_server_cancel.restype = ctypes.c_int
    lib.ts_server_now.argtypes = []
    lib.ts_server_now.restype = ctypes.c_double
    lib.ts_server_free.argtypes = [vp]
    lib.ts_server_free.restype = None
    lib._serve_ready = True


class Server:
    def __init__(self, series, n_streams=4, max_batch=32, max_nout=4000, minmax_ratio=4, plain=False,
                 arena_bytes=0, timeout_s=0.0):
        self.lib = L.lib()
        _setup(self.lib)
        self._keep = list(series)
        arr = (L.TsSeries * len(series))()
        for i, (x, y) in enumerate(series):
            arr[i] = L.series(y, x)
        cfg = TsServerConfig(n_streams, max_batch, max_nout, minmax_ratio, 1 if plain else 0, arena_bytes,
                             float(timeout_s))
        h = ctypes.c_void_p()
        L.check(self.lib.ts_server_create(arr, len(series), ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h
        self.max_nout = max_nout
        self._res = (TsResult * 256)()
        self._cap = 256 * max_nout
        self._idx = np.empty(self._cap, np.int64)

    def now(self):
        return self.lib.ts_server_now()

    def submit(self, series, xa, xb, n_out):
        rid = ctypes.c_int64()
        L.check(self.lib.ts_server_submit(self.h, int(series), int(xa), int(xb), int(n_out), ctypes.byref(rid)))
        return rid.value

    def cancel(self, rid):
        """Cancel a request that is still pending: True if it was (its result
        then comes back with status TS_ERR_CANCELLED), False if it is already
        running or finished."""
        rc = self.lib.ts_server_cancel(self.h, int(rid))
        if rc == -1:
            return False
        L.check(rc)
        return True

    def poll(self):
        out = []
        n = ctypes.c_int32()
        ip = self._idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        while True:
            L.check(self.lib.ts_server_poll(self.h, self._res, 256, ip, self._cap, ctypes.byref(n)))
            for k in range(n.value):
                r = self._res[k]
                out.append(dict(id=r.id, series=r.series, status=r.status, i0=r.i0, i1=r.i1,
                                t_submit=r.t_submit, t_done=r.t_done, batch_size=r.batch_size,
                                t_admit=r.t_admit, t_run=r.t_run,
                                indices=self._idx[r.offset: r.offset + r.count].copy()))
            if n.value < 256:
                return out

    def stats(self):
        b, m, d, p = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        rc = self.lib.ts_server_stats(self.h, ctypes.byref(b), ctypes.byref(m), ctypes.byref(d), ctypes.byref(p))
        return dict(batches=b.value, max_batch=m.value, done=d.value, pending=p.value, error=rc)

    def close(self):
        if self.h:
            self.lib.ts_server_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Batched downsampling of many series in one pass (marshalling only).

    b = Batch([dict(algo="minmax", y=y0, n_out=1000),
               dict(algo="m4", y=y1, x=x1, n_out=2000),
               dict(algo="minmaxlttb", y=y2, x=x2, n_out=800, minmax_ratio=4)])
    b.run(graph=True)          # one hipGraph launch for the whole batch
    idx0, idx1, idx2 = b.results()

The series tensors must stay alive (and unmoved) while the Batch is used.
"""
import ctypes

import torch

from . import _lib as L


class TsTask(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("series", L.TsSeries), ("n_out", ctypes.c_int64),
                ("minmax_ratio", ctypes.c_int64), ("out_offset", ctypes.c_int64)]


def _setup(lib):
    if getattr(lib, "_batch_ready", False):
        return
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    lib.ts_batch_plan.argtypes = [ctypes.POINTER(TsTask), i64, ctypes.POINTER(vp)]
    lib.ts_batch_plan.restype = ctypes.c_int
    lib.ts_batch_workspace_bytes.argtypes = [vp]
    lib.ts_batch_workspace_bytes.restype = sz
    lib.ts_batch_out_size.argtypes = [vp]
    lib.ts_batch_out_size.restype = i64
    lib.ts_batch_run.argtypes = [vp, vp, vp, vp, sz, vp, ctypes.c_int]
    lib.ts_batch_run.restype = ctypes.c_int
    lib.ts_batch_set_tuning.argtypes = [vp, i64, i32, i64]
    lib.ts_batch_set_tuning.restype = ctypes.c_int
    lib.ts_batch_get_tuning.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i64)]
    lib.ts_batch_get_tuning.restype = ctypes.c_int
    lib.ts_batch_autotune.argtypes = [vp, vp, vp, vp, sz, vp, ctypes.c_char_p]
    lib.ts_batch_autotune.restype = ctypes.c_int
    lib.ts_plan_free.argtypes = [vp]
    lib.ts_plan_free.restype = None
    lib._batch_ready = True


class Batch:
    def __init__(self, tasks, device=None):
        self.lib = L.lib()
        _setup(self.lib)
        if not tasks:
            raise ValueError("empty batch")
        self.device = device or tasks[0]["y"].device
        self._keep = []
        arr = (TsTask * len(tasks))()
        off = 0
        self.offsets = []
        for i, t in enumerate(tasks):
            y, x = t["y"], t.get("x")
            self._keep += [y, x]
            s = L.series(y, x)
            arr[i].algo = L.ALGO[t["algo"]]
            arr[i].series = s
            arr[i].n_out = int(t["n_out"])
            arr[i].minmax_ratio = int(t.get("minmax_ratio", 4))
            arr[i].out_offset = off
            self.offsets.append(off)
            off += int(t["n_out"])
        self.ntasks = len(tasks)
        plan = ctypes.c_void_p()
        L.check(self.lib.ts_batch_plan(arr, len(tasks), ctypes.byref(plan)))
        self.plan = plan
        self.ws_bytes = int(self.lib.ts_batch_workspace_bytes(plan))
        self.out = torch.empty(max(int(self.lib.ts_batch_out_size(plan)), 1), dtype=torch.int64,
                               device=self.device)
        self.counts = torch.zeros(self.ntasks, dtype=torch.int64, device=self.device)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)

    def _args(self, stream):
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        return (self.plan, L._ptr(self.out), L._ptr(self.counts), L._ptr(self.ws), self.ws.numel(),
                ctypes.c_void_p(st.cuda_stream))

    def run(self, stream=None, graph=False):
        """Enqueue the whole batch (no host sync)."""
        L.check(self.lib.ts_batch_run(*self._args(stream), 1 if graph else 0))

    def set_tuning(self, chunk_bytes, small_bin, grid_blocks):
        L.check(self.lib.ts_batch_set_tuning(self.plan, int(chunk_bytes), int(small_bin), int(grid_blocks)))

    def tuning(self):
        c, s, g = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        L.check(self.lib.ts_batch_get_tuning(self.plan, ctypes.byref(c), ctypes.byref(s), ctypes.byref(g)))
        return c.value, s.value, g.value

    def autotune(self, cache_path=None, stream=None):
        p = cache_path.encode() if cache_path else None
        L.check(self.lib.ts_batch_autotune(*self._args(stream), p))
        return self.tuning()

    def results(self):
        """List of per-task index tensors (syncs once for the counts)."""
        cnt = self.counts.cpu().tolist()
        return [self.out[o: o + c] for o, c in zip(self.offsets, cnt)]

    def close(self):
        if self.plan:
            self.lib.ts_plan_free(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Downsampler classes with the interface of Sec. 2.3:

    downsample([x], y, n_out, **kwargs) -> indices

x is optional (absent: equally sampled), y mandatory, n_out the number of
output points (positional or keyword).  numpy inputs are copied to the
current HIP device, downsampled there and answered with a uint64 numpy array
(the paper's return type); torch CUDA tensors stay on their device and the
answer is a device int64 tensor.  `parallel` is accepted for interface
compatibility and ignored: every call runs on the GPU.  MinMaxLTTB takes
minmax_ratio (default 4, Sec. 4).  NaNMinMaxDownsampler and NaNM4Downsampler
skip NaN values of y (an all-NaN bin keeps its first index); the others
require y without NaN.
"""
import numpy as np
import torch

from . import api

_NP_TO_TORCH = {
    np.dtype(np.int8): torch.int8, np.dtype(np.int16): torch.int16, np.dtype(np.int32): torch.int32,
    np.dtype(np.int64): torch.int64, np.dtype(np.uint8): torch.uint8, np.dtype(np.uint16): torch.uint16,
    np.dtype(np.uint32): torch.uint32, np.dtype(np.uint64): torch.uint64, np.dtype(np.float16): torch.float16,
    np.dtype(np.float32): torch.float32, np.dtype(np.float64): torch.float64,
}


def _to_device(a, device):
    if isinstance(a, torch.Tensor):
        return a.contiguous() if a.device.type == "cuda" else a.contiguous().to(device)
    a = np.ascontiguousarray(a)
    if a.ndim != 1:
        raise ValueError("inputs must be 1-D")
    if a.dtype not in _NP_TO_TORCH:
        raise ValueError(f"unsupported dtype {a.dtype}")
    return torch.from_numpy(a).to(device)


class AbstractDownsampler:
    _kwargs = ()

    def _call(self, y, n_out, x, **kw):
        raise NotImplementedError

    def downsample(self, *args, n_out=None, parallel=False, **kwargs):
        args = list(args)
        if n_out is None:
            if not args or isinstance(args[-1], (np.ndarray, torch.Tensor)):
                raise TypeError("n_out is required")
            n_out = args.pop()
        if len(args) not in (1, 2):
            raise TypeError("downsample([x], y, n_out): give y, or x and y")
        unknown = set(kwargs) - set(self._kwargs)
        if unknown:
            raise TypeError(f"unexpected keyword arguments {sorted(unknown)}")
        n_out = int(n_out)
        y = args[-1]
        x = args[0] if len(args) == 2 else None
        host = not isinstance(y, torch.Tensor)
        device = y.device if not host and y.device.type == "cuda" else torch.device("cuda", torch.cuda.current_device())
        yd = _to_device(y, device)
        xd = _to_device(x, device) if x is not None else None
        if xd is not None and xd.numel() != yd.numel():
            raise ValueError("x and y must have the same length")
        idx = self._call(yd, n_out, xd, **kwargs)
        return idx.cpu().numpy().astype(np.uint64) if host else idx


class MinMaxDownsampler(AbstractDownsampler):
    """MinMax (Sec. 2.1-2.2): per bin the first argmin and argmax, n_out / 2 bins."""

    def _call(self, y, n_out, x):
        return api.minmax(y, n_out, x=x)


class M4Downsampler(AbstractDownsampler):
    """M4: per bin the first, argmin, argmax and last index, n_out / 4 bins."""

    def _call(self, y, n_out, x):
        return api.m4(y, n_out, x=x)


class NaNMinMaxDownsampler(AbstractDownsampler):
    """MinMax with NaN values skipped; an all-NaN bin keeps its first index."""

    def _call(self, y, n_out, x):
        return api.nan_minmax(y, n_out, x=x)


class NaNM4Downsampler(AbstractDownsampler):
    """M4 with NaN values skipped in the argmin/argmax."""

    def _call(self, y, n_out, x):
        return api.nan_m4(y, n_out, x=x)


class LTTBDownsampler(AbstractDownsampler):
    """LTTB over all points (Sec. 4)."""

    def _call(self, y, n_out, x):
        return api.lttb(y, n_out, x=x)


class MinMaxLTTBDownsampler(AbstractDownsampler):
    """MinMaxLTTB (Sec. 4): MinMax preselection of n_out * minmax_ratio points, then LTTB."""
    _kwargs = ("minmax_ratio",)

    def _call(self, y, n_out, x, minmax_ratio=4):
        return api.minmaxlttb(y, n_out, x=x, minmax_ratio=int(minmax_ratio))


class EveryNthDownsampler(AbstractDownsampler):
    """EveryNth: every k-th index, k = ceil(n / n_out); x is not used."""

    def _call(self, y, n_out, x):
        return api.everynth(y, n_out, x=x)

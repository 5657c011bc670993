"""MI355X-native time-series downsampling hot path (arXiv 2307.05389).

    import paper_2307_05389_amd as tsds
    idx = tsds.minmax(y, n_out)             # y: 1-D CUDA tensor, any of 11 dtypes
    idx = tsds.m4(y, n_out, x=timestamps)   # optional sorted x
    idx = tsds.lttb(y, n_out)
    idx = tsds.minmaxlttb(y, n_out, minmax_ratio=4)
    idx = tsds.everynth(y, n_out)
    x_sel, y_sel = tsds.gather(y, idx, x=timestamps)   # the selected points
    idx = tsds.MinMaxLTTBDownsampler().downsample(x_np, y_np, n_out=1000)   # numpy in, uint64 out

Each call returns a device int64 tensor of selected indices (strictly
increasing).  The work runs in libtsds.so's HIP kernels on the tensors'
device and the current stream; see include/tsds.h for the exact semantics.
"""
from .api import (  # noqa: F401
    bin_argminmax, bin_edges, downsample_into, everynth, gather, lttb, lttb_centres, m4, minmax, minmaxlttb,
    minmaxlttb_noalloc,
    nan_m4, nan_minmax,
    set_tuning, window, workspace_bytes,
)
from .downsamplers import (  # noqa: F401
    EveryNthDownsampler, LTTBDownsampler, M4Downsampler, MinMaxDownsampler, MinMaxLTTBDownsampler,
    NaNM4Downsampler, NaNMinMaxDownsampler,
)
from ._lib import TsArgError, TsError, lib  # noqa: F401
from .batch import Batch  # noqa: F401
from .serve import Server  # noqa: F401

__all__ = ["minmax", "m4", "lttb", "minmaxlttb", "everynth", "gather", "nan_minmax", "nan_m4",
           "NaNMinMaxDownsampler", "NaNM4Downsampler", "MinMaxDownsampler", "M4Downsampler",
           "LTTBDownsampler", "MinMaxLTTBDownsampler", "EveryNthDownsampler", "downsample_into", "workspace_bytes", "bin_edges",
           "bin_argminmax", "lttb_centres", "window", "set_tuning", "Batch", "Server", "TsError", "TsArgError"]

"""ts_minmaxlttb_noalloc (MinMaxLTTB over the library's static device scratch,
for callers that cannot allocate) against ts_minmaxlttb with a caller
workspace: bit-identical indices and counts over consecutive calls, each
later call on a smaller input than the one before (the scratch keeps the
previous call's contents), plus one call with n <= n_out."""
import numpy as np
import pytest
import torch

import synthetic as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _with_workspace(yd, n_out, ratio, xd):
    """The existing entry point with a workspace the test allocates."""
    import paper_2307_05389_amd as tsds
    out = torch.full((n_out,), -1, dtype=torch.int64, device=yd.device)
    cnt = torch.full((1,), -1, dtype=torch.int64, device=yd.device)
    need = tsds.workspace_bytes("minmaxlttb", yd, n_out, x=xd, minmax_ratio=ratio)
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=yd.device)
    tsds.downsample_into("minmaxlttb", yd, n_out, out, cnt, x=xd, minmax_ratio=ratio, workspace=ws)
    torch.cuda.synchronize()
    return out[: int(cnt.item())].cpu().numpy()


def _noalloc(yd, n_out, ratio, xd):
    import paper_2307_05389_amd as tsds
    out = torch.full((n_out,), -1, dtype=torch.int64, device=yd.device)
    cnt = torch.full((1,), -1, dtype=torch.int64, device=yd.device)
    tsds.minmaxlttb_noalloc(yd, n_out, out, cnt, x=xd, minmax_ratio=ratio)
    torch.cuda.synchronize()
    return out[: int(cnt.item())].cpu().numpy()


# (n, y dtype, x, n_out, ratio): largest first, each later call smaller
CASES = [
    (12_000_017, np.float32, True, 2000, 4),
    (3_000_001, np.int16, False, 1000, 8),
    (200_003, np.float64, True, 4000, 4),
    (1_000, np.float32, False, 2000, 4),       # n <= n_out: all indices
]


def test_noalloc_equals_workspace_call():
    from paper_2307_05389_amd import _lib as L
    assert L.lib().ts_noalloc_scratch_bytes() == 64 << 20
    dev = torch.device("cuda:0")
    for n, dt, with_x, n_out, ratio in CASES:
        say(f"[noalloc] n={n} {np.dtype(dt).name} x={with_x} n_out={n_out} ratio={ratio}")
        y = S.walk(n, dt, seed=n % 97)
        yd = torch.from_numpy(y).to(dev)
        xd = torch.from_numpy(S.timestamps(n, 100, seed=n % 89)).to(dev) if with_x else None
        ref = _with_workspace(yd, n_out, ratio, xd)
        for rep in range(2):     # twice on the same input: the second sees its own stale scratch
            got = _noalloc(yd, n_out, ratio, xd)
            assert np.array_equal(got, ref), (n, rep)
        if n <= n_out:
            assert np.array_equal(ref, np.arange(n))


def test_noalloc_rejects_a_series_beyond_the_scratch():
    """Checked on the host before anything is enqueued; no device memory is
    touched (the series pointer is a real but small buffer)."""
    from paper_2307_05389_amd import _lib as L
    import ctypes
    dev = torch.device("cuda:0")
    y = torch.zeros(16, dtype=torch.float32, device=dev)
    out = torch.full((2000,), -1, dtype=torch.int64, device=dev)
    cnt = torch.full((1,), -1, dtype=torch.int64, device=dev)
    s = L.TsSeries(None, L.TS_NONE, y.data_ptr(), 9, 10_000_000_000)
    rc = L.lib().ts_minmaxlttb_noalloc(ctypes.byref(s), 2000, 4, L._ptr(out), L._ptr(cnt), None)
    assert rc == -4 and b"scratch" in L.lib().ts_last_error()
    torch.cuda.synchronize()
    assert int(cnt.item()) == -1 and bool((out == -1).all())

"""GPU parity of EveryNth, the gather of selected points and the Downsampler
classes (numpy and torch inputs) against the CPU oracle.  Indices are
compared bit-exactly; gathered values are compared as raw bytes with numpy's
own indexing of the same inputs."""
import ctypes

import numpy as np
import pytest
import torch

import synthetic as S

pytestmark = pytest.mark.gpu

ALL = [np.int8, np.int16, np.int32, np.int64, np.uint8, np.uint16, np.uint32, np.uint64,
       np.float16, np.float32, np.float64]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ts():
    import paper_2307_05389_amd as t
    t.set_tuning()
    return t


@pytest.mark.parametrize("n", [0, 1, 2, 5, 999, 1000, 1001, 4097, 12345, 10**7 + 3])
def test_everynth_parity(ts, oracle_mod, n):
    y = torch.zeros(max(n, 1), dtype=torch.int8, device="cuda")[:n]
    for n_out in (1, 2, 3, 7, 100, 1000, 1001, 4096, 5000):
        say("everynth", n, n_out)
        got = ts.everynth(y, n_out).cpu().numpy()
        exp = oracle_mod.everynth(n, n_out)
        assert got.tolist() == exp.tolist(), (n, n_out)


def test_everynth_full_size(ts, oracle_mod):
    """1e8 points, 4000 outputs: the size of the other headline workloads."""
    n = 10**8
    y = torch.empty(n, dtype=torch.uint8, device="cuda")
    for n_out in (4000, 3999, 2):
        got = ts.everynth(y, n_out).cpu().numpy()
        assert np.array_equal(got, oracle_mod.everynth(n, n_out)), n_out


def _raw_gather(ts, y, x, idx, count, cap, fill=0x5A):
    """Calls ts_gather through the C ABI with outputs pre-filled with `fill`
    bytes, so untouched positions are visible."""
    from paper_2307_05389_amd import _lib as L
    yd, xd = dev(y), (None if x is None else dev(x))
    s = L.series(yd, xd)
    yo = torch.full((cap * y.itemsize,), fill, dtype=torch.uint8, device="cuda")
    xo = None if x is None else torch.full((cap * x.itemsize,), fill, dtype=torch.uint8, device="cuda")
    it = dev(np.asarray(idx, np.int64)) if len(idx) else torch.zeros(1, dtype=torch.int64, device="cuda")
    ct = torch.tensor([count], dtype=torch.int64, device="cuda")
    L.check(L.lib().ts_gather(ctypes.byref(s), L._ptr(it), L._ptr(ct), cap, L._ptr(xo), L._ptr(yo),
                              L.stream_ptr()))
    torch.cuda.synchronize()
    ys = yo.cpu().numpy().view(y.dtype)
    xs = None if x is None else xo.cpu().numpy().view(x.dtype)
    return xs, ys


def _expect(a, idx, count, cap, fill=0x5A):
    out = np.frombuffer(bytes([fill]) * (cap * a.itemsize), dtype=a.dtype).copy()
    m = max(0, min(count, cap))
    for i in range(m):
        j = idx[i]
        if 0 <= j < len(a):
            out[i] = a[j]
    return out


@pytest.mark.parametrize("dt", ALL)
@pytest.mark.parametrize("xk", ["none", "i32", "i64", "u64", "f32", "f64"])
def test_gather_parity(ts, dt, xk):
    n = 5000
    rng = np.random.default_rng(7)
    y = S.walk(n, dt, seed=11)
    x = None
    if xk != "none":
        x = {"i32": np.int32, "i64": np.int64, "u64": np.uint64, "f32": np.float32, "f64": np.float64}[xk]
        x = np.sort(rng.integers(0, 10**6, n)).astype(x)
    idx = np.sort(rng.choice(n, 700, replace=False)).astype(np.int64)
    idx[[3, 50]] = [-1, n]                         # out of range: left untouched
    for count, cap in ((700, 700), (400, 700), (900, 700), (-3, 700), (0, 700), (700, 1)):
        say("gather", np.dtype(dt).name, xk, count, cap)
        xs, ys = _raw_gather(ts, y, x, idx, count, cap)
        assert ys.tobytes() == _expect(y, idx, count, cap).tobytes(), (count, cap)
        if x is not None:
            assert xs.tobytes() == _expect(x, idx, count, cap).tobytes(), (count, cap)


def test_gather_follows_device_count(ts, oracle_mod):
    """Downsample then gather with the device count, no host sync between."""
    n = 10**6 + 17
    y = S.walk(n, np.float32, seed=3)
    x = S.timestamps(n, 1000, seed=4)
    yd, xd = dev(y), dev(x)
    out = torch.empty(2000, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ts.downsample_into("minmaxlttb", yd, 2000, out, cnt, x=xd, minmax_ratio=4)
    xs, ys = ts.gather(yd, out, x=xd, count=cnt)
    torch.cuda.synchronize()
    exp = oracle_mod.minmaxlttb(y, 2000, 4, x=x)
    m = int(cnt.item())
    assert m == len(exp)
    assert np.array_equal(ys.cpu().numpy()[:m], y[exp])
    assert np.array_equal(xs.cpu().numpy()[:m], x[exp])


def test_gather_full_size(ts):
    """1e8 f64 points with int64 x: gather of the M4 selection (4000 outputs)."""
    n = 10**8
    yd = torch.empty(n, dtype=torch.float64, device="cuda").uniform_(-1, 1)
    xd = torch.arange(n, dtype=torch.int64, device="cuda") * 7 + 11
    idx = ts.m4(yd, 4000, x=xd)
    xs, ys = ts.gather(yd, idx, x=xd)
    ii = idx.cpu().numpy()
    assert np.array_equal(xs.cpu().numpy(), ii * 7 + 11)
    assert np.array_equal(ys.cpu().numpy(), yd[idx].cpu().numpy())


CLASSES = [("MinMaxDownsampler", "minmax", {}), ("M4Downsampler", "m4", {}), ("LTTBDownsampler", "lttb", {}),
           ("MinMaxLTTBDownsampler", "minmaxlttb", {"minmax_ratio": 3}), ("EveryNthDownsampler", "everynth", {})]


@pytest.mark.parametrize("cls,algo,kw", CLASSES)
@pytest.mark.parametrize("with_x", [False, True])
def test_downsampler_classes(ts, oracle_mod, cls, algo, kw, with_x):
    n, n_out = 200_003, 1000
    y = S.walk(n, np.float32, seed=5)
    x = S.timestamps(n, 100, seed=6) if with_x else None
    if algo == "minmaxlttb":
        exp = oracle_mod.minmaxlttb(y, n_out, kw["minmax_ratio"], x=x)
    elif algo == "everynth":
        exp = oracle_mod.everynth(n, n_out)
    else:
        exp = getattr(oracle_mod, algo)(y, n_out, x=x)
    d = getattr(ts, cls)()
    args = (y,) if x is None else (x, y)
    say(cls, with_x)
    got = d.downsample(*args, n_out=n_out, parallel=True, **kw)          # numpy in: uint64 numpy out
    assert isinstance(got, np.ndarray) and got.dtype == np.uint64
    assert np.array_equal(got.astype(np.int64), exp)
    got2 = d.downsample(*args, n_out, **kw)                               # n_out positional
    assert np.array_equal(got2, got)
    targs = tuple(dev(a) for a in args)
    got3 = d.downsample(*targs, n_out=n_out, **kw)                        # torch in: device int64 out
    assert got3.device.type == "cuda" and got3.dtype == torch.int64
    assert np.array_equal(got3.cpu().numpy(), exp)


def test_listing2_usage(ts, oracle_mod):
    """The usage of Listing 2: a numpy series, MinMaxLTTB to 1000 points."""
    y = S.walk(10**6, np.float64, seed=8)
    got = ts.MinMaxLTTBDownsampler().downsample(y, n_out=1000)
    assert got.dtype == np.uint64 and len(got) == 1000
    assert np.array_equal(got.astype(np.int64), oracle_mod.minmaxlttb(y, 1000, 4))

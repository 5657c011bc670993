"""GPU parity of the NaN-aware MinMax and M4 (NaN skipped, an all-NaN bin
keeps its first index) with the CPU oracle, bit-exact, through the C ABI."""
import numpy as np
import pytest
import torch

import synthetic as S

pytestmark = pytest.mark.gpu

FLOATS = [np.float16, np.float32, np.float64]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ts():
    import paper_2307_05389_amd as t
    t.set_tuning()
    yield t
    t.set_tuning()


def with_nan(y, frac, seed, runs=False):
    """NaN at a fraction of the points, optionally as long runs; with any NaN,
    also a negative and a signalling NaN bit pattern of the type."""
    y = y.copy()
    n = len(y)
    rng = np.random.default_rng(seed)
    if runs:
        for _ in range(max(1, int(frac * 20))):
            a = int(rng.integers(0, max(n - 1, 1)))
            y[a: a + int(rng.integers(1, max(2, n // 10)))] = np.nan
    else:
        y[rng.random(n) < frac] = np.nan
    if n > 8 and frac > 0:
        ut = {np.dtype(np.float16): np.uint16, np.dtype(np.float32): np.uint32, np.dtype(np.float64): np.uint64}
        bits = y.view(ut[y.dtype])
        neg_nan = {2: 0xFE00, 4: 0xFFC00000, 8: 0xFFF8000000000000}[y.itemsize]
        snan = {2: 0x7C01, 4: 0x7F800001, 8: 0x7FF0000000000001}[y.itemsize]
        bits[n // 3] = neg_nan
        bits[n // 2] = snan
    return y


def xs(kind, n, seed):
    if kind == "none":
        return None
    g = S.timestamps(n, 1000, seed=seed)
    if n > 10:
        g[n // 3:] += 10**7                 # empty bins
        g[2 * n // 3: 2 * n // 3 + 5] = g[2 * n // 3]
        g = np.maximum.accumulate(g)
    if kind == "i64":
        return g
    if kind == "i32":
        return (g // 16).astype(np.int32)
    return g.astype(np.float64)


def run(ts, kind, y, n_out, x):
    r = getattr(ts, "nan_" + kind)(dev(y), n_out, x=None if x is None else dev(x))
    torch.cuda.synchronize()
    return r.cpu().numpy()


@pytest.mark.parametrize("dt", FLOATS)
@pytest.mark.parametrize("xk", ["none", "i64", "i32", "f64"])
@pytest.mark.parametrize("n", [1000, 33333, 300001])
def test_nan_parity(ts, oracle_mod, dt, xk, n):
    base = S.walk(n, dt, seed=n % 97)
    x = xs(xk, n, seed=7)
    for frac, runs in ((0.0, False), (0.01, False), (0.5, False), (0.99, False), (1.0, False), (0.3, True)):
        y = with_nan(base, frac, seed=int(frac * 100) + 1, runs=runs)
        for kind, n_out in (("minmax", 4), ("minmax", 100), ("minmax", 8000), ("m4", 4), ("m4", 1000),
                            ("m4", 8000)):
            say("nan", np.dtype(dt).name, xk, n, frac, runs, kind, n_out)
            got = run(ts, kind, y, n_out, x)
            exp = getattr(oracle_mod, "nan_" + kind)(y, n_out, x=x)
            assert np.array_equal(got, exp), (kind, n_out, frac, runs)


@pytest.mark.parametrize("chunk", [4096, 16384])
def test_nan_bins_straddling_many_chunks(ts, oracle_mod, chunk):
    """Small chunks: bins span many chunks, NaN-only chunks inside a bin and
    NaN-only bins that straddle chunk boundaries go through the merge."""
    n = 400_003
    y = S.walk(n, np.float32, seed=3)
    y[1000:150_000] = np.nan                 # whole bins and chunk runs of NaN
    y[300_000:300_050] = np.nan
    ts.set_tuning(chunk_bytes=chunk)
    try:
        for kind, n_out in (("minmax", 4), ("minmax", 20), ("m4", 8), ("m4", 400), ("minmax", 4000)):
            say("straddle", chunk, kind, n_out)
            got = run(ts, kind, y, n_out, None)
            assert np.array_equal(got, getattr(oracle_mod, "nan_" + kind)(y, n_out)), (kind, n_out)
    finally:
        ts.set_tuning()


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 8, 9, 63, 64, 65, 129])
def test_nan_small_and_edge(ts, oracle_mod, n):
    rng = np.random.default_rng(n)
    y = rng.normal(size=n)
    y[rng.random(n) < 0.4] = np.nan
    for kind, outs in (("minmax", (2, 4, 6)), ("m4", (4, 8))):
        for n_out in outs:
            assert np.array_equal(run(ts, kind, y, n_out, None), getattr(oracle_mod, "nan_" + kind)(y, n_out))


@pytest.mark.parametrize("dt", [np.int16, np.uint8, np.int64])
def test_nan_variant_on_integers_equals_plain(ts, dt):
    y = S.walk(100_000, dt, seed=4)
    for kind in ("minmax", "m4"):
        a = run(ts, kind, y, 400, None)
        b = getattr(ts, kind)(dev(y), 400).cpu().numpy()
        assert np.array_equal(a, b)


def test_nan_full_size(ts, oracle_mod):
    """1e8 f32 points with 1% NaN and NaN runs, int64 x, M4 to 4000 points."""
    n = 100_000_000
    say("nan full size: generating")
    y = with_nan(S.walk(n, np.float32, seed=9), 0.01, seed=9)
    y[10_000_000:10_500_000] = np.nan
    x = S.timestamps(n, 100, seed=10)
    got = run(ts, "m4", y, 4000, x)
    exp = oracle_mod.nan_m4(y, 4000, x=x)
    assert np.array_equal(got, exp)
    got = run(ts, "minmax", y, 2000, None)
    assert np.array_equal(got, oracle_mod.nan_minmax(y, 2000))


@pytest.mark.parametrize("cls,kind", [("NaNMinMaxDownsampler", "minmax"), ("NaNM4Downsampler", "m4")])
def test_nan_downsampler_classes(ts, oracle_mod, cls, kind):
    y = with_nan(S.walk(50_001, np.float64, seed=2), 0.1, seed=2)
    got = getattr(ts, cls)().downsample(y, n_out=400)
    assert got.dtype == np.uint64
    assert np.array_equal(got.astype(np.int64), getattr(oracle_mod, "nan_" + kind)(y, 400))


def test_nan_batched(ts, oracle_mod):
    """NaN-aware MinMax / M4 tasks in one batch with plain tasks: each task
    equals the oracle and the single call, eager and replayed from a graph,
    at two chunk sizes."""
    rng = np.random.default_rng(5)
    specs = []
    dts = [np.float32, np.float16, np.float64, np.int16]
    for i in range(24):
        L = int(np.exp(rng.uniform(np.log(100), np.log(4e5))))
        dt = dts[i % 4]
        y = S.walk(L, dt, seed=300 + i)
        if dt != np.int16:
            y = with_nan(y, [0.0, 0.05, 0.6, 1.0][(i // 4) % 4], seed=400 + i, runs=bool(i % 2))
        algo = ["nan_minmax", "nan_m4", "minmax" if dt == np.int16 else "nan_m4"][i % 3]
        n_out = int(rng.integers(8, 1200))
        n_out = 4 * (n_out // 4) if algo.endswith("m4") else 2 * (n_out // 2)
        x = S.timestamps(L, 100, seed=500 + i) if i % 5 == 2 else None
        specs.append(dict(algo=algo, y=y, x=x, n_out=n_out))
    dev_specs = []
    for s in specs:
        d = dict(s)
        d["y"] = dev(s["y"])
        d["x"] = None if s["x"] is None else dev(s["x"])
        dev_specs.append(d)
    b = ts.Batch(dev_specs)
    try:
        for chunk, graph in ((-1, False), (-1, True), (4096, True)):
            if chunk > 0:
                cb, sb, gb = b.tuning()
                b.set_tuning(chunk, sb, gb)
            b.out.fill_(-7)
            b.run(graph=graph)
            b.run(graph=graph)
            res = [r.cpu().numpy() for r in b.results()]
            for i, (s, d) in enumerate(zip(specs, dev_specs)):
                say("nan batch", chunk, graph, i, s["algo"], np.dtype(s["y"].dtype).name, len(s["y"]), s["n_out"])
                if s["algo"].startswith("nan_"):
                    exp = getattr(oracle_mod, s["algo"])(s["y"], s["n_out"], x=s["x"])
                    one = getattr(ts, s["algo"])(d["y"], s["n_out"], x=d["x"]).cpu().numpy()
                else:
                    exp = getattr(oracle_mod, s["algo"])(s["y"], s["n_out"], x=s["x"])
                    one = getattr(ts, s["algo"])(d["y"], s["n_out"], x=d["x"]).cpu().numpy()
                assert np.array_equal(res[i], exp), (chunk, graph, i)
                assert np.array_equal(res[i], one), (chunk, graph, i)
    finally:
        b.close()


@pytest.mark.parametrize("dt", FLOATS)
def test_nan_signed_zero_and_inf(ts, oracle_mod, dt):
    """Signed zeros, infinities and NaN repeated across lanes and vectors:
    the first occurrence of an extreme (zeros compare equal) must match the
    oracle, also where a vector holds only NaN or only infinities."""
    rng = np.random.default_rng(7)
    n = 200003
    pick = rng.integers(0, 6, n)
    y = np.choose(pick, [np.float64(-0.0), 0.0, -np.inf, np.inf, np.nan, 1.0]).astype(dt)
    y[1000:5000] = np.nan
    y[9000:9100] = np.inf
    for kind, per in (("minmax", 2), ("m4", 4)):
        for nb in (3, 40, 1000, 20000):
            say(f"[nan zeros/inf] {np.dtype(dt).name} {kind} nb={nb}")
            got = run(ts, kind, y, per * nb, None)
            exp = getattr(oracle_mod, "nan_" + kind)(y, per * nb)
            assert np.array_equal(got, exp), (kind, nb)

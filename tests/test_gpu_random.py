"""Randomised parity over many shapes, fixed seeds and case counts: single
series (every integer and float dtype, lengths 1e2..6e6, bin sizes from two
points to tens of thousands, misaligned device pointers, tie runs, with and
without int64 x, default tuning or forced LDS staging) against the oracle, and
mixed batches (MinMax, M4, MinMaxLTTB and the NaN-aware variants, eager and
graph runs, each replayed twice) against one plain call per task and, for the
first tasks of each batch, the oracle.  Every comparison is bit-exact."""
import numpy as np
import pytest
import torch

import synthetic as S

pytestmark = pytest.mark.gpu

DT = [np.uint8, np.int8, np.int16, np.uint16, np.float16, np.int32, np.uint32, np.float32, np.int64, np.uint64,
      np.float64]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ts():
    import paper_2307_05389_amd as t
    t.set_tuning()
    yield t
    t.set_tuning()


def _orc(oracle_mod, algo, y, n_out, x):
    if algo == "minmaxlttb":
        return oracle_mod.minmaxlttb(y, n_out, 4, x=x)
    return getattr(oracle_mod, algo)(y, n_out, x=x)


def test_random_series(ts, oracle_mod):
    rng = np.random.default_rng(20261203)
    for k in range(500):
        dt = DT[rng.integers(len(DT))]
        n = int(10 ** rng.uniform(2, 6.8))
        algo = ("minmax", "m4", "minmaxlttb")[rng.integers(3)]
        per = 4 if algo == "m4" else 2
        avg = 10 ** rng.uniform(0.3, 4.5)
        n_out = max(per, int(per * n / avg) // per * per)
        if algo == "minmaxlttb":
            n_out = max(4, min(n_out, n // 4))
        yfull = S.walk(n + 16, dt, seed=int(rng.integers(1 << 30)))
        if rng.random() < 0.5:
            S.tie_runs(yfull, float(rng.uniform(0.05, 0.6)), seed=int(rng.integers(1 << 30)))
        off = int(rng.integers(0, 16))
        y = np.ascontiguousarray(yfull[off:off + n])
        x = S.timestamps(n, int(rng.integers(1, 2000)), seed=int(rng.integers(1 << 30))) if rng.random() < 0.3 else None
        stage = int(rng.integers(-1, 2)) if rng.random() < 0.4 else -1
        say(f"[random {k}] {np.dtype(dt).name} n={n} off={off} {algo} n_out={n_out} x={x is not None} stage={stage}")
        yd = torch.from_numpy(yfull).to("cuda")[off:off + n]
        xd = None if x is None else torch.from_numpy(x).to("cuda")
        ts.set_tuning(stage=stage)
        try:
            r = ts.minmaxlttb(yd, n_out, x=xd) if algo == "minmaxlttb" else getattr(ts, algo)(yd, n_out, x=xd)
            got = r.cpu().numpy()
        finally:
            ts.set_tuning()
        assert np.array_equal(got, _orc(oracle_mod, algo, y, n_out, x)), k


def test_random_batches(ts, oracle_mod):
    rng = np.random.default_rng(31)
    fdt = [np.uint8, np.int8, np.int16, np.float16, np.int32, np.float32, np.int64, np.float64]
    for k in range(60):
        ntask = int(rng.integers(1, 80))
        tasks, host = [], []
        for _ in range(ntask):
            dt = fdt[rng.integers(len(fdt))]
            n = int(10 ** rng.uniform(1, 6.3))
            algo = ("minmax", "m4", "minmaxlttb", "nan_minmax", "nan_m4")[rng.integers(5)]
            if algo.startswith("nan") and np.dtype(dt).kind != "f":
                algo = algo[4:]
            per = 4 if algo.endswith("m4") else 2
            n_out = max(per, int(per * n / 10 ** rng.uniform(0.3, 5)) // per * per)
            if algo == "minmaxlttb":
                n_out = max(4, n_out)
            y = S.walk(n, dt, seed=int(rng.integers(1 << 30)))
            if algo.startswith("nan"):
                y = y.copy()
                y[rng.random(n) < 0.02] = np.nan
            x = S.timestamps(n, int(rng.integers(1, 500)), seed=int(rng.integers(1 << 30))) if rng.random() < 0.3 else None
            tasks.append(dict(algo=algo, y=torch.from_numpy(y).cuda(), x=None if x is None else torch.from_numpy(x).cuda(),
                              n_out=n_out))
            host.append((algo, y, x, n_out))
        graph = bool(rng.integers(2))
        say(f"[random batch {k}] {ntask} tasks graph={graph}")
        b = ts.Batch(tasks)
        try:
            for rep in range(2):
                b.counts.zero_()
                b.out.fill_(-1)
                b.run(graph=graph)
                torch.cuda.synchronize()
                for i, (t, r) in enumerate(zip(tasks, b.results())):
                    a = t["algo"]
                    p = ts.minmaxlttb(t["y"], t["n_out"], x=t["x"]) if a == "minmaxlttb" else \
                        getattr(ts, a)(t["y"], t["n_out"], x=t["x"])
                    got = r.cpu().numpy()
                    assert np.array_equal(p.cpu().numpy(), got), (k, i, a)
                    if rep == 0 and i < 4:
                        algo, y, x, n_out = host[i]
                        assert np.array_equal(_orc(oracle_mod, algo, y, n_out, x), got), (k, i, a)
        finally:
            b.close()

"""Batched mode: one persistent launch (eager or hipGraph) over many series of
mixed dtype, length, algorithm and n_out must give, task by task, exactly the
oracle's result and exactly the plain single-series call's result."""
import numpy as np
import pytest
import torch

import synthetic as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ts():
    import paper_2307_05389_amd as t
    return t


def make_batch(seed=0, n_series=48):
    rng = np.random.default_rng(seed)
    dts = [np.float32, np.float16, np.int16, np.uint8, np.float64, np.int8, np.uint64, np.int32]
    specs = []
    for i in range(n_series):
        L = int(np.exp(rng.uniform(np.log(50), np.log(3e5))))
        algo = ["minmax", "m4", "minmaxlttb"][i % 3]
        n_out = int(rng.integers(10, 1500))
        n_out = 4 * (n_out // 4) if algo == "m4" else (2 * (n_out // 2) if algo == "minmax" else max(3, n_out))
        n_out = max(n_out, 4)
        y = S.walk(L, dts[i % len(dts)], seed=100 + i)
        x = S.timestamps(L, 200, seed=200 + i) if i % 4 == 1 else None
        if x is not None and i % 8 == 1:
            x[L // 2:] += 10**6   # empty bins
        specs.append(dict(algo=algo, y=y, x=x, n_out=n_out, minmax_ratio=4))
    # edge cases: tiny, empty, n == n_out, MinMaxLTTB without preselection
    specs.append(dict(algo="minmax", y=S.walk(0, np.float32, 1), x=None, n_out=10))
    specs.append(dict(algo="m4", y=S.walk(12, np.float32, 2), x=None, n_out=12))
    specs.append(dict(algo="minmaxlttb", y=S.walk(900, np.float32, 3), x=None, n_out=300, minmax_ratio=4))
    specs.append(dict(algo="minmaxlttb", y=S.walk(200, np.int16, 4), x=None, n_out=300))
    return specs


def oracle_of(oracle_mod, s):
    if s["algo"] == "minmaxlttb":
        return oracle_mod.minmaxlttb(s["y"], s["n_out"], s.get("minmax_ratio", 4), x=s["x"])
    return getattr(oracle_mod, s["algo"])(s["y"], s["n_out"], x=s["x"])


def to_dev(specs):
    out = []
    for s in specs:
        d = dict(s)
        d["y"] = torch.from_numpy(np.ascontiguousarray(s["y"])).to("cuda")
        d["x"] = None if s["x"] is None else torch.from_numpy(s["x"]).to("cuda")
        out.append(d)
    return out


def test_batch_matches_oracle_and_plain(ts, oracle_mod):
    specs = make_batch(0)
    dev = to_dev(specs)
    say(f"[batch] plan {len(dev)} tasks")
    b = ts.Batch(dev)
    b.run()
    res = [r.cpu().numpy() for r in b.results()]
    for i, (s, d) in enumerate(zip(specs, dev)):
        say(f"[batch] task {i} {s['algo']} {s['y'].dtype} n={len(s['y'])} n_out={s['n_out']} x={s['x'] is not None}")
        exp = oracle_of(oracle_mod, s)
        assert np.array_equal(res[i], exp), i
        if len(s["y"]):
            if s["algo"] == "minmaxlttb":
                plain = ts.minmaxlttb(d["y"], s["n_out"], x=d["x"], minmax_ratio=s.get("minmax_ratio", 4))
            else:
                plain = getattr(ts, s["algo"])(d["y"], s["n_out"], x=d["x"])
            assert np.array_equal(res[i], plain.cpu().numpy()), i
    b.close()


def test_batch_graph_replays_and_tunings(ts):
    specs = make_batch(1, n_series=30)
    dev = to_dev(specs)
    b = ts.Batch(dev)
    b.run()
    ref = [r.cpu().clone() for r in b.results()]
    for rep in range(4):
        say(f"[batch] graph replay {rep}")
        b.out.fill_(-1)
        b.counts.fill_(-1)
        b.run(graph=True)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        got = [r.cpu() for r in b.results()]
        assert all(torch.equal(a, c) for a, c in zip(ref, got)), rep
        del junk
    for cb, sm, gb in ((4096, 1, 64), (65536, 4096, 2048), (8192, 32, 1), (1 << 20, 128, 300)):
        say(f"[batch] tuning {cb} {sm} {gb}")
        b.set_tuning(cb, sm, gb)
        b.out.fill_(-1)
        b.run(graph=bool(gb % 2))
        got = [r.cpu() for r in b.results()]
        assert all(torch.equal(a, c) for a, c in zip(ref, got)), (cb, sm, gb)
    b.close()


def test_batch_autotune_keeps_results(ts, tmp_path):
    specs = make_batch(2, n_series=20)
    b = ts.Batch(to_dev(specs))
    b.run()
    ref = [r.cpu().clone() for r in b.results()]
    cache = str(tmp_path / "tune.txt")
    t1 = b.autotune(cache)
    b.out.fill_(-1)
    b.run(graph=True)
    assert all(torch.equal(a, c.cpu()) for a, c in zip(ref, b.results()))
    b2 = ts.Batch(to_dev(specs))
    assert b2.autotune(cache) == t1        # served from the cache
    b.close()
    b2.close()


def test_batch_walk_maps_beyond_64k_lds(ts, oracle_mod):
    """MinMaxLTTB tasks whose walk maps need more than 64 KB of LDS (12,002
    candidates: 96 KB; 15,866: 124 KB) next to small ones, against the oracle
    and the plain call."""
    specs = [dict(algo="minmaxlttb", y=S.walk(1_000_003, np.float32, 81), x=None, n_out=3000, minmax_ratio=4),
             dict(algo="minmaxlttb", y=S.walk(200_000, np.int16, 82), x=S.timestamps(200_000, 50, seed=83),
                  n_out=1500, minmax_ratio=4),
             dict(algo="minmax", y=S.walk(50_000, np.uint8, 84), x=None, n_out=1000)]
    for tail in (None, dict(algo="minmaxlttb", y=S.walk(600_000, np.float64, 85), x=None, n_out=3966,
                             minmax_ratio=4)):
        sp = specs + ([tail] if tail else [])
        dev = to_dev(sp)
        b = ts.Batch(dev)
        for graph in (False, True):
            say(f"[batch lds] {len(sp)} tasks graph={graph}")
            b.run(graph=graph)
            res = [r.cpu().numpy() for r in b.results()]
            for i, (s, d) in enumerate(zip(sp, dev)):
                assert np.array_equal(res[i], oracle_of(oracle_mod, s)), i
                if s["algo"] == "minmaxlttb":
                    plain = ts.minmaxlttb(d["y"], s["n_out"], x=d["x"], minmax_ratio=s["minmax_ratio"])
                    assert np.array_equal(res[i], plain.cpu().numpy()), i
        b.close()


def test_batch_direct_bins(ts, oracle_mod):
    """Tasks without x whose bins hold 4..512 KB of y are reduced one
    wavefront per bin (no chunks, no merge), beside chunked and staged tasks
    and tasks with x in the same batch: every dtype, MinMax, M4 and the
    MinMaxLTTB preselection, bins around both size limits, series off the
    16-byte grid; equal to the oracle and to plain calls, graph replays
    included."""
    rng = np.random.default_rng(91)
    dts = [np.float32, np.float16, np.int16, np.uint8, np.float64, np.int8, np.uint64, np.int32]
    specs = []
    for i, dt in enumerate(dts):
        es = np.dtype(dt).itemsize
        for bin_bytes in (4096, 20_000, 500_000):
            algo = ["minmax", "m4", "minmaxlttb"][(i + bin_bytes) % 3]
            L = int(rng.integers(1_000_000, 3_000_000)) // es
            per = {"minmax": 2, "m4": 4, "minmaxlttb": 1}[algo]
            ratio = 2
            nb = max(1, L * es // bin_bytes)
            n_out = per * nb if algo != "minmaxlttb" else max(3, nb)
            y = S.walk(L + 3, dt, seed=300 + 3 * i + bin_bytes % 7)[3:]   # off the 16-byte grid
            specs.append(dict(algo=algo, y=y, x=None, n_out=n_out, minmax_ratio=ratio))
    # neighbours on the other paths: x, staged (short bins), chunked (long bins)
    specs.append(dict(algo="m4", y=S.walk(400_000, np.float32, 401), x=S.timestamps(400_000, 20, seed=402),
                      n_out=400, minmax_ratio=4))
    specs.append(dict(algo="minmax", y=S.walk(300_000, np.int16, 403), x=None, n_out=20_000, minmax_ratio=4))
    specs.append(dict(algo="minmax", y=S.walk(3_000_000, np.float32, 404), x=None, n_out=8, minmax_ratio=4))
    dev = to_dev(specs)
    b = ts.Batch(dev)
    b.run()
    res = [r.cpu().numpy() for r in b.results()]
    for i, (s, d) in enumerate(zip(specs, dev)):
        say(f"[batch direct] task {i} {s['algo']} {s['y'].dtype} n={len(s['y'])} n_out={s['n_out']}")
        assert np.array_equal(res[i], oracle_of(oracle_mod, s)), i
        if s["algo"] == "minmaxlttb":
            plain = ts.minmaxlttb(d["y"], s["n_out"], x=d["x"], minmax_ratio=s["minmax_ratio"])
        else:
            plain = getattr(ts, s["algo"])(d["y"], s["n_out"], x=d["x"])
        assert np.array_equal(res[i], plain.cpu().numpy()), i
    ref = [r.cpu().clone() for r in b.results()]
    for rep in range(3):
        say(f"[batch direct] graph replay {rep}")
        b.out.fill_(-1)
        b.counts.fill_(-1)
        b.run(graph=True)
        torch.cuda.synchronize()
        assert all(torch.equal(a, c.cpu()) for a, c in zip(ref, b.results())), rep
    b.close()

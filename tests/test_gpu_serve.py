"""Serving: every request served from the continuous-batching engine equals
the oracle on its window, and equals the same request served alone (plain
mode, no batching) -- results do not depend on what else is in the batch."""
import time

import numpy as np
import pytest
import torch

import synthetic as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def resident():
    series = []
    for s in range(4):
        n = [300_000, 1_000_003, 77_777, 2_000_000][s]
        x = S.timestamps(n, 100, seed=10_000 + s)
        y = S.walk(n, [np.float32, np.float32, np.int16, np.float64][s], seed=20_000 + s)
        series.append((x, y))
    dev = [(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()) for x, y in series]
    return series, dev


def requests(series, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        s = int(rng.integers(0, len(series)))
        x = series[s][0]
        R = int(x[-1] - x[0])
        w = float(np.exp(rng.uniform(np.log(1e-4), 0.0)))
        xa = int(x[0]) + int(rng.random() * (1 - w) * R) - (50 if i % 17 == 0 else 0)
        xb = xa + int(w * R)
        n_out = int(rng.integers(40, 1000)) // 2 * 2
        if i % 23 == 0:
            xb = xa - 1                      # empty window
        out.append((s, xa, xb, n_out))
    return out


def collect(srv, n, timeout=60):
    got = {}
    t0 = time.time()
    while len(got) < n and time.time() - t0 < timeout:
        for r in srv.poll():
            got[r["id"]] = r
        time.sleep(0.001)
    return got


def test_served_equals_oracle_and_alone(resident, oracle_mod):
    import paper_2307_05389_amd as ts
    series, dev = resident
    reqs = requests(series, 300, seed=1)
    srv = ts.Server(dev, n_streams=4, max_batch=16, max_nout=1000, minmax_ratio=4)
    say("[serve] submitting 300 requests")
    ids = [srv.submit(*q) for q in reqs]
    got = collect(srv, len(ids))
    st = srv.stats()
    srv.close()
    assert len(got) == len(ids) and st["error"] == 0
    assert st["max_batch"] > 1, st                      # requests were really batched
    alone_srv = ts.Server(dev, plain=True, max_nout=1000, minmax_ratio=4)
    alone_ids = [alone_srv.submit(*q) for q in reqs]
    alone = collect(alone_srv, len(alone_ids))
    alone_srv.close()
    for k, (rid, aid, q) in enumerate(zip(ids, alone_ids, reqs)):
        s, xa, xb, n_out = q
        x, y = series[s]
        r = got[rid]
        assert r["status"] == 0
        i0, i1 = oracle_mod.window(x, xa, xb)
        assert (r["i0"], r["i1"]) == (i0, i1)
        assert np.array_equal(r["indices"], alone[aid]["indices"]), k
        if k % 10 == 0 or i1 - i0 < 5000:
            say(f"[serve] oracle check request {k}: series {s} window {i1 - i0} n_out {n_out}")
            exp = i0 + oracle_mod.minmaxlttb(y[i0:i1], n_out, 4, x=x[i0:i1])
            assert np.array_equal(r["indices"], exp), k


def test_server_rejects_bad_requests(resident):
    import paper_2307_05389_amd as ts
    _, dev = resident
    srv = ts.Server(dev[:1], max_nout=500)
    with pytest.raises(ts.TsArgError):
        srv.submit(0, 0, 10, 1000)        # n_out above the server's maximum
    with pytest.raises(ts.TsArgError):
        srv.submit(3, 0, 10, 100)         # no such series
    srv.close()


def test_cancel_and_timeout_leave_the_rest_exact(resident, oracle_mod):
    """Cancelled and expired requests come back with their status and no
    indices; every other request of the same burst still equals the oracle on
    its window."""
    import paper_2307_05389_amd as ts
    series, dev = resident
    reqs = requests(series, 120, seed=5)
    # one stream, one request per batch: most of the burst waits in the queue
    srv = ts.Server(dev, n_streams=1, max_batch=1, max_nout=1000, minmax_ratio=4)
    ids = [srv.submit(*q) for q in reqs]
    cancelled = {rid for rid in ids[10::3] if srv.cancel(rid)}
    assert len(cancelled) > 10
    assert not srv.cancel(10**9)                       # unknown id
    got = collect(srv, len(ids))
    srv.close()
    say(f"[serve] cancelled {len(cancelled)} of {len(ids)}")
    assert len(got) == len(ids)
    for k, (rid, q) in enumerate(zip(ids, reqs)):
        r = got[rid]
        if rid in cancelled:
            assert r["status"] == -7 and len(r["indices"]) == 0
            continue
        assert r["status"] == 0, (k, r["status"])
        s, xa, xb, n_out = q
        x, y = series[s]
        i0, i1 = oracle_mod.window(x, xa, xb)
        exp = i0 + oracle_mod.minmaxlttb(y[i0:i1], n_out, 4, x=x[i0:i1])
        assert np.array_equal(r["indices"], exp), k
    # a 1 ms timeout on a burst that takes several: the tail expires
    srv = ts.Server(dev, n_streams=1, max_batch=1, max_nout=1000, minmax_ratio=4, timeout_s=0.001)
    ids = [srv.submit(*q) for q in reqs]
    got = collect(srv, len(ids))
    srv.close()
    status = [got[rid]["status"] for rid in ids]
    say(f"[serve] timeout: {status.count(-8)} expired, {status.count(0)} served")
    assert status.count(-8) > 0 and status.count(0) > 0 and set(status) <= {0, -8}
    for k, (rid, q) in enumerate(zip(ids, reqs)):
        r = got[rid]
        if r["status"] != 0:
            assert len(r["indices"]) == 0
            continue
        s, xa, xb, n_out = q
        x, y = series[s]
        i0, i1 = oracle_mod.window(x, xa, xb)
        exp = i0 + oracle_mod.minmaxlttb(y[i0:i1], n_out, 4, x=x[i0:i1])
        assert np.array_equal(r["indices"], exp), k


def test_single_request_batches_equal_oracle(resident, oracle_mod):
    """Requests that arrive one at a time run as batches of one (the
    single-series kernels); their results equal the oracle too."""
    import paper_2307_05389_amd as ts
    series, dev = resident
    reqs = requests(series, 40, seed=6)
    srv = ts.Server(dev, n_streams=4, max_batch=32, max_nout=1000, minmax_ratio=4)
    for k, q in enumerate(reqs):
        rid = srv.submit(*q)
        r = collect(srv, 1)[rid]
        assert r["status"] == 0 and r["batch_size"] == 1
        s, xa, xb, n_out = q
        x, y = series[s]
        i0, i1 = oracle_mod.window(x, xa, xb)
        exp = i0 + oracle_mod.minmaxlttb(y[i0:i1], n_out, 4, x=x[i0:i1])
        assert np.array_equal(r["indices"], exp), k
    srv.close()

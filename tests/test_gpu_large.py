"""Series longer than 2^31 elements (Sec. 2.1: the paper's kernel needs an
overflow-free outer loop because lane indices are narrower than the series;
here every global index is 64-bit).  One-byte series of 2^31 + 4,097 points
(2.1 GB), MinMax, M4 and MinMaxLTTB with no x, bit-exact against the oracle,
including the LDS-staged scan forced on.  Extremes are planted past 2^31 so
that the selected indices themselves need more than 31 bits."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

N = (1 << 31) + 4097


def say(*a):
    print(*a, flush=True)


def _series(dtype):
    """Wrapped random walk (every byte value occurs, long monotone runs and
    many ties), generated on the GPU, with the global extremes planted beyond
    index 2^31: the first minimum at 2^31 + 1,000 and the first maximum at
    2^31 + 3,000 (earlier equal values exist only past those points)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(71 if dtype == np.uint8 else 72)
    steps = torch.randint(-3, 4, (N,), generator=g, device="cuda", dtype=torch.int8)
    w = torch.empty(N, dtype=torch.uint8, device="cuda")
    chunk = 1 << 28
    carry = torch.zeros((), dtype=torch.int64, device="cuda")
    for s in range(0, N, chunk):
        e = min(N, s + chunk)
        c = steps[s:e].to(torch.int64).cumsum_(0)
        c += carry
        carry = c[-1].clone()
        # values 2..253 everywhere, so the planted 0/1 and 254/255 are unique
        w[s:e] = (c.remainder_(252) + 2).to(torch.uint8)
        del c
    del steps
    big = 1 << 31
    w[big + 1000] = 0
    w[big + 3000] = 255
    w[big + 2000] = 0        # a later equal minimum: the first one must win
    w[big + 4000] = 255
    w[big - 7] = 1
    w[big - 9] = 254
    if dtype == np.int8:
        w = (w.to(torch.int16) - 128).to(torch.int8)
    torch.cuda.synchronize()
    return w


@pytest.fixture(scope="module", params=[np.uint8, np.int8], ids=["u8", "i8"])
def big(request):
    yd = _series(request.param)
    yh = yd.cpu().numpy()
    assert len(yh) == N and yh.dtype == np.dtype(request.param)
    yield request.param, yd, yh
    del yd
    torch.cuda.empty_cache()


CASES = [("minmax", 2, 4), ("minmax", 1000, 4), ("minmax", 2_000_000, 4), ("m4", 4, 4), ("m4", 4000, 4),
         ("minmaxlttb", 2000, 4), ("minmaxlttb", 3, 2)]


def _gpu(ts, algo, yd, n_out, ratio):
    if algo == "minmaxlttb":
        r = ts.minmaxlttb(yd, n_out, minmax_ratio=ratio)
    else:
        r = getattr(ts, algo)(yd, n_out)
    torch.cuda.synchronize()
    return r.cpu().numpy()


def _oracle(oracle_mod, algo, yh, n_out, ratio):
    if algo == "minmaxlttb":
        return oracle_mod.minmaxlttb(yh, n_out, ratio)
    return getattr(oracle_mod, algo)(yh, n_out)


@pytest.mark.parametrize("stage", [-1, 1], ids=["auto", "staged"])
def test_beyond_2_31_bit_exact(oracle_mod, big, stage):
    import paper_2307_05389_amd as ts
    dtype, yd, yh = big
    # the oracle runs in threads (it releases the interpreter lock) while the
    # GPU computes the same cases
    with ThreadPoolExecutor(max_workers=len(CASES)) as ex:
        futs = [ex.submit(_oracle, oracle_mod, a, yh, n_out, r) for a, n_out, r in CASES]
        try:
            ts.set_tuning(stage=stage, chunk_bytes=(16384 if stage == 1 else -1))
            got = []
            for algo, n_out, ratio in CASES:
                say(f"[2^31+4097] {np.dtype(dtype).name} stage={stage} {algo} n_out={n_out} ratio={ratio}")
                got.append(_gpu(ts, algo, yd, n_out, ratio))
        finally:
            ts.set_tuning()
        for (algo, n_out, ratio), g, f in zip(CASES, got, futs):
            exp = f.result()
            assert np.array_equal(g, exp), (algo, n_out, ratio, len(g), len(exp))
            if algo == "minmax" and n_out == 2:
                # one bin: the planted extremes, both past 2^31
                assert g.tolist() == [(1 << 31) + 1000, (1 << 31) + 3000]
            assert g.max() < N
    assert int(np.count_nonzero(np.asarray(got[2]) >= (1 << 31))) > 0

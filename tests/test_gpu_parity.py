"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element
by element, on seeded inputs.  MinMax, M4 and the MinMaxLTTB preselection
must match bit-exactly; LTTB picks are compared exactly and through the
step-wise near-tie rule as the stated tolerance."""
import numpy as np
import pytest
import torch

import synthetic as S
from lttb_check import stepwise_check

pytestmark = pytest.mark.gpu

ALL = [np.int8, np.int16, np.int32, np.int64, np.uint8, np.uint16, np.uint32, np.uint64,
       np.float16, np.float32, np.float64]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module")
def ts():
    import paper_2307_05389_amd as t
    t.set_tuning()
    yield t
    t.set_tuning()


def say(*a):
    print(*a, flush=True)


def gpu(ts, algo, y, n_out, x=None, ratio=4):
    yd, xd = dev(y), (None if x is None else dev(x))
    if algo == "minmaxlttb":
        r = ts.minmaxlttb(yd, n_out, x=xd, minmax_ratio=ratio)
    else:
        r = getattr(ts, algo)(yd, n_out, x=xd)
    torch.cuda.synchronize()
    return r.cpu().numpy()


def orc(oracle_mod, algo, y, n_out, x=None, ratio=4):
    if algo == "minmaxlttb":
        return oracle_mod.minmaxlttb(y, n_out, ratio, x=x)
    return getattr(oracle_mod, algo)(y, n_out, x=x)


def xs_for(n, seed):
    rng = np.random.default_rng(seed)
    g = S.timestamps(n, 1000, seed=seed)
    gap = g.copy()
    if n > 10:
        gap[n // 3:] += 10**7          # empty bins
        gap[2 * n // 3: 2 * n // 3 + 5] = gap[2 * n // 3]   # duplicates
        gap = np.maximum.accumulate(gap)
    return {
        "none": None,
        "i64": gap,
        "i32": (g % (2**31 - 1)).astype(np.int32) if g[-1] < 2**31 else None,
        "u64": gap.astype(np.uint64) + np.uint64(2**63),
        "f64": np.sort(rng.random(n) * 1e6),
        "f32": np.sort(rng.random(n).astype(np.float32) * np.float32(1e4)),
    }


@pytest.mark.parametrize("dtype", ALL, ids=lambda d: np.dtype(d).name)
@pytest.mark.parametrize("algo", ["minmax", "m4"])
def test_parity_matrix(ts, oracle_mod, algo, dtype):
    for n in (1000, 33333, 300001):
        y = S.walk(n, dtype, seed=n % 97)
        for xname, x in xs_for(n, n % 89).items():
            if x is None and xname != "none":
                continue
            for n_out in (4, 100, 1000, 8000):
                say(f"[parity] {algo} {np.dtype(dtype).name} n={n} x={xname} n_out={n_out}")
                got = gpu(ts, algo, y, n_out, x)
                exp = orc(oracle_mod, algo, y, n_out, x)
                assert np.array_equal(got, exp), (algo, dtype, n, xname, n_out)


@pytest.mark.parametrize("algo", ["minmax", "m4", "lttb", "minmaxlttb"])
def test_edge_sizes(ts, oracle_mod, algo):
    for dtype in ALL:
        for n in (0, 1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 63, 64, 65):
            y = S.walk(n, dtype, seed=3) if n else np.zeros(0, dtype)
            for n_out in (4, 8, 12, 16):
                if algo == "minmaxlttb" and n_out * 4 % 2:
                    continue
                say(f"[edge] {algo} {np.dtype(dtype).name} n={n} n_out={n_out}")
                got = gpu(ts, algo, y, n_out)
                exp = orc(oracle_mod, algo, y, n_out)
                assert np.array_equal(got, exp), (algo, dtype, n, n_out, got, exp)


def _tie_cases(n):
    rng = np.random.default_rng(1)
    base = rng.integers(0, 3, n)
    return {
        "f64_zeros": np.where(base == 0, -0.0, np.where(base == 1, 0.0, 1.0)),
        "f32_inf": np.where(base == 0, -np.inf, np.where(base == 1, 0.0, np.inf)).astype(np.float32),
        "f16_zeros": np.where(base == 0, -0.0, np.where(base == 1, 0.0, -1.0)).astype(np.float16),
        "i64_ext": np.where(base == 0, np.iinfo(np.int64).min, np.where(base == 1, 0, np.iinfo(np.int64).max)),
        "u64_ext": np.where(base == 0, 0, np.where(base == 1, 1, 2**64 - 1)).astype(np.uint64),
        "i8_ext": np.where(base == 0, -128, np.where(base == 1, 0, 127)).astype(np.int8),
        "const": np.full(n, 7, np.int16),
    }


def test_ties_signed_zero_and_extremes(ts, oracle_mod):
    cases = _tie_cases(200003)
    for name, y in cases.items():
        for algo in ("minmax", "m4"):
            for n_out in (2 if algo == "minmax" else 4, 40, 4000, 100000):
                say(f"[ties] {name} {algo} n_out={n_out}")
                assert np.array_equal(gpu(ts, algo, y, n_out), orc(oracle_mod, algo, y, n_out)), (name, algo, n_out)


@pytest.mark.parametrize("mode", [1, 2])
def test_ties_per_bin_modes(ts, oracle_mod, mode):
    """The tie and extreme-value cases with a wavefront per bin (mode 1) and
    a workgroup of four per bin (mode 2, where the wavefronts' results meet
    in LDS): the first index of a tie and -0 / +0 order must survive both."""
    cases = _tie_cases(200003)
    try:
        ts.set_tuning(direct=mode)
        for name, y in cases.items():
            for algo in ("minmax", "m4"):
                for n_out in (2 if algo == "minmax" else 4, 40, 4000):
                    say(f"[ties mode={mode}] {name} {algo} n_out={n_out}")
                    assert np.array_equal(gpu(ts, algo, y, n_out), orc(oracle_mod, algo, y, n_out)), (name, algo, n_out)
    finally:
        ts.set_tuning()


@pytest.mark.parametrize("chunk,small,stage,xclass",
                         [(4096, -1, 0, -1), (4096, 1, 0, -1), (65536, 100000, 0, -1), (8192, 7, 0, -1),
                          (-1, 1 << 20, 0, -1), (8192, -1, 1, -1), (4096, -1, 1, -1), (32768, -1, 1, -1),
                          (-1, -1, -1, -1), (4096, -1, 0, 1), (65536, 7, 0, 1), (-1, -1, 0, 0)])
def test_tuning_does_not_change_results(ts, oracle_mod, chunk, small, stage, xclass):
    """Chunk size, the one-lane-per-bin threshold, LDS staging and x
    classification only change the work split (bins split over many chunks,
    many bins per wavefront, bins reduced from LDS, bins found from x)."""
    ts.set_tuning(chunk, small, -1, stage, xclass)
    try:
        for dtype in (np.float32, np.uint8, np.float64, np.int16):
            y = S.walk(250007, dtype, seed=5)
            x = S.timestamps(250007, 50, seed=6)
            for algo, n_out in (("minmax", 2), ("minmax", 600), ("m4", 40000), ("m4", 8)):
                for xx in (None, x):
                    say(f"[tuning] chunk={chunk} small={small} stage={stage} xclass={xclass} "
                        f"{np.dtype(dtype).name} {algo} {n_out}")
                    assert np.array_equal(gpu(ts, algo, y, n_out, xx), orc(oracle_mod, algo, y, n_out, xx))
    finally:
        ts.set_tuning()


@pytest.mark.parametrize("dtype", [np.uint8, np.int8, np.int16, np.float16, np.uint32, np.float32, np.float64,
                                   np.int64, np.uint64])
def test_streamed_chunks(ts, oracle_mod, dtype):
    """The scan variant that walks each chunk's tiles once, in order, and
    folds every tile into the bin segments it overlaps: bins of one element
    to several chunks, chunks of 4, 16 and 64 KB and the default, the one-lane
    threshold on and off, with and without x, series starting off the
    16-byte grid."""
    n = 200_003
    y = S.walk(n, dtype, seed=71)
    x = S.timestamps(n, 30, seed=72)
    try:
        for chunk in (-1, 4096, 16384, 65536):
            for small in (-1, 1):
                ts.set_tuning(chunk, small, 4, 0, 0)
                for off in (0, 3):
                    yd = dev(y)[off:]
                    for xx in (None, x[off:]):
                        xd = None if xx is None else dev(xx)
                        for algo, n_out in (("minmax", 2), ("minmax", 40), ("minmax", 2000), ("m4", 400),
                                            ("m4", 40000), ("minmax", 200000), ("minmaxlttb", 1000)):
                            say(f"[stream] {np.dtype(dtype).name} chunk={chunk} small={small} off={off} "
                                f"x={xx is not None} {algo} {n_out}")
                            if algo == "minmaxlttb":
                                got = ts.minmaxlttb(yd, n_out, x=xd, minmax_ratio=4)
                            else:
                                got = getattr(ts, algo)(yd, n_out, x=xd)
                            torch.cuda.synchronize()
                            want = orc(oracle_mod, algo, y[off:], n_out, xx)
                            assert np.array_equal(got.cpu().numpy(), want), (algo, n_out, chunk, small, off)
    finally:
        ts.set_tuning()


def _direct_cases(ts, oracle_mod, y, x, off, tag):
    n = len(y)
    yd = dev(y)[off:]
    for xx in (None, x[off:]):
        xd = None if xx is None else dev(xx)
        for algo, n_out in (("minmax", 2), ("m4", 4), ("minmax", 600), ("m4", 4000), ("minmax", 100000),
                            ("minmax", 2 * n), ("minmaxlttb", 1000)):
            say(f"[direct] {tag} off={off} x={xx is not None} {algo} {n_out}")
            if algo == "minmaxlttb":
                got = ts.minmaxlttb(yd, n_out, x=xd, minmax_ratio=4)
            else:
                got = getattr(ts, algo)(yd, n_out, x=xd)
            torch.cuda.synchronize()
            want = orc(oracle_mod, algo, y[off:], n_out, xx, 4)
            assert np.array_equal(got.cpu().numpy(), want), (algo, n_out, off)


@pytest.mark.parametrize("dtype", [np.uint8, np.int8, np.int16, np.float16, np.float32, np.int32, np.float64,
                                   np.uint64])
def test_direct_bins(ts, oracle_mod, dtype):
    """One wavefront, or one workgroup of four, per bin reducing the whole bin
    (no chunks, no merge): forced on for bins of one element to the whole
    series, with and without x, off the 16-byte grid; and chosen
    automatically for series without x above the small-series limit (a
    wavefront for >= 2000 bins of a few kilobytes, a workgroup for 500-1999
    bins, 250-1999 for eight-byte types, of >= 256 KB)."""
    n = 300_007
    y = S.walk(n, dtype, seed=81)
    S.tie_runs(y, 0.1, seed=82)
    x = S.timestamps(n, 40, seed=83)
    try:
        for mode in (1, 2):                  # a wavefront per bin, a workgroup per bin
            for variant in (-1, 0, 1, 2, 3):     # the automatic tile shape, then each shape
                ts.set_tuning(direct=mode, scan_variant=variant)
                for off in ((0, 5) if variant == -1 else (5,)):
                    _direct_cases(ts, oracle_mod, y, x, off, f"{np.dtype(dtype).name} mode={mode} variant={variant}")
    finally:
        ts.set_tuning()
    # automatic choice: > 8 MB, no x, >= 2000 bins of 4-512 KB; 500-1999 bins
    # (eight-byte types 250-1999) of >= 256 KB: a workgroup per bin
    from paper_2307_05389_amd import _lib as L
    es = np.dtype(dtype).itemsize
    nbig = (16 << 20) // es + 13
    ybig = S.walk(nbig, dtype, seed=84)
    for bin_bytes in (4096, 5000, 8192):
        nb = nbig * es // bin_bytes
        if nb < 2000:
            continue
        assert L.scan_config(dev(ybig[:8]).dtype, nbig, nb)[2].startswith("tsds::k_bins_direct<")
        for algo, per in (("minmax", 2), ("m4", 4)):
            say(f"[direct auto] {np.dtype(dtype).name} bin_bytes={bin_bytes} {algo}")
            assert np.array_equal(gpu(ts, algo, ybig, per * nb), orc(oracle_mod, algo, ybig, per * nb))
    if dtype in (np.uint8, np.float32, np.float64):
        nbb = 503
        n8 = nbb * (256 << 10) // es + 7
        y8 = S.walk(n8, dtype, seed=85)
        S.tie_runs(y8, 0.05, seed=86)
        td = dev(y8[:8]).dtype
        assert L.scan_config(td, n8, nbb)[2].startswith("tsds::k_bins_block<")
        assert L.scan_config(td, n8, 4 * nbb)[2].startswith("tsds::k_bins_direct<")  # 64 KB bins: a wave each
        assert not L.scan_config(td, n8 // 2, nbb)[2].startswith("tsds::k_bins")  # 128 KB bins: chunks
        assert L.scan_config(td, n8, 499)[2].startswith("tsds::k_bins_block<") == (es == 8)
        assert not L.scan_config(td, n8, 249)[2].startswith("tsds::k_bins_block<")
        for algo, per in (("minmax", 2), ("m4", 4)):
            say(f"[block auto] {np.dtype(dtype).name} {nbb} bins of 256 KB {algo}")
            assert np.array_equal(gpu(ts, algo, y8, per * nbb), orc(oracle_mod, algo, y8, per * nbb))
        say(f"[block auto] {np.dtype(dtype).name} minmaxlttb 2 * {nbb}")
        assert np.array_equal(gpu(ts, "minmaxlttb", y8, 2 * nbb), orc(oracle_mod, "minmaxlttb", y8, 2 * nbb))


def x_patterns(n, seed):
    """int64 x layouts that stress finding bins from x: steady timestamps,
    long gaps (runs of empty bins, some spanning many chunks), runs of equal
    timestamps across chunk ends, one constant value (every point in the last
    bin), and a range close to the whole int64 span."""
    rng = np.random.default_rng(seed)
    steady = S.timestamps(n, 1000, seed=seed)
    gaps = steady.copy()
    for k in range(1, 6):
        gaps[k * n // 6:] += rng.integers(1, 10**9)
    dup = np.repeat(S.timestamps((n + 4095) // 4096 * 8, 50, seed=seed + 1), 512)[:n]
    wide = np.sort(rng.integers(np.iinfo(np.int64).min // 2 * 2 + 1, np.iinfo(np.int64).max, n, dtype=np.int64))
    wide[0], wide[-1] = np.iinfo(np.int64).min + 1, np.iinfo(np.int64).max
    return {"steady": steady, "gaps": gaps, "dup": dup.astype(np.int64),
            "const": np.full(n, -123456789, np.int64), "wide": wide}


@pytest.mark.parametrize("xclass", [1, 0])
def test_x_classified_chunks(ts, oracle_mod, xclass):
    """Chunks that find their bins from int64 x give the same bins (and the
    same edge array) as the separate edge search, for any bin length: many
    boundaries per chunk, none, and runs of empty bins."""
    ts.set_tuning(-1, -1, -1, 0, xclass)
    try:
        for n in (1, 2, 4097, 300001):
            xs = x_patterns(n, seed=n)
            for dtype in (np.float64, np.float32, np.int16, np.uint8):
                y = S.walk(n, dtype, seed=n + 3)
                for name, x in xs.items():
                    for algo, n_out in (("m4", 4), ("m4", 40), ("minmax", 1000), ("m4", 4000), ("minmax", 2 * n + 2)):
                        say(f"[xclass={xclass}] n={n} {np.dtype(dtype).name} x={name} {algo} {n_out}")
                        assert np.array_equal(gpu(ts, algo, y, n_out, x), orc(oracle_mod, algo, y, n_out, x)), \
                            (n, name, algo, n_out)
                if n > 2:
                    for name in ("gaps", "dup"):
                        say(f"[xclass={xclass}] n={n} {np.dtype(dtype).name} x={name} minmaxlttb")
                        got = gpu(ts, "minmaxlttb", y, 200, xs[name], 4)
                        assert np.array_equal(got, orc(oracle_mod, "minmaxlttb", y, 200, xs[name], 4)), (n, name)
    finally:
        ts.set_tuning()


def test_staged_vectors_ties(ts, oracle_mod):
    """LDS-staged chunks with whole vectors per lane (bins of at least a
    vector per lane): signed zeros, infinities and integer extremes repeat
    across the lanes of a group and across vectors, so the first occurrence
    rests on the (value, vector) reduction and the in-vector search."""
    cases = _tie_cases(100003)
    ts.set_tuning(-1, -1, -1, 1, -1)
    try:
        for name, y in cases.items():
            for avg in (70, 300, 2000):
                for algo, per in (("minmax", 2), ("m4", 4)):
                    n_out = per * (len(y) // avg)
                    say(f"[staged ties] {name} avg={avg} {algo} n_out={n_out}")
                    assert np.array_equal(gpu(ts, algo, y, n_out), orc(oracle_mod, algo, y, n_out)), (name, avg)
    finally:
        ts.set_tuning()


@pytest.mark.parametrize("dtype", ALL)
def test_staged_lanes_per_bin(ts, oracle_mod, dtype):
    """LDS-staged chunks reduce a bin with 1, 4, 16 or 64 lanes depending on
    the bin length; every width must give the first occurrence, also when
    the extreme repeats across the lanes of one group (tie runs)."""
    n = 120011
    y = S.walk(n, dtype, seed=41)
    S.tie_runs(y, 0.3, seed=42)
    ts.set_tuning(-1, -1, -1, 1, -1)
    try:
        for avg in (3, 30, 150, 700, 3000):
            for algo, per in (("minmax", 2), ("m4", 4)):
                n_out = per * max(1, n // avg)
                say(f"[staged] {np.dtype(dtype).name} avg={avg} {algo} n_out={n_out}")
                assert np.array_equal(gpu(ts, algo, y, n_out), orc(oracle_mod, algo, y, n_out)), (avg, algo)
    finally:
        ts.set_tuning()


@pytest.mark.parametrize("dtype", [np.float32, np.uint8, np.int64, np.float16])
def test_many_bins_compaction(ts, oracle_mod, dtype):
    """Above 4,096 bins the compaction runs over many workgroups (block sums,
    then the writes, each workgroup summing the block sums in front of it; the
    scan of the block sums in a launch of its own above 512 workgroups),
    1,024 bins per workgroup; n <= n_out fills 0..n-1 from many workgroups.
    Bin counts around the limits."""
    if dtype == np.float32:
        n2 = 1_200_007
        y2 = S.walk(n2, dtype, seed=53)
        for algo, n_out in (("minmax", 1_100_000), ("minmax", 2 * 512 * 1024), ("minmax", 2 * (512 * 1024 + 1))):
            say(f"[many bins] {np.dtype(dtype).name} {algo} {n_out} (n={n2})")
            assert np.array_equal(gpu(ts, algo, y2, n_out), orc(oracle_mod, algo, y2, n_out))
    n = 1_000_003
    y = S.walk(n, dtype, seed=51)
    x = S.timestamps(n, 40, seed=52)
    for xx in (None, x):
        for algo, n_out in (("minmax", 300_000), ("m4", 400_000), ("minmax", 131_074), ("m4", 1_600_000),
                            ("minmax", 8192), ("minmax", 8194), ("m4", 16392), ("minmax", 2 * 5121),
                            ("m4", 4 * 1023)):
            say(f"[many bins] {np.dtype(dtype).name} x={xx is not None} {algo} {n_out}")
            assert np.array_equal(gpu(ts, algo, y, n_out, xx), orc(oracle_mod, algo, y, n_out, xx))
        say(f"[many bins] {np.dtype(dtype).name} x={xx is not None} minmaxlttb 40000")
        assert np.array_equal(gpu(ts, "minmaxlttb", y, 40_000, xx, 4), orc(oracle_mod, "minmaxlttb", y, 40_000, xx, 4))


@pytest.mark.parametrize("dtype", [np.int8, np.float16, np.float32, np.float64, np.int64])
def test_misaligned_series_pointer(ts, oracle_mod, dtype):
    """Slices start at any element: the scan realigns to 16-byte vectors."""
    y = S.walk(100000, dtype, seed=9)
    yd = dev(y)
    for off in range(0, 17):
        sub = yd[off:]
        for algo, n_out in (("minmax", 200), ("m4", 400)):
            say(f"[align] {np.dtype(dtype).name} off={off} {algo}")
            got = getattr(ts, algo)(sub, n_out).cpu().numpy()
            assert np.array_equal(got, orc(oracle_mod, algo, y[off:], n_out))


def test_cross_dtype_consistency(ts):
    y0 = np.clip(np.rint(S.walk(150000, np.float64, seed=21) / 20), -60, 120)
    for algo, n_out in (("minmax", 1000), ("m4", 1000), ("minmaxlttb", 500), ("lttb", 500)):
        base = gpu(ts, algo, y0.astype(np.float64), n_out)
        for dt in ALL:
            yy = y0 + (60 if np.dtype(dt).kind == "u" else 0)
            say(f"[xdtype] {algo} {np.dtype(dt).name}")
            assert np.array_equal(gpu(ts, algo, yy.astype(dt), n_out), base), (algo, dt)


def test_determinism_repeat(ts):
    y = dev(S.walk(3_000_001, np.float32, seed=22))
    for algo, n_out in (("minmax", 1000), ("m4", 2000), ("minmaxlttb", 1000), ("lttb", 1000)):
        r1 = getattr(ts, algo)(y, n_out).cpu()
        r2 = getattr(ts, algo)(y, n_out).cpu()
        assert torch.equal(r1, r2)


def test_bin_edges_and_argminmax_steps(ts, oracle_mod):
    n = 123457
    y = S.walk(n, np.float32, seed=23)
    x = S.timestamps(n, 700, seed=24)
    for nb in (1, 3, 500, 4000):
        for xx in (None, x, x.astype(np.float64)):
            say(f"[edges] nb={nb} x={None if xx is None else xx.dtype}")
            e = ts.bin_edges(dev(y), nb, None if xx is None else dev(xx)).cpu().numpy()
            assert np.array_equal(e, oracle_mod.edges(n, nb, xx))
    # caller edges that skip a prefix/suffix and include empty bins
    edges = np.array([10, 10, 500, 501, 70000, 70000, 123000], np.int64)
    imin, imax = ts.bin_argminmax(dev(y), dev(edges))
    for b in range(len(edges) - 1):
        lo, hi = edges[b], edges[b + 1]
        if lo == hi:
            assert imin[b].item() == -1 and imax[b].item() == -1
        else:
            assert (imin[b].item(), imax[b].item()) == oracle_mod.argminmax(y, lo, hi)


def test_window(ts, oracle_mod):
    x = S.timestamps(1_000_003, 100, seed=25)
    xd = dev(x)
    rng = np.random.default_rng(26)
    for _ in range(50):
        a, b = sorted(int(v) for v in rng.integers(-1000, int(x[-1]) + 1000, 2))
        r = ts.window(xd, a, b).cpu().numpy()
        assert tuple(r) == oracle_mod.window(x, a, b)


# ------------------------------------------------------------------ LTTB


@pytest.mark.parametrize("dtype", [np.float32, np.float64, np.int32, np.uint8, np.float16, np.int64])
@pytest.mark.parametrize("with_x", [False, True])
def test_lttb_parity(ts, oracle_mod, dtype, with_x):
    for n, n_out in ((1000, 10), (50000, 1000), (200001, 3), (20000, 4000), (777, 776)):
        y = S.walk(n, dtype, seed=n % 31)
        x = S.timestamps(n, 30, seed=7) if with_x else None
        say(f"[lttb] {np.dtype(dtype).name} x={with_x} n={n} n_out={n_out}")
        got = gpu(ts, "lttb", y, n_out, x)
        exp = orc(oracle_mod, "lttb", y, n_out, x)
        near = stepwise_check(oracle_mod, y, n_out, got, x=x)
        assert near == 0 and np.array_equal(got, exp)


@pytest.mark.parametrize("n,n_out", [
    (10, 3),                  # one group: one chain
    (300, 102),               # two-level chain, entries in LDS
    (2_000_000, 200_002),     # > 2,048 groups (entries in the workspace), two-level chain
    (32_000_000, 1_000_002),  # buckets of 32: too many super-group entries for LDS, one chain
])
def test_lttb_small_walk_levels(ts, oracle_mod, n, n_out):
    """The small-bucket walk's group chain in each of its forms, bit-exact."""
    y = S.walk(n, np.float32, seed=n % 97)
    say(f"[lttb walk] n={n} n_out={n_out}")
    got = gpu(ts, "lttb", y, n_out)
    assert np.array_equal(got, orc(oracle_mod, "lttb", y, n_out))


def hull_cases(n, dtype, seed):
    """Series for the hull-pruned LTTB walk: a random walk, the same with long
    constant runs (exact area ties), a constant series (every area zero) and
    a parabola (every point on the hull, so slices overflow and buckets are
    walked in full)."""
    walk = S.walk(n, dtype, seed=seed)
    ties = S.tie_runs(S.walk(n, dtype, seed=seed + 1), 0.5, seed=seed + 2, lmin=600, lmax=5000)
    j = np.arange(n, dtype=np.float64)
    if np.issubdtype(dtype, np.floating):
        par = ((j - n / 2) ** 2 / (4 * n)).astype(dtype)  # below 25,001: finite in float16
    else:
        par = (((j % 2000) - 1000) ** 2 // 64).astype(dtype)
    mixed = walk.copy()
    mixed[n // 2:] = par[n // 2:]  # some buckets pruned, some walked in full
    # convex bumps of 64 points on a walk: slice hulls overflow and are re-read
    bumps = (S.walk(n, np.float64, seed=seed + 3) * 50 + ((j % 64) - 32) ** 2).astype(dtype) \
        if np.issubdtype(dtype, np.floating) or np.dtype(dtype).itemsize >= 4 else walk
    return {"walk": walk, "ties": ties, "const": np.full(n, 3, dtype), "parabola": par, "mixed": mixed,
            "bumps": bumps}


@pytest.mark.parametrize("dtype", [np.float32, np.float64, np.int16, np.uint8, np.float16, np.int64])
def test_lttb_hull_walk(ts, oracle_mod, dtype):
    """Plain LTTB with buckets of at least 512 points walks only each bucket's
    convex-hull vertices and first point.  Step by step against the oracle:
    the same pick except near ties of the stated tolerance."""
    n = 400_003
    xs = {"none": None,
          "i64dup": np.repeat(S.timestamps((n + 2) // 3, 50, seed=64), 3)[:n],
          "f64": S.timestamps(n, 20, seed=65).astype(np.float64) * 0.25}
    for name, y in hull_cases(n, dtype, seed=66).items():
        for xname, x in xs.items():
            for n_out in (500, 100, 3):
                say(f"[lttb hull] {np.dtype(dtype).name} {name} x={xname} n_out={n_out}")
                got = gpu(ts, "lttb", y, n_out, x)
                near = stepwise_check(oracle_mod, y, n_out, got, x=x)
                say(f"    near-tie acceptances: {near}")
                # the hull keeps every point that can reach the maximum, so the
                # walk is the oracle's step for step, with no tolerance used
                assert near == 0 and np.array_equal(got, orc(oracle_mod, "lttb", y, n_out, x))
    y = S.walk(100_000, dtype, seed=67)
    say(f"[lttb hull] {np.dtype(dtype).name} MinMaxLTTB keeping every point")
    got = gpu(ts, "minmaxlttb", y, 150, None, 1000)
    near = stepwise_check(oracle_mod, y, 150, got)
    say(f"    near-tie acceptances: {near}")
    assert near == 0


@pytest.mark.parametrize("dtype", [np.float32, np.float64, np.int16, np.uint8, np.float16])
@pytest.mark.parametrize("xname", ["none", "i64", "f64"])
def test_minmaxlttb_parity(ts, oracle_mod, dtype, xname):
    # (1_000_003, 3000, 4) and (500_000, 3966, 4): the walk's maps take 96 KB
    # and 124 KB of LDS; (500_000, 3970, 4): just over, maps in global memory
    for n, n_out, ratio in ((100000, 500, 4), (1_000_003, 2000, 4), (30000, 1000, 8), (5000, 1000, 4),
                            (4000, 1000, 4), (250000, 3, 2), (1_000_003, 3000, 4), (500_000, 3966, 4),
                            (500_000, 3970, 4)):
        y = S.walk(n, dtype, seed=n % 13)
        x = xs_for(n, 3)[xname]
        say(f"[mmlttb] {np.dtype(dtype).name} x={xname} n={n} n_out={n_out} r={ratio}")
        got = gpu(ts, "minmaxlttb", y, n_out, x, ratio)
        exp = orc(oracle_mod, "minmaxlttb", y, n_out, x, ratio)
        assert np.array_equal(got, exp), (dtype, xname, n, n_out)


def test_lttb_centres_bit_exact(ts, oracle_mod):
    for dtype in (np.float32, np.float64, np.int32, np.uint64):
        y = S.walk(100003, dtype, seed=27)
        x = S.timestamps(100003, 10, seed=28)
        for xx in (None, x, x.astype(np.float64)):
            cx, cy = ts.lttb_centres(dev(y), 700, None if xx is None else dev(xx))
            ecx, ecy = oracle_mod.lttb_centres(y, 700, x=xx)
            assert np.array_equal(cx.cpu().numpy(), ecx) and np.array_equal(cy.cpu().numpy(), ecy)


def _bits_equal(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return a.shape == b.shape and np.array_equal(a.view(np.uint64), b.view(np.uint64))


def _centre_cases(n, seed):
    """Float series whose bucket sums are exact in some tiles and rounded in
    others: a walk crossing zero (tiny values beside large partial sums),
    full-mantissa float64 noise (every tile rounds), mixed magnitudes, exact
    small integers, all negative zeros, and +-inf (a NaN centre)."""
    rng = np.random.default_rng(seed)
    walk = S.walk(n, np.float32, seed=seed)
    noise = rng.standard_normal(n)
    mixed = np.where(rng.random(n) < 0.5, 1e30, 1e-30).astype(np.float32) * np.sign(rng.standard_normal(n))
    mixed = mixed.astype(np.float32)
    ints = rng.integers(-1000, 1000, n).astype(np.float32)
    zeros = np.full(n, -0.0, np.float32)
    infs = walk.copy()
    infs[n // 3] = np.inf
    infs[n // 3 + 5] = -np.inf
    infs[2 * n // 3] = np.inf
    halves = S.walk(n, np.float16, seed=seed + 1)
    return {"walk": walk, "noise64": noise, "mixed": mixed, "ints": ints, "zeros": zeros, "infs": infs,
            "halves": halves}


@pytest.mark.parametrize("n,n_out", [(2_000_003, 60), (3_000_017, 1000), (1_300_021, 5)])
def test_lttb_long_bucket_centres_bit_exact(ts, oracle_mod, n, n_out):
    """Centres of long buckets (a workgroup per bucket, tile summaries folded
    into the sequential sum where no rounding can occur, point by point where
    it can): bit-identical to the oracle's index-order double sums, signed
    zeros and NaN included, with and without float x; buckets of ~33k, ~3k
    and ~433k points (several rounds of tile summaries)."""
    rng = np.random.default_rng(n)
    xs = {"none": None, "f64": S.timestamps(n, 10, seed=n).astype(np.float64),
          "f32": (np.cumsum(rng.integers(1, 4, n)) * 0.125).astype(np.float32)}
    for name, y in _centre_cases(n, seed=n % 1000).items():
        for xn, xx in xs.items():
            say(f"[centres] n={n} n_out={n_out} y={name} x={xn}")
            cx, cy = ts.lttb_centres(dev(y), n_out, None if xx is None else dev(xx))
            ecx, ecy = oracle_mod.lttb_centres(y, n_out, x=xx)
            assert _bits_equal(cy.cpu().numpy(), ecy), (name, xn)
            assert _bits_equal(cx.cpu().numpy(), ecx), (name, xn)
        if name in ("walk", "noise64", "mixed"):
            say(f"[centres] lttb n={n} n_out={n_out} y={name}")
            assert np.array_equal(gpu(ts, "lttb", y, n_out), oracle_mod.lttb(y, n_out))


# ------------------------------------------------------------------ errors


def test_error_paths(ts):
    from paper_2307_05389_amd import TsArgError, TsError
    y = dev(S.walk(10000, np.float32, seed=1))
    with pytest.raises(TsArgError):
        ts.minmax(y, 1001)
    with pytest.raises(TsArgError):
        ts.m4(y, 10)
    with pytest.raises(TsArgError):
        ts.minmaxlttb(y, 101, minmax_ratio=1)
    out = torch.empty(100, dtype=torch.int64, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    small_ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(TsError) as ei:
        ts.downsample_into("minmax", y, 100, out, cnt, workspace=small_ws)
    assert ei.value.code == -4
    # nothing was written on error
    out.fill_(-7)
    with pytest.raises(TsError):
        ts.downsample_into("m4", y, 100, out, cnt, workspace=small_ws)
    torch.cuda.synchronize()
    assert bool((out == -7).all())


def test_lttb_in_a_captured_graph(ts, oracle_mod):
    """Plain LTTB with long buckets forks its centres onto a side stream and
    joins them back; captured in a graph (first call inside the capture, and
    after an eager call created the side stream) every replay equals the
    eager result and the oracle, with eager work and synchronisation between
    replays."""
    n, n_out = 3_000_017, 200
    y = S.walk(n, np.float32, seed=95)
    yd = dev(y)
    want = oracle_mod.lttb(y, n_out)
    for eager_first in (False, True):
        out = torch.full((n_out,), -1, dtype=torch.int64, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        need = ts.workspace_bytes("lttb", yd, n_out)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        side = torch.cuda.Stream()
        if eager_first:
            with torch.cuda.stream(side):
                ts.downsample_into("lttb", yd, n_out, out, cnt, workspace=ws)
            torch.cuda.synchronize()
            assert np.array_equal(out[: int(cnt.item())].cpu().numpy(), want)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            ts.downsample_into("lttb", yd, n_out, out, cnt, workspace=ws, stream=torch.cuda.current_stream())
        for rep in range(3):
            say(f"[lttb graph] eager_first={eager_first} replay {rep}")
            out.fill_(-1)
            g.replay()
            torch.cuda.synchronize()
            assert int(cnt.item()) == n_out and np.array_equal(out.cpu().numpy(), want), rep
            junk = torch.randn(1 << 20, device="cuda").sum()
            del junk

"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value comes
from a brute-force restatement (tests/brute.py: per-point bin ids, numpy
argmin/argmax, exact rational LTTB), from an identity the paper states
(equally sampled x == no x, Sec. 2.2), from the paper's key maps (Sec. 2.1.2),
from closed-form special cases, or from hand-worked fixtures in tests/golden.
"""
import itertools
import json
import os

import numpy as np
import pytest

import brute
import synthetic as S

ALL_DTYPES = [np.int8, np.int16, np.int32, np.int64, np.uint8, np.uint16, np.uint32, np.uint64,
              np.float16, np.float32, np.float64]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _valid_nouts(kind, n):
    hi = n + 4
    if kind == "minmax":
        return [v for v in range(2, hi + 1) if v % 2 == 0]
    return [v for v in range(4, hi + 1) if v % 4 == 0]


# ------------------------------------------------------------ exhaustive tiny


@pytest.mark.parametrize("alphabet", [
    np.array([0, 1, 2], np.int64),
    np.array([-0.0, 0.0, 1.0], np.float64),
    np.array([-np.inf, 0.0, np.inf], np.float64),
    np.array([np.iinfo(np.int64).min, 0, np.iinfo(np.int64).max], np.int64),
])
def test_exhaustive_tiny_no_x(oracle_mod, alphabet):
    for n in range(0, 7):
        for combo in itertools.product(range(len(alphabet)), repeat=n):
            y = alphabet[list(combo)] if n else alphabet[:0]
            for kind in ("minmax", "m4"):
                for n_out in _valid_nouts(kind, n):
                    got = getattr(oracle_mod, kind)(y, n_out)
                    exp = getattr(brute, kind)(y, n_out)
                    assert np.array_equal(got, exp), (kind, y, n_out, got, exp)


def test_exhaustive_tiny_int_x(oracle_mod):
    rng = np.random.default_rng(5)
    for n in range(1, 9):
        for trial in range(60):
            # sorted x with duplicates and gaps, including all-equal x
            x = np.sort(rng.integers(-5, 20, n)).astype(np.int64)
            if trial % 10 == 0:
                x[:] = x[0]
            y = rng.integers(0, 3, n).astype(np.int32)
            for kind in ("minmax", "m4"):
                for n_out in _valid_nouts(kind, n):
                    got = getattr(oracle_mod, kind)(y, n_out, x=x)
                    exp = getattr(brute, kind)(y, n_out, x=x)
                    assert np.array_equal(got, exp), (kind, x, y, n_out, got, exp)


def test_edges_match_per_point_bins(oracle_mod):
    rng = np.random.default_rng(6)
    for _ in range(300):
        n = int(rng.integers(1, 400))
        nb = int(rng.integers(1, 60))
        ids = brute.bin_ids_nox(n, nb)
        exp = np.array([np.searchsorted(ids, b, "left") for b in range(nb)] + [n])
        assert np.array_equal(oracle_mod.edges(n, nb), exp), (n, nb)
        x = np.cumsum(rng.integers(0, 50, n)).astype(np.int64) - 300
        ids = brute.bin_ids_int_x(x, nb)
        exp = np.array([np.searchsorted(ids, b, "left") for b in range(nb)] + [n])
        for xd in (np.int64, np.int32):
            assert np.array_equal(oracle_mod.edges(n, nb, x.astype(xd)), exp), (n, nb, xd)
        xu = (x - x.min()).astype(np.uint64) + np.uint64(2**63)
        assert np.array_equal(oracle_mod.edges(n, nb, xu), exp)


def test_float_x_edges_agree_with_exact_bins_away_from_edges(oracle_mod):
    """Float x: each point's bin agrees with the exact rational bin
    floor((x - x0) nb / R) except where x lies within a few ulps of an edge
    (the rounding of the edge value decides there)."""
    from fractions import Fraction
    rng = np.random.default_rng(7)
    for _ in range(40):
        n = int(rng.integers(2, 300))
        nb = int(rng.integers(1, 40))
        x = np.sort(rng.random(n) * 1000.0 - 200.0)
        e = oracle_mod.edges(n, nb, x)
        got = np.searchsorted(e, np.arange(n), "right") - 1
        x0, R = Fraction(float(x[0])), Fraction(float(x[-1])) - Fraction(float(x[0]))
        for i, v in enumerate(x):
            q = (Fraction(float(v)) - x0) * nb / R
            exact = min(int(q), nb - 1)
            frac_dist = min(q - int(q), 1 - (q - int(q))) if q < nb else 1
            if frac_dist > Fraction(1, 10**9):
                assert got[i] == exact, (i, v, got[i], exact)


# --------------------------------------------------- special cases / identities


@pytest.mark.parametrize("dtype", ALL_DTYPES)
def test_single_bin_is_global_argmin_argmax(oracle_mod, dtype):
    y = S.walk(5000, dtype, seed=11)
    got = oracle_mod.minmax(y, 2)
    assert np.array_equal(got, np.sort(np.unique([np.argmin(y), np.argmax(y)])))
    got = oracle_mod.m4(y, 4)
    assert np.array_equal(got, np.unique([0, np.argmin(y), np.argmax(y), len(y) - 1]))


def test_n_le_nout_returns_all(oracle_mod):
    for n in range(0, 12):
        y = np.arange(n, dtype=np.float32)[::-1].copy()
        for f, n_out in ((oracle_mod.minmax, 12), (oracle_mod.m4, 12), (oracle_mod.lttb, 12),
                         (oracle_mod.minmaxlttb, 12)):
            assert np.array_equal(f(y, n_out), np.arange(n))


def test_f16_all_patterns_order(oracle_mod):
    """Every non-NaN binary16 pattern: the oracle's first argmin/argmax over a
    shuffled array equals numpy's (numeric order, -0 == +0)."""
    bits = np.arange(65536, dtype=np.uint16)
    h = bits.view(np.float16)
    h = h[~np.isnan(h)]
    rng = np.random.default_rng(8)
    for _ in range(4):
        p = h[rng.permutation(len(h))]
        assert oracle_mod.argminmax(p) == (int(np.argmin(p)), int(np.argmax(p)))
    # ties between -0 and +0 resolve to the first occurrence
    z = np.array([1, -0.0, 0.0, 2, -0.0], np.float16)
    assert oracle_mod.argminmax(z) == (1, 3)


def _i16ord(v):
    """The paper's f16 ordinal map on the i16 reinterpretation (Sec. 2.1.2)."""
    v = v.astype(np.int16)
    return ((v >> 15) & np.int16(0x7FFF)) ^ v


def test_paper_i16ord_map_is_monotone_and_self_inverse():
    bits = np.arange(65536, dtype=np.uint16).view(np.int16)
    f = bits.view(np.float16)
    ok = ~np.isnan(f)
    k = _i16ord(bits)
    assert np.array_equal(_i16ord(k), bits)           # self-inverse
    fv, kv = f[ok].astype(np.float64), k[ok].astype(np.int64)
    order = np.argsort(kv, kind="stable")
    assert np.all(np.diff(fv[order]) >= 0)            # key order = numeric order
    # the map separates the two zeros: -0 gets the key just below +0
    assert _i16ord(np.array([np.float16(-0.0)]).view(np.int16))[0] == -1
    assert _i16ord(np.array([np.float16(0.0)]).view(np.int16))[0] == 0


def test_paper_uint_xor_map_is_monotone():
    for ut, it in ((np.uint8, np.int8), (np.uint16, np.int16)):
        u = np.arange(np.iinfo(ut).max + 1, dtype=np.int64).astype(ut)
        k = u.view(it) ^ np.iinfo(it).min
        assert np.all(np.diff(k.astype(np.int64)) == 1)
    rng = np.random.default_rng(9)
    for ut, it in ((np.uint32, np.int32), (np.uint64, np.int64)):
        u = np.sort(rng.integers(0, np.iinfo(ut).max, 10000, dtype=ut, endpoint=True))
        k = (u.view(it) ^ np.iinfo(it).min).astype(np.int64 if it == np.int32 else it)
        assert np.all(np.diff(k) >= 0)


@pytest.mark.parametrize("algo", ["minmax", "m4", "minmaxlttb", "lttb"])
def test_equally_sampled_x_equals_no_x(oracle_mod, algo):
    """Sec. 2.2: passing an equally sampled x gives the same output as no x."""
    rng = np.random.default_rng(10)
    f = getattr(oracle_mod, algo)
    for n in (7, 101, 1000, 4099):
        y = S.walk(n, np.float32, seed=n)
        n_out = 40 if algo != "minmaxlttb" else 20
        base = f(y, n_out)
        xs = [np.arange(n, dtype=np.int64), np.arange(n, dtype=np.int32),
              np.arange(n, dtype=np.uint64), np.arange(n, dtype=np.float64),
              np.arange(n, dtype=np.float32)]
        if algo in ("minmax", "m4"):
            k, c = int(rng.integers(2, 1000)), int(rng.integers(-10**6, 10**6))
            xs.append(np.arange(n, dtype=np.int64) * k + c)
        for x in xs:
            assert np.array_equal(f(y, n_out, x=x), base), (algo, n, x.dtype)


@pytest.mark.parametrize("algo", ["minmax", "m4", "lttb", "minmaxlttb"])
def test_cross_dtype_consistency(oracle_mod, algo):
    """Sec. 2.2: the same small-integer data in every dtype selects the same
    indices."""
    y0 = S.walk(3000, np.float64, seed=12)
    y0 = np.clip(np.rint(y0 - y0.mean()), -100, 100) + 100   # 0..200, fits u8/i8 after shift
    y0 = y0 - 60                                              # -60..140
    y0 = np.clip(y0, -60, 120)
    f = getattr(oracle_mod, algo)
    n_out = 100 if algo != "minmaxlttb" else 50
    base = f(y0.astype(np.float64), n_out)
    for dt in ALL_DTYPES:
        yy = y0 + (60 if np.dtype(dt).kind == "u" else 0)
        assert np.array_equal(f(yy.astype(dt), n_out), base), (algo, dt)


# ------------------------------------------------------------ invariants


@pytest.mark.parametrize("dtype", ALL_DTYPES)
@pytest.mark.parametrize("with_x", [False, True])
def test_minmax_m4_invariants(oracle_mod, dtype, with_x):
    n = 20011
    y = S.walk(n, dtype, seed=13)
    x = S.timestamps(n, 1000, seed=14) if with_x else None
    if with_x:
        x[5000:9000] += 0  # keep sorted
        x[6000:] += 10**7  # a large gap -> empty bins
    for nb in (1, 7, 64, 500):
        e = oracle_mod.edges(n, nb, x)
        mm = oracle_mod.minmax(y, 2 * nb, x=x)
        m4 = oracle_mod.m4(y, 4 * nb, x=x)
        for sel, per in ((mm, 2), (m4, 4)):
            assert np.all(np.diff(sel) > 0)
            assert len(sel) <= per * nb
            assert sel.min() >= 0 and sel.max() < n
        bins_mm = np.searchsorted(e, mm, "right") - 1
        for b in range(nb):
            lo, hi = e[b], e[b + 1]
            inb = m4[(m4 >= lo) & (m4 < hi)]
            if hi > lo:
                assert lo in inb and hi - 1 in inb          # M4 keeps first and last
                sub = mm[bins_mm == b]
                assert set(sub) <= set(inb)                 # M4 contains MinMax
                assert set(inb) - set(sub) <= {lo, hi - 1}
                seg = y[lo:hi]
                assert set(sub) == {lo + int(np.argmin(seg)), lo + int(np.argmax(seg))}
            else:
                assert len(inb) == 0


# ------------------------------------------------------------ LTTB


@pytest.mark.parametrize("trial", range(12))
def test_lttb_matches_exact_rational_walk(oracle_mod, trial):
    rng = np.random.default_rng(100 + trial)
    m = int(rng.integers(5, 60))
    n_out = int(rng.integers(3, m))
    kind = trial % 3
    if kind == 0:
        y = rng.integers(-20, 20, m).astype(np.int32)
        x = None
    elif kind == 1:
        y = rng.standard_normal(m)
        x = np.cumsum(rng.integers(1, 9, m)).astype(np.int64)
    else:
        y = rng.standard_normal(m).astype(np.float32)
        x = np.sort(rng.random(m) * 50).astype(np.float64)
    got = oracle_mod.lttb(y, n_out, x=x)
    exp, near = brute.lttb_exact(y, n_out, x=x)
    # identical, except that after a step whose exact top-two areas are a near
    # tie the walks may diverge legitimately
    for k in range(len(exp)):
        if got[k] != exp[k]:
            assert k >= 1 and near[k - 1], (k, got, exp)
            break


def test_lttb_constant_data_picks_first_of_each_bucket(oracle_mod):
    for m, n_out in ((50, 7), (1000, 100), (37, 36)):
        y = np.full(m, 3.0)
        nb = n_out - 2
        starts = [1 + (k * (m - 2)) // nb for k in range(nb)]
        assert np.array_equal(oracle_mod.lttb(y, n_out), np.array([0] + starts + [m - 1]))


def test_lttb_collinear_dyadic_means_picks_first(oracle_mod):
    # y = 3 i + 1 with buckets of 4 points: every centre is exact, every area is 0
    m, n_out = 2 + 4 * 30, 32
    y = (3 * np.arange(m) + 1).astype(np.int64)
    exp = [0] + [1 + 4 * k for k in range(30)] + [m - 1]
    assert np.array_equal(oracle_mod.lttb(y, n_out), np.array(exp))


def test_lttb_n_out_n_minus_1_drops_one_point(oracle_mod):
    rng = np.random.default_rng(15)
    for m in (5, 17, 200):
        y = rng.standard_normal(m)
        sel = oracle_mod.lttb(y, m - 1)
        assert len(sel) == m - 1 and sel[0] == 0 and sel[-1] == m - 1
        assert np.all(np.diff(sel) > 0)


def test_lttb_invariants_random(oracle_mod):
    for seed, (m, n_out) in enumerate(((10000, 500), (777, 13), (5000, 4998))):
        y = S.walk(m, np.float64, seed=seed)
        sel = oracle_mod.lttb(y, n_out)
        nb = n_out - 2
        assert len(sel) == n_out and sel[0] == 0 and sel[-1] == m - 1
        b = [1 + (k * (m - 2)) // nb for k in range(nb + 1)]
        for k in range(nb):
            assert b[k] <= sel[k + 1] < b[k + 1]


def test_lttb_centres_are_bucket_means(oracle_mod):
    rng = np.random.default_rng(16)
    m, n_out = 103, 12
    y = rng.integers(-1000, 1000, m).astype(np.int16)
    x = np.cumsum(rng.integers(1, 100, m)).astype(np.int64)
    cx, cy = oracle_mod.lttb_centres(y, n_out, x=x)
    nb = n_out - 2
    b = [1 + (k * (m - 2)) // nb for k in range(nb + 1)]
    from fractions import Fraction
    for k in range(nb - 1):
        lo, hi = b[k + 1], b[k + 2]
        assert cx[k] == float(Fraction(int(x[lo:hi].sum()), hi - lo))
        assert cy[k] == float(Fraction(int(y[lo:hi].astype(np.int64).sum()), hi - lo))
    assert cx[-1] == float(x[-1]) and cy[-1] == float(y[-1])


def _float_mean_cases(ydt, xdt, seed):
    """A walk in y (float dtype ydt), optional float x (xdt) that crosses zero,
    and two buckets forced to (nearly) cancel: one in y (+-A pairs plus a small
    residue) and, through x's sign change, one in x."""
    m, n_out = 20_000, 40
    y = S.walk(m, ydt, seed=seed).astype(np.float64)
    nb = n_out - 2
    b = [1 + (k * (m - 2)) // nb for k in range(nb + 1)]
    lo, hi = b[7], b[8]
    rng = np.random.default_rng(seed + 1)
    big = (1000.0 + rng.random((hi - lo) // 2) * 500.0)
    canc = np.zeros(hi - lo)
    canc[0:2 * len(big):2] = big
    canc[1:2 * len(big):2] = -big
    canc[-1] += 0.375
    y[lo:hi] = canc
    y = y.astype(ydt)
    x = None
    if xdt is not None:
        # strictly increasing, from about -m/2 to m/2 (quarter steps)
        x = ((S.timestamps(m, 3, seed=seed + 2).astype(np.float64) - 1.0 * m) * 0.25).astype(xdt)
    return y, x, n_out


def _exact_mean_and_scale(vals):
    """Exact rational mean of the doubles in vals, and the mean of their
    absolute values (the scale the mean error is measured against)."""
    from fractions import Fraction
    fr = [Fraction(float(v)) for v in vals]
    n = len(fr)
    return sum(fr, Fraction(0)) / n, sum((abs(v) for v in fr), Fraction(0)) / n


@pytest.mark.parametrize("ydt", [np.float16, np.float32, np.float64])
@pytest.mark.parametrize("xdt", [None, np.float32, np.float64])
@pytest.mark.parametrize("use_sel", [False, True])
def test_lttb_float_centres_near_exact_means(oracle_mod, ydt, xdt, use_sel):
    """Float coordinates (Sec. 4: LTTB's next-bucket means): each centre is
    within 1e-12 of the exact rational bucket mean, measured relative to the
    bucket's mean absolute value (which is the mean itself when the values
    share a sign, and stays meaningful for a bucket that cancels to ~0).
    Accumulating in float32, dropping a term, or averaging the wrong bucket
    misses this by many orders of magnitude."""
    from fractions import Fraction
    y, x, n_out = _float_mean_cases(ydt, xdt, seed=30 + 3 * ALL_DTYPES.index(ydt))
    m = len(y)
    sel = None
    if use_sel:
        # MinMaxLTTB's candidate set (first point, interior MinMax, last point)
        sel = oracle_mod.minmaxlttb_candidates(y, 1000, 8, x=x)
    cx, cy = oracle_mod.lttb_centres(y, n_out, x=x, sel=sel)
    idx = np.arange(m) if sel is None else sel
    mp = len(idx)
    nb = n_out - 2
    b = [1 + (k * (mp - 2)) // nb for k in range(nb + 1)]
    X = (idx.astype(np.float64) if x is None else x[idx].astype(np.float64))
    Y = y[idx].astype(np.float64)
    worst = 0.0
    for k in range(nb - 1):
        lo, hi = b[k + 1], b[k + 2]
        for got, vals in ((cx[k], X[lo:hi]), (cy[k], Y[lo:hi])):
            mu, scale = _exact_mean_and_scale(vals)
            err = abs(Fraction(float(got)) - mu)
            assert err <= Fraction(1, 10**12) * scale, (k, float(got), float(mu))
            if scale:
                worst = max(worst, float(err / scale))
    # the last bucket's centre is the last point itself
    assert cx[-1] == X[-1] and cy[-1] == Y[-1]
    print(f"max mean error / mean |v|: {worst:.3g}")


def test_lttb_cancelling_bucket_is_present():
    """The float-mean cases above really contain a bucket whose exact mean is
    tiny next to its values (so a relative-to-the-mean check would be
    meaningless there, and the scale matters)."""
    y, _, n_out = _float_mean_cases(np.float32, None, seed=33)
    m, nb = len(y), n_out - 2
    b = [1 + (k * (m - 2)) // nb for k in range(nb + 1)]
    mu, scale = _exact_mean_and_scale(y[b[7]:b[8]])
    assert abs(mu) < scale / 1000


def test_lttb_step_areas_match_exact_areas(oracle_mod):
    """oracle.lttb_step's areas (the step-wise checker's inputs): for every
    point of every bucket, the doubled area the oracle reports is the exact
    rational |cross(P_b - A, C - A)| of the same doubles, up to the rounding
    of four subtractions, two products and one difference; the pick's area is
    the largest, reached first."""
    from fractions import Fraction
    rng = np.random.default_rng(41)
    for trial in range(6):
        m = int(rng.integers(30, 300))
        n_out = int(rng.integers(4, m // 3))
        y = S.walk(m, (np.float32, np.float64, np.int16)[trial % 3], seed=50 + trial)
        x = None if trial % 2 == 0 else np.cumsum(rng.integers(1, 7, m)).astype(np.float64) * 0.5
        walk = oracle_mod.lttb(y, n_out, x=x)
        cx, cy = oracle_mod.lttb_centres(y, n_out, x=x)
        nb = n_out - 2
        b = [1 + (k * (m - 2)) // nb for k in range(nb + 1)]
        X = np.arange(m, dtype=np.float64) if x is None else x.astype(np.float64)
        Y = y.astype(np.float64)
        for k in range(nb):
            A = int(walk[k])
            C = (Fraction(float(cx[k])), Fraction(float(cy[k])))
            XA, YA = Fraction(float(X[A])), Fraction(float(Y[A]))
            areas = []
            for j in range(b[k], b[k + 1]):
                pick, best, other = oracle_mod.lttb_step(y, n_out, k, A, j, x=x)
                t1 = (XA - C[0]) * (Fraction(float(Y[j])) - YA)
                t2 = (XA - Fraction(float(X[j]))) * (C[1] - YA)
                exact = abs(t1 - t2)
                assert abs(Fraction(other) - exact) <= Fraction(8, 2**53) * (abs(t1) + abs(t2)) + \
                    Fraction(1, 2**1070), (trial, k, j)
                areas.append(other)
                assert pick == int(walk[k + 1])
                if j == pick:
                    assert other == best
            assert best == max(areas) and areas.index(best) == pick - b[k]


# ------------------------------------------------------------ MinMaxLTTB


def test_minmaxlttb_equals_lttb_when_preselection_keeps_all(oracle_mod):
    rng = np.random.default_rng(17)
    for m, n_out, ratio in ((100, 20, 5), (98, 24, 4), (1000, 250, 4)):
        y = rng.standard_normal(m)
        assert n_out * ratio >= m - 2
        assert np.array_equal(oracle_mod.minmaxlttb(y, n_out, ratio), oracle_mod.lttb(y, n_out))


def test_minmaxlttb_is_minmax_then_lttb(oracle_mod):
    rng = np.random.default_rng(18)
    n = 50000
    y = S.walk(n, np.float32, seed=19)
    x = S.timestamps(n, 100, seed=20)
    for xx in (None, x):
        n_out, ratio = 300, 4
        pre = oracle_mod.minmax(y[1:-1], n_out * ratio, x=None if xx is None else xx[1:-1]) + 1
        cand = np.concatenate([[0], pre, [n - 1]])
        assert np.array_equal(oracle_mod.minmaxlttb_candidates(y, n_out, ratio, x=xx), cand)
        sub = oracle_mod.lttb(y[cand], n_out, x=(cand if xx is None else xx[cand]))
        assert np.array_equal(oracle_mod.minmaxlttb(y, n_out, ratio, x=xx), cand[sub])


def test_listing2_shape_minmaxlttb(oracle_mod):
    """The paper's illustrative example: 10 M standard normal values reduced
    to 1000 points by MinMaxLTTB (Sec. 3)."""
    y = np.random.default_rng(0).standard_normal(10_000_000)
    sel = oracle_mod.minmaxlttb(y, 1000, 4)
    assert len(sel) == 1000 and sel[0] == 0 and sel[-1] == len(y) - 1
    assert np.all(np.diff(sel) > 0)


# ------------------------------------------------------------ window


def test_window_matches_searchsorted(oracle_mod):
    x = S.timestamps(10000, 100, seed=21)
    rng = np.random.default_rng(22)
    for _ in range(200):
        a, b = sorted(rng.integers(-100, int(x[-1]) + 100, 2))
        i0, i1 = oracle_mod.window(x, a, b)
        assert i0 == np.searchsorted(x, a, "left") and i1 == np.searchsorted(x, b, "right")


# ------------------------------------------------------------ EveryNth


def test_everynth_invariants(oracle_mod):
    """Every-k-th selection: starts at 0, constant stride k, fits n_out, and k
    is the smallest stride that fits (any smaller stride would overflow)."""
    for n in list(range(0, 40)) + [97, 1000, 1001, 12345]:
        for n_out in range(1, 45):
            got = oracle_mod.everynth(n, n_out)
            if n <= n_out:
                assert got.tolist() == list(range(n))
                continue
            assert got[0] == 0 and len(got) <= n_out
            d = np.diff(got)
            k = int(d[0]) if len(d) else n
            assert (d == k).all()
            assert got[-1] + k >= n and got[-1] < n           # nothing beyond the last stride is dropped
            for s in range(1, k):                             # minimality by brute force
                assert len(range(0, n, s)) > n_out


def test_everynth_hand_values(oracle_mod):
    assert oracle_mod.everynth(10, 3).tolist() == [0, 4, 8]
    assert oracle_mod.everynth(10, 5).tolist() == [0, 2, 4, 6, 8]
    assert oracle_mod.everynth(11, 5).tolist() == [0, 3, 6, 9]
    assert oracle_mod.everynth(7, 1).tolist() == [0]
    assert oracle_mod.everynth(0, 4).tolist() == []


# ------------------------------------------------------------ NaN-aware MinMax / M4


@pytest.mark.parametrize("alphabet", [
    np.array([np.nan, 0.0, 1.0]),
    np.array([np.nan, -np.inf, np.inf]),
    np.array([-0.0, np.nan, 0.0]),
])
@pytest.mark.parametrize("dt", [np.float16, np.float32, np.float64])
def test_nan_exhaustive_tiny(oracle_mod, alphabet, dt):
    """Every series of length <= 6 over a NaN-holding alphabet, against
    numpy's nanargmin / nanargmax per brute-force bin."""
    alphabet = alphabet.astype(dt)
    for n in range(0, 7):
        for combo in itertools.product(range(len(alphabet)), repeat=n):
            y = alphabet[list(combo)] if n else alphabet[:0]
            for kind in ("minmax", "m4"):
                for n_out in _valid_nouts(kind, n):
                    got = getattr(oracle_mod, "nan_" + kind)(y, n_out)
                    exp = brute.nan_binned(y, n_out, kind)
                    assert np.array_equal(got, exp), (kind, y, n_out, got, exp)


def test_nan_random_with_x(oracle_mod):
    rng = np.random.default_rng(31)
    for trial in range(40):
        n = int(rng.integers(10, 400))
        y = rng.normal(size=n)
        y[rng.random(n) < rng.choice([0.0, 0.2, 0.9, 1.0])] = np.nan
        x = np.sort(rng.integers(0, 5 * n, n)).astype(np.int64) if trial % 2 else None
        for kind, n_out in (("minmax", 8), ("minmax", 40), ("m4", 8), ("m4", 40)):
            got = getattr(oracle_mod, "nan_" + kind)(y, n_out, x=x)
            assert np.array_equal(got, brute.nan_binned(y, n_out, kind, x=x)), (trial, kind, n_out)


@pytest.mark.parametrize("dtype", ALL_DTYPES)
def test_nan_variants_equal_plain_without_nan(oracle_mod, dtype):
    """No NaN in y: the NaN-aware selection is the plain one."""
    y = S.walk(3001, dtype, seed=12)
    x = S.timestamps(3001, 50, seed=13)
    for kind, n_out in (("minmax", 100), ("m4", 100)):
        for xx in (None, x):
            assert np.array_equal(getattr(oracle_mod, "nan_" + kind)(y, n_out, x=xx),
                                  getattr(oracle_mod, kind)(y, n_out, x=xx))


def test_nan_all_nan_series(oracle_mod):
    y = np.full(1000, np.nan)
    edges = [-(-(b * 999) // 50) for b in range(50)] + [1000]
    assert oracle_mod.nan_minmax(y, 100).tolist() == edges[:50]
    assert oracle_mod.nan_m4(y, 200).tolist() == sorted(set(edges[:50]) | {e - 1 for e in edges[1:]})


# ------------------------------------------------------------ golden fixtures


def test_golden_hand_worked_examples(oracle_mod):
    with open(os.path.join(GOLDEN, "hand_worked.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        y = np.array(c["y"], dtype=c["dtype"])
        x = None if c.get("x") is None else np.array(c["x"], dtype=np.int64)
        fn = getattr(oracle_mod, c["algo"])
        args = (y, c["n_out"]) + ((c["ratio"],) if c["algo"] == "minmaxlttb" else ())
        got = fn(*args, x=x)
        assert got.tolist() == c["expected"], (c["name"], got.tolist())


# ------------------------------------------------------------ CPU baseline driver


@pytest.mark.parametrize("algo", ["minmax", "m4"])
def test_bin_parallel_driver_equals_serial(oracle_mod, algo):
    """The all-cores CPU baseline splits the bins over threads and finds each
    edge by bisection; it must select exactly what the serial scan does, with
    and without x (integer with gaps and duplicates, float, unsigned), for
    more threads than bins too."""
    rng = np.random.default_rng(90)
    for trial in range(12):
        n = int(rng.integers(1, 30_000))
        dt = ALL_DTYPES[trial % len(ALL_DTYPES)]
        y = S.walk(n, dt, seed=trial)
        xs = [None, np.maximum.accumulate(S.timestamps(n, 50, seed=trial) * (1 + (np.arange(n) > n // 2) * 40)),
              np.sort(rng.random(n) * 1e3), S.timestamps(n, 9, seed=trial + 1).astype(np.uint64)]
        xs[1][n // 3: n // 3 + 7] = xs[1][n // 3]
        for x in xs:
            for n_out in (4, 100, 4 * int(rng.integers(1, 3000))):
                exp = getattr(oracle_mod, algo)(y, n_out, x=x)
                for th in (1, 3, 16, 64):
                    got = oracle_mod.binned_parallel(algo, y, n_out, x=x, threads=th)
                    assert np.array_equal(got, exp), (trial, n, n_out, th)

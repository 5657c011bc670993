"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and casts them; it holds none of the
downsampling arithmetic, and both the GPU path's tests/benchmarks and the
oracle checks take their inputs from here.  The paper benchmarks on arrays
of random values (Sec. 4) and gives no dataset; the shapes below (random
walks, timestamps with gaps, sinusoids with spikes, tie runs, mixed batches,
zoom windows) are the stand-ins.

Host generators use numpy's PCG64 (``default_rng(seed)``); the on-device
variants (for series too large for host RAM) use torch's Philox generator on
the GPU and are therefore different numbers for the same seed.
"""
import math

import numpy as np

_INT_RANGES = {
    np.dtype(np.int8): (-128, 127), np.dtype(np.int16): (-32768, 32767),
    np.dtype(np.int32): (-2**31, 2**31 - 1), np.dtype(np.int64): (-2**63, 2**63 - 1),
    np.dtype(np.uint8): (0, 255), np.dtype(np.uint16): (0, 65535),
    np.dtype(np.uint32): (0, 2**32 - 1), np.dtype(np.uint64): (0, 2**64 - 1),
}

CHUNK = 1 << 24


def cast_walk(w, dtype):
    """Cast a float64 walk to `dtype`: floats round to nearest; signed
    integers are rounded and clipped; unsigned integers are shifted to the
    middle of their range, rounded and clipped."""
    dtype = np.dtype(dtype)
    if dtype.kind == "f":
        return w.astype(dtype)
    lo, hi = _INT_RANGES[dtype]
    if dtype.kind == "u":
        w = w + (hi + 1) / 2
    if dtype.itemsize == 8:
        # float64 cannot hold the 64-bit bounds exactly; clip inside them
        lo_f, hi_f = float(lo) * (1 - 2**-52), float(hi) * (1 - 2**-52)
        return np.clip(np.rint(w), lo_f, hi_f).astype(dtype)
    return np.clip(np.rint(w), lo, hi).astype(dtype)


def walk(n, dtype=np.float32, seed=0):
    """Random walk: cumulative sum of standard normal steps (float64 carry,
    drawn in chunks of 2^24), cast to `dtype`."""
    rng = np.random.default_rng(seed)
    out = np.empty(n, np.dtype(dtype))
    carry = 0.0
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        w = np.cumsum(rng.standard_normal(e - s)) + carry
        carry = float(w[-1])
        out[s:e] = cast_walk(w, dtype)
    return out


def tie_runs(y, frac=0.05, seed=2, lmin=16, lmax=4096):
    """Overwrite runs y[s:s+L] = y[s] (s uniform, L uniform in lmin..lmax)
    until the runs cover `frac` of the series (tie stress).  In place."""
    n = len(y)
    rng = np.random.default_rng(seed + 7919)
    covered = 0
    while covered < frac * n:
        s = int(rng.integers(0, n))
        L = int(rng.integers(lmin, lmax + 1))
        y[s: s + L] = y[s]
        covered += L
    return y


def timestamps(n, gap_max=1000, seed=1, dtype=np.int64):
    """Strictly increasing timestamps: x[0] = 0, x[i] = x[i-1] + g_i with
    g_i uniform in 1..gap_max."""
    rng = np.random.default_rng(seed)
    out = np.empty(n, dtype)
    carry = 0
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        g = rng.integers(1, gap_max + 1, e - s, dtype=np.int64)
        if s == 0:
            g[0] = 0
        c = np.cumsum(g) + carry
        carry = int(c[-1])
        out[s:e] = c
    return out


def sines_with_spikes(x, seed=1):
    """y = 3 sin(2 pi 7 t) + 2 sin(2 pi 113 t + 0.5) + sin(2 pi 2029 t + 1.3)
    + N(0, 0.1) with t = x / x[-1]; 1% of the points get a +-50 spike."""
    rng = np.random.default_rng(seed + 104729)
    n = len(x)
    out = np.empty(n, np.float64)
    span = float(x[-1]) if float(x[-1]) != 0 else 1.0
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        t = x[s:e].astype(np.float64) / span
        v = (3 * np.sin(2 * math.pi * 7 * t) + 2 * np.sin(2 * math.pi * 113 * t + 0.5)
             + np.sin(2 * math.pi * 2029 * t + 1.3) + rng.normal(0.0, 0.1, e - s))
        spike = rng.random(e - s) < 0.01
        sign = np.where(rng.random(e - s) < 0.5, -50.0, 50.0)
        out[s:e] = v + np.where(spike, sign, 0.0)
    return out


def m4_with_x(n, seed=1):
    """M4-with-x workload: int64 timestamps with gaps 1..1000 and a float64
    signal of three sinusoids, noise and 1% spikes."""
    x = timestamps(n, 1000, seed)
    return x, sines_with_spikes(x, seed)


def batch_specs(n_series=512, seed=3, lmin=1e4, lmax=2e7):
    """Mixed batch: lengths log-uniform in [lmin, lmax], dtypes cycling
    f32/f16/i16/u8, MinMax for even i//4 else M4, n_out a multiple of 4
    drawn uniformly in 500..4000.  Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    dts = [np.float32, np.float16, np.int16, np.uint8]
    specs = []
    for i in range(n_series):
        L = int(math.floor(math.exp(rng.uniform(math.log(lmin), math.log(lmax)))))
        n_out = 4 * (int(rng.integers(500, 4001)) // 4)
        specs.append({"n": L, "dtype": np.dtype(dts[i % 4]),
                      "algo": "minmax" if (i // 4) % 2 == 0 else "m4",
                      "n_out": n_out, "seed": 1000 + i})
    return specs


def zoom_requests(n_req, n_series, x_first, x_last, seed=4, qps=1000.0,
                  nout_lo=800, nout_hi=4000, wmin=1e-3):
    """Zoom/pan requests with Poisson arrivals at `qps`: series uniform,
    window width fraction log-uniform in [wmin, 1], position uniform,
    n_out uniform in nout_lo..nout_hi (even).  x_first/x_last: per-series
    first and last timestamp."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / qps, n_req))
    reqs = []
    for i in range(n_req):
        s = int(rng.integers(0, n_series))
        R = int(x_last[s]) - int(x_first[s])
        w = math.exp(rng.uniform(math.log(wmin), 0.0))
        xa = int(x_first[s]) + int(math.floor(rng.random() * (1 - w) * R))
        xb = xa + int(math.floor(w * R))
        n_out = 2 * (int(rng.integers(nout_lo, nout_hi + 1)) // 2)
        reqs.append({"t": float(t[i]), "series": s, "xa": xa, "xb": xb, "n_out": n_out})
    return reqs


# ---------------------------------------------------------------- on device


def device_walk(n, seed, device="cuda", dtype=None, chunk=1 << 26):
    """Random walk generated on the GPU (torch Philox normal steps, float64
    running sum carried across chunks), cast to float32 unless `dtype`."""
    import torch
    dtype = dtype or torch.float32
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = torch.empty(n, dtype=dtype, device=device)
    carry = torch.zeros((), dtype=torch.float64, device=device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        w = torch.randn(e - s, generator=g, device=device, dtype=torch.float64).cumsum_(0)
        w += carry
        carry = w[-1].clone()
        out[s:e] = w.to(dtype)
        del w
    return out


def device_timestamps(n, seed, gap_max=100, device="cuda", chunk=1 << 26):
    """Strictly increasing int64 timestamps on the GPU: x[0] = 0, gaps
    uniform in 1..gap_max."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = torch.empty(n, dtype=torch.int64, device=device)
    carry = torch.zeros((), dtype=torch.int64, device=device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        gaps = torch.randint(1, gap_max + 1, (e - s,), generator=g, device=device, dtype=torch.int64)
        if s == 0:
            gaps[0] = 0
        c = gaps.cumsum_(0)
        c += carry
        carry = c[-1].clone()
        out[s:e] = c
        del c
    return out


def device_m4_with_x(n, seed=1, device="cuda", chunk=1 << 25):
    """The M4-with-x workload generated on the GPU (torch Philox): int64
    timestamps with gaps uniform in 1..1000, and float64 y = 3 sin(2 pi 7 t)
    + 2 sin(2 pi 113 t + 0.5) + sin(2 pi 2029 t + 1.3) + N(0, 0.1) with
    t = x / x[-1], plus a +-50 spike on 1% of the points.  The same
    distributions as m4_with_x, other numbers."""
    import torch
    x = device_timestamps(n, seed, gap_max=1000, device=device)
    g = torch.Generator(device=device)
    g.manual_seed(seed + 104729)
    y = torch.empty(n, dtype=torch.float64, device=device)
    span = float(x[-1].item()) or 1.0
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        t = x[s:e].to(torch.float64) / span
        v = (3 * torch.sin(2 * math.pi * 7 * t) + 2 * torch.sin(2 * math.pi * 113 * t + 0.5)
             + torch.sin(2 * math.pi * 2029 * t + 1.3))
        v += 0.1 * torch.randn(e - s, generator=g, device=device, dtype=torch.float64)
        spike = torch.rand(e - s, generator=g, device=device, dtype=torch.float64) < 0.01
        sign = torch.where(torch.rand(e - s, generator=g, device=device, dtype=torch.float64) < 0.5, -50.0, 50.0)
        y[s:e] = v + torch.where(spike, sign, torch.zeros_like(sign))
        del t, v, spike, sign
    return x, y


def device_walk_cast(n, dtype, seed, device="cuda"):
    """Random walk generated on the GPU in float64 (torch Philox), then cast
    like cast_walk: floats round to nearest, integers are rounded and clipped
    (unsigned shifted to mid-range).  `dtype` is a numpy dtype."""
    import torch
    dtype = np.dtype(dtype)
    tdt = {np.dtype(np.float16): torch.float16, np.dtype(np.float32): torch.float32,
           np.dtype(np.float64): torch.float64, np.dtype(np.int8): torch.int8, np.dtype(np.int16): torch.int16,
           np.dtype(np.int32): torch.int32, np.dtype(np.int64): torch.int64, np.dtype(np.uint8): torch.uint8}[dtype]
    w = device_walk(n, seed, device, dtype=torch.float64)
    if dtype.kind == "f":
        return w.to(tdt)
    lo, hi = _INT_RANGES[dtype]
    if dtype.kind == "u":
        w += (hi + 1) / 2
    return torch.clamp(torch.round(w), lo, hi).to(tdt)

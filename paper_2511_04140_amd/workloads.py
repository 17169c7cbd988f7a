"""Seeded synthetic inputs shaped like the paper's workloads.

The paper measures on twelve datasets (Sec. 5.1.1, Table 2) that are not
shipped with it; these generators stand in for them with the decimal
structure the paper describes (beta_avg 3..16, values kept at a fixed number
of decimal places, occasional full-precision outliers).  No record of any of
those datasets is reproduced.

This module holds no step of the codec: it only draws numbers.  Both the CPU
oracle (through the tests) and the HIP path consume the arrays it returns.

Decimal rounding: v = rint(x * 10^d) / 10^d.  10^d is exact for d <= 22 and
the division is correctly rounded, so v is the binary64 value nearest to the
d-place decimal.  For binary32 the integer m = rint(x * 10^d) is divided in
binary32 (m < 2^24), giving the binary32 value nearest to the decimal.
Rounding a small negative number to d places yields -0.0; adding +0.0 turns
it into +0.0, as parsing the decimal text "0" would.  -0.0 appears only where
a generator draws it on purpose as a special value.
"""
from __future__ import annotations

import numpy as np

SEGMENT = 65536
_POW10 = np.array([10.0 ** k for k in range(23)])   # exact for k <= 22
# one period of the sinusoids, sin(2 pi t / P) for t = 0..P-1
_SIN_1E4 = np.sin(2.0 * np.pi * np.arange(10000) / 1e4)
_SIN_4096 = np.sin(2.0 * np.pi * np.arange(4096) / 4096.0)


def walk_f64(n: int = 1 << 20, seed: int = 1) -> np.ndarray:
    """Gaussian random walk from 100.0, step sigma 0.5, rounded to 2 places."""
    rng = np.random.default_rng(seed)
    x = 100.0 + np.cumsum(rng.normal(0.0, 0.5, n))
    return np.rint(x * 100.0) / 100.0 + 0.0


def _specials(rng: np.random.Generator, k: int) -> np.ndarray:
    """k special binary64 values drawn uniformly from: NaN (random payload and
    sign, quiet and signalling), +Inf, -Inf, -0.0, random subnormal."""
    kind = rng.integers(0, 5, k)
    sign = rng.integers(0, 2, k).astype(np.uint64) << np.uint64(63)
    payload = rng.integers(1, 1 << 51, k, dtype=np.uint64)
    quiet = rng.integers(0, 2, k).astype(np.uint64) << np.uint64(51)
    nan = sign | np.uint64(0x7FF0000000000000) | quiet | payload
    sub = sign | rng.integers(1, 1 << 52, k, dtype=np.uint64)
    out = np.where(kind == 0, nan,
          np.where(kind == 1, np.uint64(0x7FF0000000000000),
          np.where(kind == 2, np.uint64(0xFFF0000000000000),
          np.where(kind == 3, np.uint64(0x8000000000000000), sub))))
    return out.astype(np.uint64).view(np.float64)


def _pool():
    import concurrent.futures
    import os
    return concurrent.futures.ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1)))


def sensor_f64(n: int = 1 << 28, seed: int = 2, outlier_rate: float = 0.01,
               special_rate: float = 1e-5, block_segments: int = 16, rounded: bool = True) -> np.ndarray:
    """Sensor-like float64 series in 65,536-value segments.

    Each segment keeps d ~ U{1..6} decimal places; values are
    100*sin(2 pi t / 1e4) plus a random walk (step sigma 0.05).  A fraction
    outlier_rate of positions carries the unrounded value times
    (1 + U(-1e-3, 1e-3)), i.e. 16-17 significant digits; a fraction
    special_rate is replaced by a special value (NaN with payload, +-Inf,
    -0.0, subnormal).  Blocks of block_segments segments draw from their own
    generator seeded with (seed, block), so the result does not depend on
    the number of threads.  rounded=False keeps the signal unrounded (and
    without outliers or specials).
    """
    out = np.empty(n, np.float64)
    step = block_segments * SEGMENT
    blocks = [(b, lo, min(n, lo + step)) for b, lo in enumerate(range(0, n, step))]

    def walk(blk):
        b, lo, hi = blk
        rng = np.random.default_rng([seed, b])
        inc = rng.standard_normal(hi - lo, dtype=np.float32) * np.float32(0.05)
        np.cumsum(inc, dtype=np.float64, out=out[lo:hi])
        return float(out[hi - 1])

    def finish(blk, offset):
        b, lo, hi = blk
        m = hi - lo
        rng = np.random.default_rng([seed, b, 1])
        x = 100.0 * _SIN_1E4[np.arange(lo, hi) % 10000] + (out[lo:hi] + offset)
        if not rounded:
            out[lo:hi] = x
            return
        nseg = (m + SEGMENT - 1) // SEGMENT
        scale = np.repeat(_POW10[rng.integers(1, 7, nseg)], SEGMENT)[:m]
        v = np.rint(x * scale) / scale + 0.0
        outl = rng.random(m) < outlier_rate
        v[outl] = x[outl] * (1.0 + rng.uniform(-1e-3, 1e-3, int(outl.sum())))
        spec = rng.random(m) < special_rate
        v[spec] = _specials(rng, int(spec.sum()))
        out[lo:hi] = v

    with _pool() as ex:
        totals = list(ex.map(walk, blocks))
        offsets = np.concatenate([[0.0], np.cumsum(totals)[:-1]]) if blocks else []
        list(ex.map(finish, blocks, offsets))
    return out


def significant_f64(n: int, seed: int, digits: int) -> np.ndarray:
    """The unrounded sensor signal rounded to `digits` significant decimal
    digits: rint(x * 10^j) / 10^j with j = digits - 1 - floor(log10 |x|)
    (the nearest double to that decimal for digits <= 15)."""
    x = sensor_f64(n, seed, rounded=False)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log10(np.abs(x)))
    e[~np.isfinite(e)] = 0.0
    j = digits - 1 - e
    p = 10.0 ** np.abs(j)
    return np.where(j >= 0, np.rint(x * p) / p, np.rint(x / p) * p) + 0.0


def _field_f32(rng_seed, count: int, side: int = 512, lattice: int = 17, ex=None) -> np.ndarray:
    """The first count values (x fastest) of a side^3 field built by
    tri-linear interpolation of a random lattice^3 grid plus a
    U(-1e-3, 1e-3) perturbation at full binary32 precision.  The
    interpolation is done axis by axis (z, then y, then x), which is the
    same tri-linear weight product evaluated in a fixed order."""
    grid = np.random.default_rng(list(rng_seed)).standard_normal((lattice, lattice, lattice))
    coords = np.arange(side, dtype=np.float64) * (lattice - 1) / (side - 1)
    i0 = np.minimum(coords.astype(np.int64), lattice - 2)
    f = coords - i0
    out = np.empty(count, np.float32)
    plane = side * side

    def one(z):
        gz = (1.0 - f[z]) * grid[i0[z]] + f[z] * grid[i0[z] + 1]           # (y, x) lattice
        rows = (1.0 - f)[:, None] * gz[i0] + f[:, None] * gz[i0 + 1]       # side x lattice
        vals = (1.0 - f)[None, :] * rows[:, i0] + f[None, :] * rows[:, i0 + 1]  # side x side
        take = min(plane, count - z * plane)
        pert = np.random.default_rng(list(rng_seed) + [z]).uniform(-1e-3, 1e-3, take)
        out[z * plane:z * plane + take] = (vals.reshape(-1)[:take] + pert).astype(np.float32)

    list(ex.map(one, range((count + plane - 1) // plane)))
    return out


def mixed_f32(n: int = 1 << 29, seed: int = 3, side: int = 512) -> np.ndarray:
    """float32 set: first half smooth sinusoid plus N(0, 0.01^2) noise at
    d ~ U{0..4} places per 65,536-value segment; second half an HPC-like
    field with full-precision mantissas (side^3 fields, x fastest, as many
    as needed: two for the full-size set)."""
    half = n // 2
    out = np.empty(n, np.float32)
    step = 16 * SEGMENT

    def smooth(blk):
        b, lo = blk
        hi = min(half, lo + step)
        m = hi - lo
        rng = np.random.default_rng([seed, b])
        x = (_SIN_4096[np.arange(lo, hi) % 4096] +
             rng.standard_normal(m, dtype=np.float32).astype(np.float64) * 0.01)
        nseg = (m + SEGMENT - 1) // SEGMENT
        scale = np.repeat(_POW10[rng.integers(0, 5, nseg)], SEGMENT)[:m]
        mant = np.rint(x * scale).astype(np.float32)
        out[lo:hi] = mant / scale.astype(np.float32) + np.float32(0.0)

    with _pool() as ex:
        list(ex.map(smooth, enumerate(range(0, half, step))))
        rest = n - half
        per_field = side ** 3
        pos = 0
        fid = 0
        while pos < rest:
            take = min(rest - pos, per_field)
            out[half + pos:half + pos + take] = _field_f32((seed, 100 + fid), take, side=side, ex=ex)
            pos += take
            fid += 1
    return out


def decimal_f64(n: int, seed: int, places: int, magnitude: float = 100.0) -> np.ndarray:
    """Uniform values of the given magnitude rounded to `places` decimals."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-magnitude, magnitude, n)
    s = 10.0 ** places
    return np.rint(x * s) / s + 0.0


def decimal_f32(n: int, seed: int, places: int, magnitude: float = 10.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = rng.uniform(-magnitude, magnitude, n)
    m = np.rint(x * 10.0 ** places).astype(np.float32)
    return m / np.float32(10.0 ** places) + np.float32(0.0)


def _sensor_values(rng, n: int, d: int, phase: int) -> np.ndarray:
    """100 sin(2 pi t / 1e4) + random walk (sigma 0.05), rounded to d places."""
    t = (np.arange(n) + phase) % 10000
    walk = np.cumsum(rng.standard_normal(n, dtype=np.float32).astype(np.float64) * 0.05)
    x = 100.0 * _SIN_1E4[t] + walk
    s = _POW10[d]
    return np.rint(x * s) / s + 0.0


def batch_layout(count: int = 10000, seed: int = 4, lo: int = 1024, hi: int = 369_000,
                 f64_share: float = 0.6, max_places: int = 6):
    """The shape of a batch of independent series: (lengths, is_float64,
    decimal places), lengths log-uniform on [lo, hi] values, a shuffled
    f64_share of the series float64, d ~ U{0..max_places}."""
    rng = np.random.default_rng([seed, 0])
    n64 = int(round(count * f64_share))
    is64 = np.zeros(count, bool)
    is64[rng.permutation(count)[:n64]] = True
    lens = np.exp(rng.uniform(np.log(lo), np.log(hi), count)).astype(np.int64)
    places = rng.integers(0, max_places + 1, count)
    return lens, is64, places


def batch_series_one(i: int, lens, is64, places, seed: int = 4) -> np.ndarray:
    """Series i of a batch layout: sensor-like values without outliers or
    specials at its decimal places, float32 where the layout says so."""
    r = np.random.default_rng([seed, 1, i])
    v = _sensor_values(r, int(lens[i]), int(places[i]), int(r.integers(0, 10000)))
    return v if is64[i] else v.astype(np.float32)


def batch_series(count: int = 10000, seed: int = 4, lo: int = 1024, hi: int = 369_000,
                 f64_share: float = 0.6, max_places: int = 6, select=None) -> list:
    """Independent series for batched launches (batch_layout, then
    batch_series_one for each).  With the defaults the expected total is
    about 4 GB (10,000 x 62,500 values x 6.4 bytes); with hi = 2^24 it is
    about 110 GB, which callers generate a subset (select) at a time."""
    lens, is64, places = batch_layout(count, seed, lo, hi, f64_share, max_places)
    idx = range(count) if select is None else select
    with _pool() as ex:
        return list(ex.map(lambda i: batch_series_one(i, lens, is64, places, seed), idx))


def serving_payloads(count: int = 256, seed: int = 5, lo_bytes: int = 4096, hi_bytes: int = 64 << 20) -> list:
    """Request payloads for the serving loop: byte sizes log-uniform on
    [lo_bytes, hi_bytes], dtype float64 or float32 with equal odds, content
    as sensor_f64 (segments of 1-6 places, 1% outliers, specials at 1e-5)."""
    rng = np.random.default_rng([seed, 0])
    sizes = np.exp(rng.uniform(np.log(lo_bytes), np.log(hi_bytes), count)).astype(np.int64)
    f64 = rng.random(count) < 0.5
    out = []
    for i in range(count):
        es = 8 if f64[i] else 4
        n = max(1, int(sizes[i]) // es)
        v = sensor_f64(n, seed=seed * 1000 + i)
        with np.errstate(invalid="ignore", over="ignore"):
            out.append(v if f64[i] else v.astype(np.float32))
    return out

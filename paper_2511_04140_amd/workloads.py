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


def sensor_f64(n: int = 1 << 28, seed: int = 2, outlier_rate: float = 0.01,
               special_rate: float = 1e-5, block_segments: int = 64) -> np.ndarray:
    """Sensor-like float64 series in 65,536-value segments.

    Each segment keeps d ~ U{1..6} decimal places; values are
    100*sin(2 pi t / 1e4) plus a random walk (step sigma 0.05).  A fraction
    outlier_rate of positions carries the unrounded value times
    (1 + U(-1e-3, 1e-3)), i.e. 16-17 significant digits; a fraction
    special_rate is replaced by a special value (NaN with payload, +-Inf,
    -0.0, subnormal).
    """
    rng = np.random.default_rng(seed)
    out = np.empty(n, np.float64)
    walk0 = 0.0
    step = block_segments * SEGMENT
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        m = hi - lo
        t = np.arange(lo, hi, dtype=np.float64)
        walk = walk0 + np.cumsum(rng.normal(0.0, 0.05, m))
        walk0 = float(walk[-1])
        x = 100.0 * np.sin(2.0 * np.pi * t / 1e4) + walk
        nseg = (m + SEGMENT - 1) // SEGMENT
        d = np.repeat(rng.integers(1, 7, nseg), SEGMENT)[:m].astype(np.float64)
        scale = 10.0 ** d
        v = np.rint(x * scale) / scale + 0.0
        outl = rng.random(m) < outlier_rate
        v[outl] = x[outl] * (1.0 + rng.uniform(-1e-3, 1e-3, int(outl.sum())))
        spec = rng.random(m) < special_rate
        v[spec] = _specials(rng, int(spec.sum()))
        out[lo:hi] = v
    return out


def _field_f32(rng: np.random.Generator, count: int, side: int = 512, lattice: int = 17,
               start: int = 0) -> np.ndarray:
    """count values (x fastest, from flat index start) of a side^3 field built
    by tri-linear interpolation of a random lattice^3 grid plus a
    U(-1e-3, 1e-3) perturbation at full binary32 precision."""
    grid = rng.standard_normal((lattice, lattice, lattice))
    out = np.empty(count, np.float32)
    coords = np.arange(side, dtype=np.float64) * (lattice - 1) / (side - 1)
    i0 = np.minimum(coords.astype(np.int64), lattice - 2)
    f = coords - i0
    plane = side * side
    pos = 0
    flat = start
    while pos < count:
        z = flat // plane
        take = min(count - pos, plane - flat % plane)
        idx = np.arange(flat % plane, flat % plane + take)
        y = idx // side
        x = idx % side
        iz, fz = i0[z], f[z]
        iy, fy = i0[y], f[y]
        ix, fx = i0[x], f[x]
        acc = np.zeros(take)
        for dz in (0, 1):
            wz = fz if dz else 1.0 - fz
            for dy in (0, 1):
                wy = fy if dy else 1.0 - fy
                for dx in (0, 1):
                    wx = fx if dx else 1.0 - fx
                    acc += wz * wy * wx * grid[iz + dz, iy + dy, ix + dx]
        pert = rng.uniform(-1e-3, 1e-3, take)
        out[pos:pos + take] = (acc + pert).astype(np.float32)
        pos += take
        flat += take
    return out


def mixed_f32(n: int = 1 << 29, seed: int = 3, side: int = 512) -> np.ndarray:
    """float32 set: first half smooth sinusoid plus N(0, 0.01^2) noise at
    d ~ U{0..4} places per 65,536-value segment; second half an HPC-like
    field with full-precision mantissas (two side^3 fields, x fastest)."""
    rng = np.random.default_rng(seed)
    half = n // 2
    out = np.empty(n, np.float32)
    step = 64 * SEGMENT
    for lo in range(0, half, step):
        hi = min(half, lo + step)
        m = hi - lo
        t = np.arange(lo, hi, dtype=np.float64)
        x = np.sin(2.0 * np.pi * t / 4096.0) + rng.normal(0.0, 0.01, m)
        nseg = (m + SEGMENT - 1) // SEGMENT
        d = np.repeat(rng.integers(0, 5, nseg), SEGMENT)[:m]
        mant = np.rint(x * 10.0 ** d).astype(np.float32)
        out[lo:hi] = mant / (10.0 ** d).astype(np.float32) + np.float32(0.0)
    rest = n - half
    per_field = side ** 3
    pos = 0
    fid = 0
    while pos < rest:
        take = min(rest - pos, per_field)
        frng = np.random.default_rng([seed, fid])
        out[half + pos:half + pos + take] = _field_f32(frng, take, side=side)
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

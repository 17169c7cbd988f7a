"""The GPU decides a chunk's case (Eq. 3) without running Alg. 2 value by
value: it applies the stopping test to every value once at the chunk's
largest admissible scale L* = min(AMAX, BMAX - 1 - FL10(v_max)); if all
pass, it bisects the decimal places of a sample (the first value of each
lane) and tests the whole chunk at the largest of them, which is alpha_max
when every value passes there, else bisects alpha_max between it and L*
with the stopping test (after a chunk the sample settled, the GPU tries
the sample before the test at L*, which a chunk it settles then skips); it
applies the recover check once at the result, and checks a value failing
at L* at its own limit lim_i.  If no failing value is an exception, it
bisects alpha_max above L* with every value tested at min(a, lim_i), and
applies the recover check once there (see decide_case in
codec_kernels.hpp).  A value that is not an exception passes
both tests at every scale from its decimal place up to its limit (Thm. 2,
Thm. 4), so the bisections are exact when no value is an exception, and a
failed recover check at their result means some value is one.
This test restates that procedure with numpy, independently of the HIP
code, and checks that on adversarial chunks it reaches the header (A, B)
the oracle's literal Alg. 2 gives."""
from fractions import Fraction

import numpy as np
import pytest


def _pow10_table(mant_bits, lo, hi):
    out = {}
    for k in range(lo, hi + 1):
        q = Fraction(10) ** k
        out[k] = float(q) if mant_bits == 52 else np.float32(float(q))
    return out


class Spec:
    def __init__(self, dt):
        self.dt = np.dtype(dt)
        if self.dt == np.float64:
            self.U, self.A, self.B, self.M, self.bias, self.mu = np.uint64, 22, 15, 52, 1023, 2.0 ** -52
            self.P = _pow10_table(52, -22, 22)
        else:
            self.U, self.A, self.B, self.M, self.bias, self.mu = np.uint32, 10, 6, 23, 127, np.float32(2.0 ** -23)
            self.P = {k: np.float32(v) for k, v in _pow10_table(23, -10, 10).items()}
        self.F = self.dt.type

    def bits(self, v):
        return np.asarray(v, self.dt).view(self.U)

    def mag(self, b):
        return b & self.U((1 << (self.dt.itemsize * 8 - 1)) - 1)

    def fl10(self, magbits):
        e2 = ((magbits >> self.U(self.M)).astype(np.int64)) - self.bias
        k0 = (e2 * 78913) >> 18
        thr = np.array([self.bits(self.P[int(k)])[()] for k in (k0 + 1).ravel()], self.U).reshape(k0.shape)
        return k0 + (magbits >= thr)

    def eps(self, v, P):
        x = v * self.F(P)
        r = np.rint(x)
        return np.abs(x - r) <= np.abs(x) * self.F(self.mu), r

    def full(self, v, P):
        ok, r = self.eps(v, P)
        with np.errstate(all="ignore"):
            back = (r / self.F(P)).astype(self.dt)
        return ok & (self.bits(back) == self.bits(v))


def _sample(spec, v, lstar):
    """The sample: the values each lane loads first (positions 1..64,
    clamped to the chunk), each bisected for its least passing place over
    [0, L*]; returns the largest of these places, a_s."""
    samp = v[np.minimum(1 + np.arange(64), v.size - 1)]
    slo, shi = np.zeros(64, np.int64), np.full(64, lstar, np.int64)
    k = 0
    while (1 << k) < lstar + 1:
        mid = (slo + shi) >> 1
        ok = np.array([spec.eps(samp[i:i + 1], spec.P[int(mid[i])])[0][0] for i in range(64)])
        shi = np.where(ok, mid, shi)
        slo = np.where(ok, slo, mid + 1)
        k += 1
    return int(shi.max())


def fast_decide(spec, v, stats=None, sample_first=False):
    """Returns (A, B); stats counts the chunks settled by the bisection
    above L* and by the sample.  With sample_first the sample is tried
    before the test at L* (the order the GPU takes after a chunk the sample
    settled); both orders must give the same header."""
    b = spec.bits(v)
    m = spec.mag(b)
    lo, hi = spec.bits(spec.P[-spec.A])[()], spec.bits(spec.P[spec.B])[()]
    if np.any((b != 0) & ((m < lo) | (m >= hi))):
        return spec.A + 1, spec.B + 1
    vmax = m.max()
    if vmax == 0:
        return 0, 0
    maxfl = int(spec.fl10(np.array([vmax], spec.U))[0])
    lstar = min(spec.A, spec.B - 1 - maxfl)
    if sample_first:
        # every value passes both tests at a_s: no exception, alpha_max = a_s
        a_s = _sample(spec, v, lstar)
        if spec.full(v, spec.P[a_s]).all():
            if stats is not None:
                stats["first"] += 1
            return a_s, a_s + maxfl + 1
    ok_l, _ = spec.eps(v, spec.P[lstar])
    fail = ~ok_l
    if not fail.any():
        a, h = 0, lstar
        # the largest place of the sample bounds alpha_max from below, and it
        # is alpha_max when every value passes there
        a_s = _sample(spec, v, lstar)
        ok_s, _ = spec.eps(v, spec.P[a_s])
        if ok_s.all():
            if stats is not None:
                stats["sample"] += 1
            if not spec.full(v, spec.P[a_s]).all():
                return spec.A + 1, spec.B + 1
            return a_s, a_s + maxfl + 1
        a = a_s + 1
        while a < h:
            mid = (a + h) // 2
            ok, _ = spec.eps(v, spec.P[mid])
            if ok.all():
                h = mid
            else:
                a = mid + 1
        if not spec.full(v, spec.P[h]).all():
            return spec.A + 1, spec.B + 1
        return h, h + maxfl + 1
    fl = spec.fl10(m[fail])
    lim = np.minimum(spec.A, spec.B - 1 - fl)
    exc = lim == lstar
    for i, (val, li) in enumerate(zip(v[fail], lim)):
        if not exc[i] and not spec.full(np.array([val]), spec.P[int(li)])[0]:
            exc[i] = True
    if exc.any():
        return spec.A + 1, spec.B + 1
    # every value tested at min(a, lim_i): monotone in a for values that are
    # not exceptions, true at a = max lim_i, false at L*
    nz = b != 0
    lim_all = np.full(v.shape, spec.A, np.int64)
    lim_all[nz] = np.minimum(spec.A, spec.B - 1 - spec.fl10(m[nz]))

    def at(a, test):
        ok = np.ones(v.shape, bool)
        for s in np.unique(np.minimum(a, lim_all)):
            sel = np.minimum(a, lim_all) == s
            res = test(v[sel], spec.P[int(s)])
            ok[sel] = res[0] if isinstance(res, tuple) else res
        return ok

    a, h = lstar + 1, int(lim_all.max())
    while a < h:
        mid = (a + h) // 2
        if at(mid, spec.eps).all():
            h = mid
        else:
            a = mid + 1
    if not at(h, spec.full).all():
        return spec.A + 1, spec.B + 1
    if stats is not None:
        stats["above"] += 1
    return h, h + maxfl + 1


def _chunks(dt, rng, count):
    """Adversarial chunks: mixed decimal places and magnitudes, values next
    to powers of ten, sums of short decimals, 15/16/17-digit values, tiny
    and huge magnitudes, specials."""
    n = 1025
    out = []
    for i in range(count):
        kind = i % 10
        if dt == np.float64:
            maxd, maxdig = 22, 17
        else:
            maxd, maxdig = 10, 8
        if kind == 0:
            d = rng.integers(0, maxd + 1)
            mag = 10.0 ** rng.integers(-3, 8)
            v = np.rint(rng.uniform(-mag, mag, n) * 10.0 ** d) / 10.0 ** d
        elif kind == 1:   # per-value decimal places
            d = rng.integers(0, maxd // 2 + 1, n)
            v = np.rint(rng.uniform(-100, 100, n) * 10.0 ** d) / 10.0 ** d
        elif kind == 2:   # near powers of ten
            k = rng.integers(-12, 14, n).astype(np.float64)
            v = 10.0 ** k * (1 + rng.integers(-4, 5, n) * 2.0 ** -50)
        elif kind == 3:   # sums of short decimals
            v = np.rint(rng.uniform(-1, 1, n) * 1e2) / 1e2 + np.rint(rng.uniform(-1, 1, n) * 1e3) / 1e3
        elif kind == 4:   # digits around the precision guard
            dig = rng.integers(maxdig - 3, maxdig + 1)
            mm = rng.integers(10 ** (dig - 1), 10 ** dig, n).astype(np.float64)
            v = mm / 10.0 ** rng.integers(0, min(dig, maxd), n)
        elif kind == 5:   # one outlier in a clean chunk
            v = np.rint(rng.uniform(-50, 50, n) * 1e3) / 1e3
            v[rng.integers(0, n)] = rng.uniform(-50, 50)
        elif kind == 6:   # tiny magnitudes at the alpha limit
            d = maxd - rng.integers(0, 4)
            v = rng.integers(1, 100, n) / 10.0 ** d
        elif kind == 7:   # big integers and small decimals mixed (beta_hat > BMAX)
            v = np.where(rng.random(n) < 0.5, rng.integers(1, 10 ** (maxdig - 4), n).astype(np.float64),
                         rng.integers(1, 100, n) / 10.0 ** 4)
        elif kind == 9:   # high-precision values of mixed magnitudes (a zero crossing)
            dig = rng.integers(maxdig - 5, maxdig - 1)
            x = rng.uniform(-1, 1, n) * 10.0 ** rng.integers(-3, 3, n)
            e = np.floor(np.log10(np.abs(x)))
            p = 10.0 ** (dig - 1 - e)
            v = np.rint(x * p) / p
        else:             # random binary patterns
            nb = 64 if dt == np.float64 else 32
            v = rng.integers(0, 1 << nb, n, dtype=np.uint64, endpoint=False)
            v = v.view(np.float64) if dt == np.float64 else v.astype(np.uint32).view(np.float32)
        v = np.asarray(v, dt)
        if dt == np.float32 and kind not in (8,):
            v = np.asarray(v.astype(np.float64), np.float32)
        out.append(np.where(v == 0, dt(0), v).astype(dt) + dt(0))
    return out


@pytest.mark.parametrize("dt,count", [(np.float64, 1800), (np.float32, 1800)])
def test_fast_decision_matches_literal_alg2(orc, dt, count):
    spec = Spec(dt)
    rng = np.random.default_rng(20251105 + (dt == np.float32))
    mismatches = []
    stats = {"above": 0, "sample": 0, "first": 0}
    for ch in _chunks(dt, rng, count):
        A, B, w, _ = orc.chunk_info(ch)
        for first in (False, True):
            with np.errstate(all="ignore"):
                got = fast_decide(spec, ch, stats, sample_first=first)
            if got != (A, B):
                mismatches.append((ch[:4], first, got, (A, B)))
    assert not mismatches, mismatches[:5]
    assert stats["above"] > count // 10
    assert stats["sample"] > count // 10
    assert stats["first"] > count // 10


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_own_limit_shortcut(dt):
    """The GPU first tests a failing value's own limit against L* with one
    magnitude compare: lim_i == L* exactly when L* == AMAX or
    |v_i| >= fl(10^FL10(v_max)).  Checked here for random magnitudes and
    maxima over the whole admissible range."""
    spec = Spec(dt)
    rng = np.random.default_rng(7 + (dt == np.float32))
    lo, hi = spec.bits(spec.P[-spec.A])[()], spec.bits(spec.P[spec.B])[()]
    for _ in range(400):
        vmax = rng.integers(lo, hi, dtype=spec.U, endpoint=False)
        m = rng.integers(lo, vmax, 64, dtype=spec.U, endpoint=True)
        maxfl = int(spec.fl10(np.array([vmax], spec.U))[0])
        lstar = min(spec.A, spec.B - 1 - maxfl)
        lim = np.minimum(spec.A, spec.B - 1 - spec.fl10(m))
        thr = spec.bits(spec.P[maxfl])[()]
        shortcut = np.full(m.shape, lstar == spec.A) | (m >= thr)
        assert np.array_equal(lim == lstar, shortcut)


def _recovers_rule_f64(v, r, P):
    """The GPU's division-free recover check (recovers() in
    codec_kernels.hpp), restated with exact rationals; None for a tie."""
    from fractions import Fraction
    e = float(Fraction(r) - Fraction(v) * Fraction(P))      # one rounding, as the FMA
    b = int(np.float64(v).view(np.uint64))
    half = float(P) * 2.0 ** (((b >> 52) & 0x7FF) - 1076)   # P * ulp(v) / 2
    toward_zero = (e > 0) != (v > 0)
    tol = half / 2 if toward_zero and (b & ((1 << 52) - 1)) == 0 else half
    if abs(e) < tol:
        return True
    if abs(e) > tol:
        return False
    return None


def _recovers_rule_f32(v, r, P):
    e = np.float32(float(r) - float(v) * float(P))           # exact in binary64, then one rounding
    b = int(np.float32(v).view(np.uint32))
    half = np.float32(float(P) * 2.0 ** (((b >> 23) & 0xFF) - 151))
    toward_zero = (e > 0) != (v > 0)
    tol = np.float32(half / 2) if toward_zero and (b & ((1 << 23) - 1)) == 0 else half
    if abs(e) < tol:
        return True
    if abs(e) > tol:
        return False
    return None


def test_division_free_recover_check():
    """The recover check of Alg. 2 (r / 10^a must give back v after IEEE
    division) is taken on the GPU from the sign and size of the fused
    residual r - v * 10^a against v's rounding interval.  It must agree with
    the division on decimal strings, random magnitudes, powers of two (whose
    interval is lopsided) and their neighbours, in both precisions."""
    rng = np.random.default_rng(2511)
    checked = 0
    for i in range(6000):
        kind = i % 4
        if kind == 0:
            v = float(f"{int(rng.integers(1, 10 ** int(rng.integers(1, 16))))}e-{int(rng.integers(0, 16))}")
        elif kind == 1:
            v = float(rng.standard_normal() * 10.0 ** rng.integers(-20, 15))
        elif kind == 2:
            v = float(2.0 ** int(rng.integers(-60, 50)))
        else:
            v = float(np.nextafter(2.0 ** int(rng.integers(-30, 40)), 0.0))
        v = -v if rng.random() < 0.5 else v
        if v == 0 or abs(v) < 1e-22 or abs(v) >= 1e15:
            continue
        for a in range(0, 23):
            P = 10.0 ** a
            x = v * P
            if abs(x) >= 2.0 ** 52:
                break
            r = float(np.rint(x))
            if r == 0:
                continue
            got = _recovers_rule_f64(v, r, P)
            if got is not None:
                assert got == (r / P == v), (v, a)
                checked += 1
    assert checked > 50000
    for i in range(3000):
        kind = i % 3
        if kind == 0:
            v = np.float32(float(f"{int(rng.integers(1, 10 ** int(rng.integers(1, 8))))}e-{int(rng.integers(0, 8))}"))
        elif kind == 1:
            v = np.float32(rng.standard_normal() * 10.0 ** rng.integers(-9, 6))
        else:
            v = np.nextafter(np.float32(2.0 ** int(rng.integers(-20, 19))), np.float32(0))
        if v == 0 or abs(v) < 1e-10 or abs(v) >= 1e6:
            continue
        for a in range(0, 11):
            P = np.float32(10.0 ** a)
            x = np.float32(v * P)
            if abs(float(x)) >= 2.0 ** 23:
                break
            r = np.rint(x)
            if r == 0:
                continue
            got = _recovers_rule_f32(v, r, P)
            if got is not None:
                assert got == bool(np.float32(r / P) == v), (v, a)

"""Pins of the oracle's ablation variants (Sec. 5.4.2, Fig. 12b).

Fal_Elf takes decimal places with the trial-and-error test of Sec. 1;
Fal_Sparse and Fal_Dense write every bit-plane row in one scheme.  The
variants are checked against the values the paper prints for the trial test,
against closed forms (binary fractions, all-dense sizes, the all-sparse worst
case), against what Thm. 4 implies about the two stopping tests, and against
each other: the dense payload holds the rows verbatim, so it fixes every
row's non-zero byte count, which fixes the sparse size and the adaptive
choice of Sec. 3.3.
"""
import os
from decimal import Decimal

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")
VARIANTS = ("falcon", "elf", "sparse", "dense")


def _rows(name):
    for line in open(os.path.join(GOLD, name)):
        line = line.split("#")[0].strip()
        if line:
            yield [p.strip() for p in line.split("|")]


def test_trial_test_examples_printed_in_paper(orc):
    n = 0
    for v, a_elf, a_falcon in _rows("elf_examples.txt"):
        x = np.array([float(v)])
        assert orc.dpds_many(x, "elf")[0][0] == int(a_elf), v
        assert orc.dpds_many(x, "falcon")[0][0] == int(a_falcon), v
        n += 1
    assert n == 3
    # the chunk header follows: a chunk holding 1.11 gets alpha_max 3 under
    # the trial test and 2 under Alg. 2
    x = np.array([1.11, 2.5, 7.0])
    assert orc.encode_chunk(x, variant="elf")[0] == 3
    assert orc.encode_chunk(x)[0] == 2


def _decimal_sample(rng, n):
    """Decimal strings m * 10^-s (up to 15 digits) and random doubles."""
    m = rng.integers(1, 10 ** rng.integers(1, 16, n), dtype=np.int64)
    s = rng.integers(0, 23, n)
    x1 = np.array([float(f"{a}e-{b}") for a, b in zip(m.tolist(), s.tolist())])
    x2 = rng.standard_normal(n) * 10.0 ** rng.integers(-10, 10, n)
    x = np.concatenate([x1, -x1[: n // 3], x2])
    return x[np.isfinite(x) & (x != 0)]


def test_trial_test_never_finds_fewer_places(orc):
    """An exact integer passes the bound of Thm. 4, so the trial test stops
    no earlier than Alg. 2.  It can stop later (1.11), or at no alpha: it
    never succeeds where Alg. 2 reports an exception, because a recover check
    passing at some alpha with beta <= 15 means the value has at most 15
    significant digits and alpha decimals, and then Alg. 2 stops at its
    decimal place with the recover check passing (Thm. 2, Thm. 4)."""
    rng = np.random.default_rng(11)
    x = _decimal_sample(rng, 30000)
    af, bf, ef = orc.dpds_many(x, "falcon")
    ae, be, ee = orc.dpds_many(x, "elf")
    assert not (ef & ~ee).any()
    both = ~ef & ~ee
    assert (ae[both] >= af[both]).all()
    assert (be[both] - ae[both] == bf[both] - af[both]).all()  # beta = alpha + FL10 + 1
    # the sample shows the effect the paper describes
    assert (ae[both] > af[both]).mean() > 0.01
    assert (ee & ~ef).mean() > 0.001


def test_binary_fractions_get_the_same_places(orc):
    """v = m / 2^k (m odd, |m| < 2^20, k <= 8): v * 10^i = m * 5^i / 2^(k-i)
    is exact in binary64 and an integer exactly from i = k on, so both tests
    give alpha = k; Definition 2 gives DP = k and DS from the digits."""
    rng = np.random.default_rng(12)
    for k in range(0, 9):
        m = rng.integers(-(1 << 20), 1 << 20, 2000) | 1
        v = m.astype(np.float64) / 2.0 ** k
        for variant in ("falcon", "elf"):
            a, b, e = orc.dpds_many(v, variant)
            assert not e.any() and (a == k).all(), (k, variant)
            ds = [k + Decimal(repr(float(t))).adjusted() + 1 for t in v]
            assert b.tolist() == ds


def _chunks(x):
    return [x[i: i + 1025] for i in range(0, x.size, 1025)]


def _header(p, zb):
    w = p[2 + zb]
    nflag = (w + 7) // 8
    flags = int.from_bytes(p[3 + zb: 3 + zb + nflag], "big")
    return w, nflag, flags, 3 + zb + nflag


def _workloads():
    from paper_2511_04140_amd import workloads as W
    rng = np.random.default_rng(13)
    s = W.sensor_f64(6 * 1025 + 77, seed=5)
    s[rng.integers(0, s.size, 20)] = np.array([np.nan, np.inf, -0.0, 5e-324])[rng.integers(0, 4, 20)]
    return [("sensor_f64", s),
            ("walk_f64", W.walk_f64(5 * 1025, seed=6)),
            ("decimal_f64", W.decimal_f64(4 * 1025 + 3, seed=7, places=3)),
            ("mixed_f32", W.mixed_f32(8 * 1025 + 9, seed=8, side=16)),
            ("decimal_f32", W.decimal_f32(3 * 1025, seed=9, places=2))]


def test_static_schemes_against_the_dense_rows(orc):
    """Per chunk: Fal_Dense writes 128 bytes per row with every flag set;
    its rows give each row's non-zero byte count nnz_r; Fal_Sparse then takes
    16 + nnz_r per row with no flag set, and the adaptive scheme
    min(128, 16 + nnz_r) (sparse iff more than 16 zero bytes, Sec. 3.3).
    Headers (alpha_max, beta_hat_max, z_1, w) agree, and every variant
    decodes back to the chunk."""
    for name, x in _workloads():
        zb = 8 if x.dtype == np.float64 else 4
        for c in _chunks(x):
            pd = orc.encode_chunk(c, variant="dense")
            ps = orc.encode_chunk(c, variant="sparse")
            pf = orc.encode_chunk(c)
            w, nflag, flags, h = _header(pd, zb)
            assert pd[:h - nflag] == ps[:h - nflag] == pf[:h - nflag], name
            assert flags == (1 << w) - 1 and len(pd) == h + 128 * w, name
            rows = np.frombuffer(pd[h:], np.uint8).reshape(w, 128) if w else np.zeros((0, 128), np.uint8)
            nnz = (rows != 0).sum(axis=1)
            ws, _, flags_s, _ = _header(ps, zb)
            assert ws == w and flags_s == 0 and len(ps) == h + int((16 + nnz).sum()), name
            assert len(pf) == h + int(np.minimum(128, 16 + nnz).sum()), name
            _, _, flags_f, _ = _header(pf, zb)
            want = sum(1 << (w - 1 - r) for r in range(w) if nnz[r] >= 112)
            assert flags_f == want, name
            for p in (pd, ps, pf):
                y = orc.decode_chunk(p, x.dtype)[: c.size]
                assert np.array_equal(y.view(np.uint8), c.view(np.uint8)), name


def test_all_sparse_worst_case_reaches_its_bound(orc):
    """Case 2 (a NaN) with values alternating +0.0 and 2.0: every delta of
    zigzag(bits) is 2^63 (2^31), whose zigzag has every bit set, so each row
    byte is 0xFF and an all-sparse row takes 16 + 128 bytes."""
    v = np.where(np.arange(1025) % 2 == 0, 0.0, 2.0)
    v[0] = np.nan
    p = orc.encode_chunk(v, variant="sparse")
    assert len(p) == 11 + 8 + 64 * 144 == orc.bound(1025, np.float64, "sparse") - 36
    assert len(orc.encode_chunk(v, variant="dense")) == 8211
    y = orc.decode_chunk(p, np.float64)
    assert np.array_equal(y.view(np.uint8), v.view(np.uint8))
    v32 = np.where(np.arange(1025) % 2 == 0, 0.0, 2.0).astype(np.float32)
    v32[0] = np.nan
    p = orc.encode_chunk(v32, variant="sparse")
    assert len(p) == 7 + 4 + 32 * 144 == orc.bound(1025, np.float32, "sparse") - 36
    for variant in ("falcon", "elf", "dense"):
        assert orc.bound(5000, np.float64, variant) == orc.bound(5000, np.float64)


@pytest.mark.parametrize("variant", VARIANTS)
def test_variant_streams_roundtrip(orc, variant):
    for name, x in _workloads():
        s = orc.compress(x, variant)
        assert len(s) <= orc.bound(x.size, x.dtype, variant)
        y = orc.decompress(s)
        assert np.array_equal(y.view(np.uint8), x.view(np.uint8)), (name, variant)
        # only the canonical (adaptive, Alg. 2) stream passes the validator
        assert (orc.validate(s) == 0) == (variant == "falcon" or s == orc.compress(x)), (name, variant)
    e = orc.compress(np.zeros(0), variant)
    assert len(e) == 32 and orc.decompress(e).size == 0

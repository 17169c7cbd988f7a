"""Pins of the oracle's per-value decimal-place search at full scale, and
closed-form pins of the float32 chunk header.

The scale checks run tests/pins/def2_check.cpp, which takes Definition 2 from
the shortest round-trip decimal string of each value (std::to_chars, a
library routine) and compares the oracle's answer value by value:
- every one of the 2^32 binary32 bit patterns;
- 2 x 10^7 binary64 values from four families (random bits, short decimals,
  sums of short decimals, neighbours of powers of ten);
- every decimal string +-m * 10^-s with m < 10^6 (s <= 24 for binary64,
  s <= 12 for binary32).
"""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pins", "def2_check.cpp")


@pytest.fixture(scope="module")
def checker(tmp_path_factory, orc):
    exe = str(tmp_path_factory.mktemp("pins") / "def2_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", SRC, "-o", exe, "-ldl"], check=True)
    from oracle import build
    return exe, build.LIB


def _run(checker, *args):
    exe, lib = checker
    threads = str(max(1, min(16, os.cpu_count() or 1)))
    r = subprocess.run([exe, args[0], lib, threads, *map(str, args[1:])], capture_output=True, text=True)
    out = r.stdout.strip()
    assert r.returncode == 0, out + r.stderr
    head = out.splitlines()[0].split()
    fields = dict(zip(head[1::2], head[2::2]))
    return {k: int(v, 0) for k, v in fields.items()}


@pytest.mark.slow
def test_alg2_equals_definition2_every_f32_pattern(checker):
    r = _run(checker, "f32-all")
    assert r["checked"] == 1 << 32 and r["mismatches"] == 0
    # every decimal place 0..10 occurs among the values Case 1 can take
    assert r["alpha_seen"] == (1 << 11) - 1 and r["regular"] > 10 ** 7


def test_alg2_equals_definition2_f64_sample(checker):
    for seed in (1, 2):
        r = _run(checker, "f64-random", 10_000_000, seed)
        assert r["checked"] == 10_000_000 and r["mismatches"] == 0
        assert r["alpha_seen"] == (1 << 23) - 1 and 0.1 < r["regular"] / r["checked"] < 0.9


def test_alg2_decimal_strings_below_1e6(checker):
    r = _run(checker, "f64-decimals", 10 ** 6)
    assert r["checked"] == 2 * 25 * (10 ** 6 - 1) and r["mismatches"] == 0
    assert r["alpha_seen"] == (1 << 23) - 1
    r = _run(checker, "f32-decimals", 10 ** 6)
    assert r["checked"] == 2 * 13 * (10 ** 6 - 1) and r["mismatches"] == 0
    assert r["alpha_seen"] == (1 << 11) - 1


# ---------------------------------------------------------------------------
# float32 chunk header (Sec. 3.2.3, Eq. 3) in closed form
# ---------------------------------------------------------------------------
def _shortest_int(v, d):
    """The integer m with v = m * 10^-d, read off v's shortest string."""
    from decimal import Decimal
    return int(Decimal(np.format_float_scientific(np.float32(v), unique=True)).scaleb(d))


@pytest.mark.parametrize("d,magnitude,fl", [(d, 9.4, 0) for d in range(0, 6)] +
                         [(d, 99.0, 1) for d in range(0, 5)] + [(0, 99999.0, 4), (1, 99999.0, 4)])
def test_f32_case1_header_closed_form(orc, d, magnitude, fl):
    """A chunk of d-place binary32 decimals (at most 6 significant digits, so
    each value's shortest string is its decimal) whose largest magnitude has
    FL10 = fl is Case 1 with alpha_max = d and beta_hat_max = d + fl + 1, and
    g_1 is the decimal's integer m_1 (Eq. 3)."""
    from paper_2511_04140_amd import workloads as W
    v = W.decimal_f32(1025, seed=40 + d, places=d, magnitude=magnitude)
    assert int(np.floor(np.log10(np.abs(v).max()))) == fl
    A, B, w, _ = orc.chunk_info(v)
    assert (A, B) == (d, d + fl + 1)
    p = orc.encode_chunk(v)
    assert int.from_bytes(p[2:6], "little", signed=True) == _shortest_int(v[0], d)
    y = orc.decode_chunk(p, np.float32)
    assert np.array_equal(y.view(np.uint32), v.view(np.uint32))


def test_f32_header_edges(orc):
    # all +0.0: alpha_max = 0, beta_hat_max = 0, w = 0
    assert orc.chunk_info(np.zeros(1025, np.float32))[:3] == (0, 0, 0)
    # beta_hat_max = 3 + 3 + 1 = 7 > 6 with no exception: Case 2 keeps the
    # real header (3, 7), not the exception header (11, 7)
    v = np.array([1000.0, 0.001] * 300, np.float32)
    A, B, w, _ = orc.chunk_info(v)
    assert (A, B) == (3, 7)
    # one value with 7 significant digits is an exception: header (11, 7)
    v = np.full(1025, 1.5, np.float32)
    v[10] = np.float32(1.234567)
    assert orc.chunk_info(v)[:2] == (11, 7)
    # the Case-1 integer limit: 999999 (6 digits) at place 0 stays Case 1
    v = np.array([999999.0, -999999.0, 0.0] * 100, np.float32)
    assert orc.chunk_info(v)[:2] == (0, 6)

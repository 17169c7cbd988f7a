"""The decoder's inverse of Eq. 3 for Case 1 chunks, v = g / 10^alpha, takes
no division: with y = RN(1/P), q = RN(g * y), it computes
RN(q + RN(g - q * P) * y) (Markstein's correction step, two fused
multiply-adds; see decompress_chunk in codec_kernels.hpp for why it is the
correctly rounded quotient).  tests/pins/quotient_check.c compares that
formula with the IEEE quotient bit for bit using the C library's correctly
rounded fma: every binary32 case Case 1 can produce (|g| < 10^6, alpha
<= 10), and for binary64 every |g| <= 2 * 10^6 plus 2 * 10^6 random g below
10^15 at each alpha <= 21 (alpha = 22 keeps the division in the kernel).
Without the correction step the same program finds millions of
mismatches.  The compressor's recover check of Alg. 2 (recovers_int, used
by the case decision's sample) computes the same quotient for integers
r = round(v * 10^alpha) in the same ranges."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pins", "quotient_check.c")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("quot") / "quotient_check")
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", SRC, "-o", out, "-lm"],
                   check=True)
    return out


def _run(exe, *args):
    r = subprocess.run([exe, *map(str, args)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    f = r.stdout.split()
    return int(f[f.index("checked") + 1]), int(f[f.index("mismatches") + 1])


def test_binary32_every_case1_quotient(exe):
    checked, bad = _run(exe, "f32")
    assert checked == 11 * (2 * 999999 + 1) and bad == 0


def test_binary64_quotients(exe):
    checked, bad = _run(exe, "f64", 2_000_000, 20251105)
    assert checked == 22 * (4_000_001 + 2_000_000) and bad == 0

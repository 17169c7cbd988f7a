"""The HIP library loads on the CPU and exports every symbol falcon.h
declares; host-side argument checks that need no GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "falcon.h")
LIB = os.path.join(ROOT, "paper_2511_04140_amd", "libfalcon.so")


def declared_functions():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(falcon_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("falcon_create", "falcon_destroy", "falcon_compress_bound", "falcon_compress",
                 "falcon_decompress", "falcon_decompress_n", "falcon_sync", "falcon_stream_info",
                 "falcon_status_str", "falcon_compress_each", "falcon_decompress_each"):
        assert want in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libfalcon.so not built")
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_compress_bound_and_stream_info_on_host():
    L = ctypes.CDLL(LIB)
    L.falcon_compress_bound.restype = ctypes.c_size_t
    L.falcon_compress_bound.argtypes = [ctypes.c_size_t, ctypes.c_int]
    assert L.falcon_compress_bound(0, 2) == 32
    assert L.falcon_compress_bound(1, 2) == 32 + 4 + 8211
    assert L.falcon_compress_bound(1025, 1) == 32 + 4 + 4107
    assert L.falcon_compress_bound(1026, 2) == 32 + 2 * (4 + 8211)
    assert L.falcon_compress_bound(10, 3) == 0
    from oracle import oracle
    import numpy as np
    s = oracle.compress(np.arange(3000, dtype=np.float32))
    n = ctypes.c_size_t()
    dt = ctypes.c_int()
    L.falcon_stream_info.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_int)]
    buf = ctypes.create_string_buffer(s, len(s))
    assert L.falcon_stream_info(buf, len(s), ctypes.byref(n), ctypes.byref(dt)) == 0
    assert (n.value, dt.value) == (3000, 1)
    bad = ctypes.create_string_buffer(b"FLCX" + s[4:32], 32)
    assert L.falcon_stream_info(bad, 32, ctypes.byref(n), ctypes.byref(dt)) == 3
    L.falcon_status_str.restype = ctypes.c_char_p
    assert L.falcon_status_str(3) == b"corrupt stream"


def test_decimal_exponent_estimate():
    """The kernels estimate floor(e2 * log10 2) as (e2 * 78913) >> 18; check
    it against exact integer arithmetic over every binary64 exponent."""
    for e2 in range(-1100, 1100):
        k = (e2 * 78913) >> 18
        # exact: 10^k <= 2^e2 < 10^(k+1)
        if e2 >= 0:
            assert 10 ** k <= 2 ** e2 < 10 ** (k + 1), e2
        else:
            # 2^e2 = 1 / 2^-e2
            assert (k < 0 and 2 ** -e2 <= 10 ** -k and 10 ** (-k - 1) < 2 ** -e2) or \
                   (k >= 0 and False), e2


def test_struct_layouts_match_the_binding(tmp_path):
    """The ctypes mirrors of the ABI's structs have the C layout (sizes and
    field offsets from a C program built against falcon.h)."""
    import subprocess
    import sys
    sys.path.insert(0, ROOT)
    from paper_2511_04140_amd import codec as C
    pairs = [(C.Opts, "falcon_opts"), (C.Series, "falcon_series"), (C.PlanInfo, "falcon_plan_info"),
             (C.ServerOpts, "falcon_server_opts"), (C.Request, "falcon_request"),
             (C.Completion, "falcon_completion")]
    body = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HDR}"', 'int main(void) {']
    want = []
    for cls, cname in pairs:
        body.append(f'printf("%zu\\n", sizeof({cname}));')
        want.append(ctypes.sizeof(cls))
        for f, _ in cls._fields_:
            body.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
            want.append(getattr(cls, f).offset)
    body.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(body))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert [int(v) for v in out] == want


def test_create_rejects_unknown_options():
    """falcon_create checks its options on the host before touching a device:
    unknown flag bits or form give FALCON_ERR_INVALID_ARG (no GPU needed)."""
    import sys
    sys.path.insert(0, ROOT)
    from paper_2511_04140_amd import codec as C
    L = C.lib()
    ctx = ctypes.c_void_p()
    for opts in (C.Opts(0x80, 0), C.Opts(0, 7), C.Opts(0, -1)):
        assert L.falcon_create(0, ctypes.byref(opts), ctypes.byref(ctx)) == 1
    assert L.falcon_create(0, None, None) == 1

"""falcon_compress_noalloc (the entry point with a fixed device scratch, for
callers that cannot allocate) through the C ABI: its streams and lengths
equal falcon_compress's on two calls in a row, the second smaller than the
first, and it rejects inputs beyond its scratch before any launch."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _noalloc():
    from paper_2511_04140_amd import codec as C
    L = C.lib()
    f = L.falcon_compress_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                  ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    return f


def _call(f, x, out, d_len):
    from paper_2511_04140_amd import codec as C
    code = C._dtype_code(x.dtype)
    st = f(ctypes.c_void_p(x.data_ptr() if x.numel() else 0), x.numel(), code, ctypes.c_void_p(out.data_ptr()),
           out.numel(), ctypes.c_void_p(d_len.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def test_noalloc_matches_falcon_compress_twice():
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    f = _noalloc()
    ref = C.Codec(0)
    cases = [("sensor_f64, 200,000 chunks", W.sensor_f64(200000 * 1025 - 77, seed=61)),
             ("mixed_f32, 3,000 chunks", W.mixed_f32(3000 * 1025 + 5, seed=62, side=64))]
    for name, x in cases:
        _log(f"[noalloc] {name}")
        xd = torch.from_numpy(x).cuda()
        want = ref.compress(xd).clone()
        out = torch.full((C.compress_bound(x.size, xd.dtype),), 0xAB, dtype=torch.uint8, device="cuda")
        d_len = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        assert _call(f, xd, out, d_len) == 0
        torch.cuda.synchronize()
        n = int(d_len.item())
        assert n == want.numel(), name
        assert torch.equal(out[:n], want), name
        del xd, out
        torch.cuda.empty_cache()
    ref.close()


def test_noalloc_empty_and_limits():
    from paper_2511_04140_amd import codec as C
    f = _noalloc()
    ref = C.Codec(0)
    x = torch.zeros(0, dtype=torch.float64, device="cuda")
    out = torch.zeros(64, dtype=torch.uint8, device="cuda")
    d_len = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    assert _call(f, x, out, d_len) == 0
    torch.cuda.synchronize()
    assert int(d_len.item()) == 32
    assert torch.equal(out[:32], ref.compress(x))
    # beyond the fixed scratch (2^19 chunks): rejected on the host, nothing launched
    big = 537_395_200 + 1
    code = 1
    cap = C.compress_bound(big, torch.float32)
    assert f(ctypes.c_void_p(16), big, code, ctypes.c_void_p(16), cap, None, None) == 5
    # output too small and misaligned pointers: rejected on the host
    assert f(ctypes.c_void_p(16), 1000, 2, ctypes.c_void_p(16), 100, None, None) == 2
    assert f(ctypes.c_void_p(12), 1000, 2, ctypes.c_void_p(16), 1 << 20, None, None) == 1
    ref.close()

"""GPU parity: the HIP codec (through the C ABI) against the CPU oracle.

Streams must be byte-identical to the oracle's; decompression must give
back every input bit.  Small cases span several chunks and a ragged tail;
the full-size workloads (2 GiB float64 sensor series, 2 GiB float32 mixed
set) are compressed whole in the benchmark's launch configuration and
checked chunk by chunk on a sample the oracle encodes one at a time, plus
size and round-trip properties over the whole stream.
"""
import os
import struct
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def codec():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2511_04140_amd import codec as C
    return C.Codec(0)


def _gpu_compress(codec, x):
    t = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    s = codec.compress(t)
    return s


def _roundtrip_and_parity(codec, orc, x, name):
    _log(f"[parity] {name}: n={x.size} dtype={x.dtype}")
    s_gpu = _gpu_compress(codec, x)
    got = s_gpu.cpu().numpy().tobytes()
    want = orc.compress(x)
    if got != want:
        # locate the first differing chunk for the message
        n = x.size
        nc = (n + 1024) // 1025
        sz_g = np.frombuffer(got[32:32 + 4 * nc], np.uint32) if len(got) >= 32 + 4 * nc else None
        sz_w = np.frombuffer(want[32:32 + 4 * nc], np.uint32)
        first = None
        if sz_g is not None:
            diff = np.nonzero(sz_g != sz_w)[0]
            first = int(diff[0]) if diff.size else None
        pytest.fail(f"{name}: stream differs from oracle (len {len(got)} vs {len(want)}, "
                    f"first differing chunk size at {first}, header {got[:32].hex()} vs {want[:32].hex()})")
    y = codec.decompress(s_gpu).cpu().numpy()
    assert y.dtype == x.dtype and y.size == x.size
    assert np.array_equal(y.view(np.uint8), x.view(np.uint8)), name
    # the GPU decoder also takes the oracle's stream
    y2 = codec.decompress(torch.from_numpy(np.frombuffer(want, np.uint8).copy()).cuda()).cpu().numpy()
    assert np.array_equal(y2.view(np.uint8), x.view(np.uint8)), name


def _special_f64(rng, n):
    sp = np.array([0x0, 0x8000000000000000, 0x7FF0000000000000, 0xFFF0000000000000,
                   0x7FF8000000000000, 0xFFF8000000000001, 0x7FF0000000000001,
                   0x0000000000000001, 0x800FFFFFFFFFFFFF, 0x0010000000000000,
                   0x7FEFFFFFFFFFFFFF], np.uint64)
    return rng.choice(sp, n).view(np.float64)


SMALL_CASES = [
    ("walk_f64", lambda W, rng: W.walk_f64(40 * 1025 + 17, seed=1)),
    ("sensor_f64", lambda W, rng: W.sensor_f64(60 * 1025 + 3, seed=2)),
    ("sensor_f64_no_outliers", lambda W, rng: W.sensor_f64(50 * 1025 + 900, seed=5,
                                                          outlier_rate=0.0, special_rate=0.0)),
    ("mixed_f32", lambda W, rng: W.mixed_f32(80 * 1025 + 511, seed=3, side=64)),
    ("specials_f64", lambda W, rng: _special_f64(rng, 5 * 1025 + 7)),
    ("alt_max_f64", lambda W, rng: np.tile([np.finfo(np.float64).max, -np.finfo(np.float64).max], 2100)),
    ("alt_max_f32", lambda W, rng: np.tile([np.finfo(np.float32).max, -np.finfo(np.float32).max],
                                           2100).astype(np.float32)),
    ("zeros_f64", lambda W, rng: np.zeros(3000)),
    ("const_f32", lambda W, rng: np.full(4100, 3.25, np.float32)),
    ("int_edge_f64", lambda W, rng: np.tile([999999999999999.0, -999999999999999.0, 0.0], 800)),
    ("big_small_f64", lambda W, rng: np.array([1e10, 0.00001] * 1500)),
    ("random_bits_f64", lambda W, rng: rng.integers(0, 1 << 64, 6000, dtype=np.uint64,
                                                    endpoint=False).view(np.float64)),
    ("random_bits_f32", lambda W, rng: rng.integers(0, 1 << 32, 6000, dtype=np.uint64)
     .astype(np.uint32).view(np.float32)),
]
for d in range(0, 16):
    SMALL_CASES.append((f"decimal{d}_f64",
                        lambda W, rng, d=d: W.decimal_f64(7 * 1025 + 100, seed=100 + d, places=d,
                                                          magnitude=10.0 ** (12 - min(d, 12)))))
for d in range(16, 23):
    # the largest decimal places of Case 1: the decoder's division-free
    # quotient up to 21 places, the IEEE division at 22
    SMALL_CASES.append((f"decimal{d}_f64",
                        lambda W, rng, d=d: W.decimal_f64(7 * 1025 + 100, seed=100 + d, places=d,
                                                          magnitude=10.0 ** (12 - d))))
for d in (12, 14, 15, 16):
    # mixed magnitudes at high precision: chunks whose small values need more
    # places than L* allows (the bisection above L*)
    SMALL_CASES.append((f"significant{d}_f64",
                        lambda W, rng, d=d: W.significant_f64(30 * 1025 + 77, seed=300 + d, digits=d)))
for d in range(0, 8):
    SMALL_CASES.append((f"decimal{d}_f32",
                        lambda W, rng, d=d: W.decimal_f32(7 * 1025 + 100, seed=200 + d, places=d,
                                                          magnitude=10.0 ** (5 - min(d, 5)))))
for d in (8, 9, 10):
    # up to AMAX = 10 places in Case 1 (five significant digits)
    SMALL_CASES.append((f"decimal{d}_f32",
                        lambda W, rng, d=d: W.decimal_f32(7 * 1025 + 100, seed=200 + d, places=d,
                                                          magnitude=10.0 ** (5 - d))))


@pytest.mark.parametrize("name,make", SMALL_CASES, ids=[c[0] for c in SMALL_CASES])
def test_small_parity(codec, orc, name, make):
    from paper_2511_04140_amd import workloads as W
    rng = np.random.default_rng(abs(hash(name)) % (1 << 32))
    x = make(W, rng)
    _roundtrip_and_parity(codec, orc, x, name)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 1024, 1025, 1026, 2049, 4 * 1025 + 1])
def test_ragged_lengths(codec, orc, n):
    from paper_2511_04140_amd import workloads as W
    _roundtrip_and_parity(codec, orc, W.walk_f64(n, seed=n), f"walk{n}")
    _roundtrip_and_parity(codec, orc, W.decimal_f32(n, seed=n, places=3), f"dec32_{n}")


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_decompress_into_unaligned_views(codec, orc, dt):
    """Decoding into a view at every element phase of a 128-byte line: the
    value stores of every chunk start at each possible misalignment, the
    last chunk is partial, and no byte outside the view is written."""
    from paper_2511_04140_amd import workloads as W
    n = 3 * 1025 + 77
    x = W.walk_f64(n, seed=41) if dt == "f64" else W.decimal_f32(n, seed=41, places=3)
    s = torch.from_numpy(np.frombuffer(orc.compress(x), np.uint8).copy()).cuda()
    tdt = torch.float64 if dt == "f64" else torch.float32
    line = 128 // x.itemsize
    guard = torch.full((n + 2 * line + 64,), -7.25, dtype=tdt, device="cuda")
    for k in range(line):
        _log(f"[parity] unaligned view {dt} phase {k}")
        buf = guard.clone()
        y = codec.decompress(s, out=buf[line + k: line + k + n + 5])
        assert y.numel() == n
        got = buf.cpu().numpy()
        assert np.array_equal(got[line + k: line + k + n].view(np.uint8), x.view(np.uint8)), k
        assert (got[: line + k] == -7.25).all() and (got[line + k + n:] == -7.25).all(), k


def test_empty(codec, orc):
    for dt in (np.float64, np.float32):
        x = np.zeros(0, dt)
        s = codec.compress(torch.zeros(0, dtype=torch.float64 if dt == np.float64 else torch.float32,
                                       device="cuda"))
        assert s.cpu().numpy().tobytes() == orc.compress(x)
        y = codec.decompress(s)
        assert y.numel() == 0


def test_mixed_chunk_cases(codec, orc):
    """Chunks of every kind back to back: Case 1 at several decimal places,
    Case 2 by exception, Case 2 by beta_hat > 15, all-zero, constant."""
    from paper_2511_04140_amd import workloads as W
    rng = np.random.default_rng(77)
    parts = []
    for i in range(60):
        kind = i % 6
        if kind == 0:
            parts.append(W.decimal_f64(1025, seed=i, places=int(rng.integers(0, 8))))
        elif kind == 1:
            c = W.decimal_f64(1025, seed=i, places=2)
            c[int(rng.integers(0, 1025))] = np.nan
            parts.append(c)
        elif kind == 2:
            parts.append(np.array([1e10, 0.00001] * 512 + [3.0]))
        elif kind == 3:
            parts.append(np.zeros(1025))
        elif kind == 4:
            parts.append(np.full(1025, -7.125))
        else:
            c = W.decimal_f64(1025, seed=i, places=3)
            c[int(rng.integers(0, 1025))] = 0.1 + 0.2
            parts.append(c)
    _roundtrip_and_parity(codec, orc, np.concatenate(parts), "mixed_chunk_cases")


def test_repeated_calls_reuse_scratch(codec, orc):
    """Successive launches of decreasing and increasing size share the status
    array (epoch tags) and the control block."""
    from paper_2511_04140_amd import workloads as W
    for n in (300000, 5000, 1025, 90000, 1):
        _roundtrip_and_parity(codec, orc, W.sensor_f64(n, seed=n), f"rep{n}")


def test_corrupt_streams_are_rejected(codec, orc):
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    x = W.walk_f64(20 * 1025, seed=9)
    good = orc.compress(x)
    nc = 20

    def dec(b):
        return codec.decompress(torch.from_numpy(np.frombuffer(bytes(b), np.uint8).copy()).cuda())

    # truncated stream: payload runs past in_len
    with pytest.raises(C.FalconError) as ei:
        dec(good[:-5])
    assert ei.value.status == C.ERR_CORRUPT_STREAM
    # size array no longer sums to the payload byte count
    b = bytearray(good)
    s0 = struct.unpack_from("<I", b, 32)[0]
    struct.pack_into("<I", b, 32, s0 + 1)
    with pytest.raises(C.FalconError):
        dec(b)
    # a chunk size beyond the largest possible chunk
    b = bytearray(good)
    struct.pack_into("<I", b, 36, 9000)
    with pytest.raises(C.FalconError):
        dec(b)
    # bit width above 64 in the first chunk
    b = bytearray(good)
    b[32 + 4 * nc + 10] = 70
    with pytest.raises(C.FalconError):
        dec(b)
    # bad magic
    b = bytearray(good)
    b[0] ^= 0xFF
    with pytest.raises(C.FalconError):
        dec(b)
    # after the errors the context still works
    _roundtrip_and_parity(codec, orc, x, "after_errors")


def test_buffer_too_small(codec):
    from paper_2511_04140_amd import codec as C
    x = torch.ones(5000, dtype=torch.float64, device="cuda")
    with pytest.raises(C.FalconError) as ei:
        codec.compress(x, out=torch.empty(100, dtype=torch.uint8, device="cuda"))
    assert ei.value.status == C.ERR_BUFFER_TOO_SMALL
    s = codec.compress(x)
    with pytest.raises(C.FalconError) as ei:
        codec.decompress(s, out=torch.empty(10, dtype=torch.float64, device="cuda"))
    assert ei.value.status == C.ERR_BUFFER_TOO_SMALL


# ---------------------------------------------------------------------------
# Full-size workloads, sampled against the oracle
# ---------------------------------------------------------------------------
def _full_size_check(codec, orc, x, name, samples=48):
    _log(f"[full] {name}: n={x.size} ({x.nbytes / 2**30:.2f} GiB)")
    n = x.size
    nc = (n + 1024) // 1025
    xd = torch.from_numpy(x).cuda()
    s = codec.compress(xd)
    torch.cuda.synchronize()
    hdr = s[:32].cpu().numpy().tobytes()
    assert hdr[:4] == b"FLCN"
    N, payload = struct.unpack_from("<QQ", hdr, 16)
    assert N == n and s.numel() == 32 + 4 * nc + payload
    sizes = s[32:32 + 4 * nc].cpu().numpy().view(np.uint32).astype(np.int64)
    assert int(sizes.sum()) == payload
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    rng = np.random.default_rng(1234)
    pick = np.unique(np.concatenate([[0, 1, nc - 2, nc - 1], rng.integers(0, nc, samples)]))
    base = 32 + 4 * nc
    for c in pick:
        lo = int(c) * 1025
        vals = x[lo:lo + 1025]
        want = orc.encode_chunk(vals)
        got = s[base + int(offs[c]):base + int(offs[c]) + int(sizes[c])].cpu().numpy().tobytes()
        assert got == want, f"{name}: chunk {c} differs"
    y = codec.decompress(s)
    eq = torch.equal(y.view(torch.uint8), xd.view(torch.uint8))
    assert eq, f"{name}: round trip differs"
    ratio = s.numel() / x.nbytes
    _log(f"[full] {name}: ratio {ratio:.4f}")
    del xd, y, s
    torch.cuda.empty_cache()
    return ratio


def test_full_size_sensor_f64(codec, orc):
    from paper_2511_04140_amd import workloads as W
    _log("[full] generating sensor_f64 2^28")
    x = W.sensor_f64(1 << 28, seed=2)
    _full_size_check(codec, orc, x, "sensor_f64")


def test_full_size_mixed_f32(codec, orc):
    from paper_2511_04140_amd import workloads as W
    _log("[full] generating mixed_f32 2^29")
    x = W.mixed_f32(1 << 29, seed=3)
    _full_size_check(codec, orc, x, "mixed_f32")

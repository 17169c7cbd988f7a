"""The asynchronous device boundary: calls that only enqueue, one
falcon_sync for many of them, lengths delivered to host or device memory,
device-side header checks of falcon_decompress_n, ordering across streams,
the single-pass compression form, and the one-series-per-launch loops.
Every stream is compared with the oracle's, every round trip bit for bit.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _inputs():
    from paper_2511_04140_amd import workloads as W
    return [W.walk_f64(30 * 1025 + 7, seed=1), W.sensor_f64(50 * 1025 + 3, seed=2),
            W.mixed_f32(40 * 1025 + 511, seed=3, side=32), W.decimal_f32(5000, seed=4, places=3),
            np.zeros(0), np.array([1.5]), W.decimal_f64(1025, seed=5, places=4),
            np.random.default_rng(6).integers(0, 1 << 64, 9000, dtype=np.uint64,
                                              endpoint=False).view(np.float64)]


def _bound(C, x):
    return C.compress_bound(x.size, torch.float64 if x.dtype == np.float64 else torch.float32)


def test_many_calls_one_sync(orc):
    """Compressions and decompressions of several arrays enqueued back to
    back with no host wait, then one falcon_sync: host lengths filled, streams
    equal to the oracle's, values bit-exact.  Decompression takes each stream
    from its (not yet read) compression buffer, relying on the call order."""
    from paper_2511_04140_amd import codec as C
    c = C.Codec(0, blocking=False)
    xs = _inputs()
    xd = [torch.from_numpy(x).cuda() for x in xs]
    bufs = [torch.zeros(_bound(C, x), dtype=torch.uint8, device="cuda") for x in xs]
    outs = [torch.full_like(x, -1.0) for x in xd]
    lens = [c.compress_async(x, b) for x, b in zip(xd, bufs)]
    for x, b, o in zip(xd, bufs, outs):
        c.decompress_n_async(b, x.numel(), x.dtype, o)
    c.sync()
    for x, b, o, ln in zip(xs, bufs, outs, lens):
        assert b[:ln.value].cpu().numpy().tobytes() == orc.compress(x)
        assert np.array_equal(o.cpu().numpy().view(np.uint8), x.view(np.uint8))
    c.close()


def test_calls_on_two_streams_are_ordered(orc):
    """A compression on one stream and the decompression of its output on
    another: the context orders them without any host wait."""
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    c = C.Codec(0, blocking=False)
    x = W.sensor_f64(400 * 1025 + 9, seed=12)
    xd = torch.from_numpy(x).cuda()
    b = torch.zeros(_bound(C, x), dtype=torch.uint8, device="cuda")
    y = torch.zeros_like(xd)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for rep in range(3):
        ln = c.compress_async(xd, b, stream=s1)
        c.decompress_n_async(b, x.size, xd.dtype, y, stream=s2)
        c.sync()
        assert b[:ln.value].cpu().numpy().tobytes() == orc.compress(x), rep
        assert torch.equal(y.view(torch.uint8), xd.view(torch.uint8)), rep
        y.fill_(0)
        torch.cuda.synchronize()
    c.close()


def test_device_lengths(orc):
    """FALCON_OPT_DEVICE_LENGTHS: the stream lengths land in device memory in
    stream order (including the 32 of an empty input)."""
    from paper_2511_04140_amd import codec as C
    c = C.Codec(0, blocking=False, device_lengths=True)
    xs = _inputs()
    xd = [torch.from_numpy(x).cuda() for x in xs]
    bufs = [torch.zeros(_bound(C, x), dtype=torch.uint8, device="cuda") for x in xs]
    lens = torch.full((len(xs),), -1, dtype=torch.int64, device="cuda")
    for i, (x, b) in enumerate(zip(xd, bufs)):
        c.compress_async(x, b, out_len=lens[i:i + 1])
    c.sync()
    got = lens.cpu().tolist()
    for x, b, ln in zip(xs, bufs, got):
        want = orc.compress(x)
        assert ln == len(want)
        assert b[:ln].cpu().numpy().tobytes() == want
    c.close()


def test_decompress_n_checks_the_header_on_the_device(orc):
    """falcon_decompress_n never reads the stream on the host: a header that
    disagrees with the caller's count or dtype, or a damaged chunk, is found
    on the device and reported by falcon_sync; the context stays usable."""
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    c = C.Codec(0, blocking=False)
    x = W.walk_f64(20 * 1025, seed=9)
    good = orc.compress(x)
    dev = lambda bts: torch.from_numpy(np.frombuffer(bytes(bts), np.uint8).copy()).cuda()
    y = torch.empty(x.size + 10, dtype=torch.float64, device="cuda")
    cases = {
        "count one more (same chunk count)": (good, x.size + 1, torch.float64),
        "count one less": (good, x.size - 1, torch.float64),
        "wrong dtype": (good, x.size, torch.float32),
    }
    bad = bytearray(good)
    bad[32 + 4 * 20 + 10] = 70  # bit width 70 in the first chunk
    cases["bit width above 64"] = (bad, x.size, torch.float64)
    bad2 = bytearray(good)
    bad2[0] ^= 1
    cases["bad magic"] = (bad2, x.size, torch.float64)
    for name, (bts, n, dt) in cases.items():
        _log(f"[async] {name}")
        out = y if dt == torch.float64 else torch.empty(n, dtype=dt, device="cuda")
        c.decompress_n_async(dev(bts), n, dt, out)
        with pytest.raises(C.FalconError) as ei:
            c.sync()
        assert ei.value.status == C.ERR_CORRUPT_STREAM, name
    # host-side checks fail at once, before any launch
    with pytest.raises(C.FalconError) as ei:
        c.decompress_n_async(dev(good[:100]), x.size, torch.float64, y)
    assert ei.value.status == C.ERR_CORRUPT_STREAM
    with pytest.raises(C.FalconError) as ei:
        c.decompress_n_async(dev(good), x.size, torch.float64, y[:10])
    assert ei.value.status == C.ERR_BUFFER_TOO_SMALL
    # and a good stream afterwards
    c.decompress_n_async(dev(good), x.size, torch.float64, y)
    c.sync()
    assert np.array_equal(y[:x.size].cpu().numpy().view(np.uint8), x.view(np.uint8))
    c.close()


@pytest.mark.parametrize("k", range(8))
def test_single_pass_form_small(orc, k):
    """FALCON_FORM_SINGLE_PASS gives the oracle's stream (work queue and
    look-back), on the same inputs as above."""
    from paper_2511_04140_amd import codec as C
    c = C.Codec(0, form="single_pass")
    x = _inputs()[k]
    s = c.compress(torch.from_numpy(x).cuda())
    assert s.cpu().numpy().tobytes() == orc.compress(x)
    c.close()


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_single_pass_form_many_chunks_per_wave(orc, dt):
    """20,000 chunks, several per wave, through the single pass: the stream
    equals the oracle's and decodes bit for bit; repeated launches reuse the
    status words (tags) and ticket counters."""
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    c = C.Codec(0, form="single_pass")
    n = 20000 * 1025 - 333
    x = W.sensor_f64(n, seed=31) if dt == "f64" else W.mixed_f32(n, seed=32, side=128)
    want = orc.compress(x)
    xd = torch.from_numpy(x).cuda()
    for rep in range(3):
        s = c.compress(xd)
        assert s.cpu().numpy().tobytes() == want, rep
    y = c.decompress(s)
    assert torch.equal(y.view(torch.uint8), xd.view(torch.uint8))
    c.close()


def test_each_loops_match_the_oracle(orc):
    """falcon_compress_each / falcon_decompress_each (one launch sequence per
    series, one wait) on series of uneven lengths and both dtypes."""
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    rng = np.random.default_rng(44)
    xs = []
    for i in range(40):
        n = [0, 1, 1025, 2050][i] if i < 4 else int(rng.integers(1, 30 * 1025))
        xs.append(W.decimal_f64(n, seed=500 + i, places=int(rng.integers(0, 7))) if i % 2 == 0
                  else W.decimal_f32(n, seed=500 + i, places=int(rng.integers(0, 5))))
    c = C.Codec(0)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    streams = c.compress_each(xd)
    for x, s in zip(xs, streams):
        assert s.cpu().numpy().tobytes() == orc.compress(x)
    ys = c.decompress_each(streams, [x.size for x in xs], [t.dtype for t in xd])
    for x, y in zip(xs, ys):
        assert np.array_equal(y.cpu().numpy().view(np.uint8), x.view(np.uint8))
    c.close()


def test_stage_times_of_many_calls(orc):
    """falcon_call_stage_ms: after several asynchronous compressions and
    decompressions and one falcon_sync, every call's stage times can be read,
    newest first (back = 0 is the last call, as falcon_last_stage_ms):
    compressions have a size pass, a scan and a write pass, decompressions a
    scan and the decoding kernel.  The ring keeps FALCON_TIMED_CALLS calls;
    asking beyond it, or for a call never made, is refused."""
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    fresh = C.Codec(0, blocking=False)
    with pytest.raises(C.FalconError):
        fresh.call_stage_ms(0)
    fresh.close()
    c = C.Codec(0, blocking=False)
    xs = [W.sensor_f64(40 * 1025 + 3, seed=2), W.mixed_f32(30 * 1025 + 5, seed=3, side=32),
          W.walk_f64(20000, seed=1)]
    xd = [torch.from_numpy(x).cuda() for x in xs]
    bufs = [torch.zeros(_bound(C, x), dtype=torch.uint8, device="cuda") for x in xs]
    outs = [torch.empty_like(x) for x in xd]
    for x, b, o in zip(xd, bufs, outs):
        c.compress_async(x, b)
        c.decompress_n_async(b, x.numel(), x.dtype, o)
    c.sync()
    n = len(xs)
    for i in range(n):
        dec = c.call_stage_ms(2 * (n - 1 - i))
        comp = c.call_stage_ms(2 * (n - 1 - i) + 1)
        assert all(v > 0 for v in comp), (i, comp)
        assert 0 <= dec[0] < 0.5 and dec[1] > 0 and dec[2] > 0, (i, dec)  # stage 0 holds no kernel
        assert torch.equal(outs[i].view(torch.uint8), xd[i].view(torch.uint8))
    assert c.call_stage_ms(0) == c.last_stage_ms()
    assert abs(c.last_kernel_ms() - sum(c.last_stage_ms())) < 1e-3
    with pytest.raises(C.FalconError):
        c.call_stage_ms(C.TIMED_CALLS)
    # more calls than the ring holds: the oldest slot still held is readable
    small = xd[2]
    for _ in range(C.TIMED_CALLS + 6):
        c.compress_async(small, bufs[2])
    c.sync()
    assert all(v > 0 for v in c.call_stage_ms(C.TIMED_CALLS - 1))
    assert bufs[2][:32].cpu().numpy().tobytes() == orc.compress(xs[2])[:32]
    c.close()

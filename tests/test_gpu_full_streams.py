"""GPU parity on whole streams: every byte of the HIP codec's stream against
the CPU oracle, at the full sizes of the measured workloads, on every
float32 bit pattern, on batch plans with more chunks than the device holds
waves, on the 10,000-series batch of the batched measurement, and on the
oracle's own edge chunks.

A full-size stream is compared slice by slice: the oracle compresses
chunk-aligned slices of the input in threads (a chunk's encoding does not
depend on its neighbours), and each slice's size array and payload must
equal the matching run of the GPU stream's size array and payload.  Every
chunk lies in one slice, so the whole stream is covered.
"""
import os
import struct
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CHUNK = 1025


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def codec():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2511_04140_amd import codec as C
    c = C.Codec(0)
    yield c
    c.close()


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


class _Stream:
    """A GPU stream copied to the host, split into header, sizes, payload."""

    def __init__(self, s_dev, n):
        self.nc = (n + CHUNK - 1) // CHUNK
        self.hdr = s_dev[:32].cpu().numpy().tobytes()
        self.sizes = s_dev[32:32 + 4 * self.nc].cpu().numpy().view(np.uint32).astype(np.int64)
        self.payload = s_dev[32 + 4 * self.nc:].cpu().numpy()
        self.offs = np.concatenate([[0], np.cumsum(self.sizes)])
        self.length = s_dev.numel()


def _compare_slices(orc, st, make_slice, blocks, label):
    """blocks: list of (c0, c1) chunk ranges; make_slice(c0, c1) returns the
    input values of those chunks.  The oracle compresses each block in a
    thread pool; the block's sizes and payload must equal the GPU's."""
    def work(b):
        c0, c1 = b
        o = orc.compress(make_slice(c0, c1))
        k = c1 - c0
        so = np.frombuffer(o, np.uint8, 4 * k, 32).view(np.uint32).astype(np.int64)
        po = np.frombuffer(o, np.uint8, len(o) - 32 - 4 * k, 32 + 4 * k)
        if not np.array_equal(st.sizes[c0:c1], so):
            bad = c0 + int(np.nonzero(st.sizes[c0:c1] != so)[0][0])
            return f"{label}: chunk {bad} size {st.sizes[bad]} vs oracle {so[bad - c0]}"
        if not np.array_equal(st.payload[st.offs[c0]:st.offs[c1]], po):
            return f"{label}: payload of chunks {c0}..{c1 - 1} differs"
        return None
    with ThreadPoolExecutor(_threads()) as ex:
        for err in ex.map(work, blocks):
            assert err is None, err


def _blocks(nc, per):
    return [(c, min(nc, c + per)) for c in range(0, nc, per)]


def _check_header(orc, st, n, dt_code):
    assert st.hdr[:4] == b"FLCN" and st.hdr[4] == 1 and st.hdr[5] == dt_code
    N, payload = struct.unpack_from("<QQ", st.hdr, 16)
    assert N == n and payload == int(st.offs[-1]) and st.length == 32 + 4 * st.nc + payload
    # the rest of the header equals the oracle's for any stream of this dtype
    ref = orc.compress(np.zeros(1, np.float64 if dt_code == 2 else np.float32))
    assert st.hdr[:16] == ref[:16]


def _whole_stream(codec, orc, x, label, per_block=4096):
    _log(f"[stream] {label}: n={x.size} ({x.nbytes / 2**30:.3f} GiB)")
    xd = torch.from_numpy(x).cuda()
    s = codec.compress(xd)
    torch.cuda.synchronize()
    st = _Stream(s, x.size)
    _check_header(orc, st, x.size, 2 if x.dtype == np.float64 else 1)
    _compare_slices(orc, st, lambda c0, c1: x[c0 * CHUNK:c1 * CHUNK], _blocks(st.nc, per_block), label)
    y = codec.decompress(s)
    assert torch.equal(y.view(torch.uint8), xd.view(torch.uint8)), f"{label}: round trip"
    _log(f"[stream] {label}: {st.nc} chunks identical, ratio {st.length / x.nbytes:.4f}")
    del xd, s, y
    torch.cuda.empty_cache()


def test_whole_stream_walk_2p20(codec, orc):
    """The 2^20-value Gaussian walk at two decimals: one oracle call."""
    from paper_2511_04140_amd import workloads as W
    x = W.walk_f64(1 << 20, seed=1)
    xd = torch.from_numpy(x).cuda()
    got = codec.compress(xd).cpu().numpy().tobytes()
    assert got == orc.compress(x)


def test_whole_stream_sensor_f64_2gib(codec, orc):
    from paper_2511_04140_amd import workloads as W
    _log("[stream] generating sensor_f64 2^28")
    _whole_stream(codec, orc, W.sensor_f64(1 << 28, seed=2), "sensor_f64")


def test_whole_stream_mixed_f32_2gib(codec, orc):
    from paper_2511_04140_amd import workloads as W
    _log("[stream] generating mixed_f32 2^29")
    _whole_stream(codec, orc, W.mixed_f32(1 << 29, seed=3), "mixed_f32")


def test_every_float32_pattern(codec, orc):
    """All 2^32 binary32 bit patterns in increasing order, 16 GiB, through one
    compression and one decompression on the device: the round trip is
    bit-exact, and every 16th run of 4096 chunks (plus the last, partial
    one) is byte-identical to the oracle's stream of those values."""
    n = 1 << 32
    _log("[f32-all] building the 2^32 patterns on the device")
    xd = torch.empty(n, dtype=torch.int32, device="cuda")
    step = 1 << 28
    for lo in range(0, n, step):
        v = torch.arange(lo, lo + step, dtype=torch.int64, device="cuda")
        v = torch.where(v >= (1 << 31), v - (1 << 32), v)
        xd[lo:lo + step] = v.to(torch.int32)
        del v
    xf = xd.view(torch.float32)
    _log("[f32-all] compress")
    s = codec.compress(xf)
    torch.cuda.synchronize()
    st = _Stream(s, n)
    _check_header(orc, st, n, 1)
    _log(f"[f32-all] stream {st.length} bytes; decompress")
    y = codec.decompress(s)
    assert torch.equal(y.view(torch.int32), xd), "round trip of every pattern"
    del y, xd, xf, s
    torch.cuda.empty_cache()
    per = 4096
    blocks = [b for i, b in enumerate(_blocks(st.nc, per)) if i % 16 == 5 or b[1] == st.nc]

    def make(c0, c1):
        lo, hi = c0 * CHUNK, min(n, c1 * CHUNK)
        return np.arange(lo, hi, dtype=np.uint64).astype(np.uint32).view(np.float32)
    _log(f"[f32-all] oracle on {len(blocks)} runs of {per} chunks")
    _compare_slices(orc, st, make, blocks, "every_f32_pattern")


def _edge_chunks_f64():
    """Chunks whose encoding sits on an edge of the format (each 1025 values)."""
    rng = np.random.default_rng(8)
    out = []

    def ones(k):  # w = 1, exactly k non-zero row bytes (lambda = 128 - k)
        z = np.zeros(CHUNK - 1, np.int64)
        z[: 8 * k: 8] = 1
        return (1000 - np.concatenate([[0], np.cumsum(z)])).astype(np.float64)
    out += [ones(112), ones(111), ones(128), ones(1), ones(16), ones(17)]
    bits = rng.integers(0, 1 << 64, CHUNK, dtype=np.uint64, endpoint=False)
    bits[1] = np.uint64(0x7FF8000000000001)  # worst case: every row dense, w = 64
    out.append(bits.view(np.float64))
    for k in (0, 1, 2, 7, 8, 9, 30, 31, 32, 33, 49, 61, 62):
        v = np.zeros(CHUNK)
        v[500] = float(2 ** k)  # w = k + 2
        out.append(v)
    # the worked values of Alg. 2, each inside a chunk of two-place decimals
    examples = [-0.0314, 1.11, 111.0, 111.00000000000001, 1.02, 2.5, 8.04, 9.110900773177071,
                1.23456789876543e-09, 0.0, 7.15, -1.2]
    for i, e in enumerate(examples):
        v = np.round(rng.normal(0, 50, CHUNK), 2)
        v[(37 * i) % CHUNK] = e
        out.append(v)
        out.append(np.full(CHUNK, e))
    # Case 1 at the integer limit of Eq. 3 and beta-hat = 15 exactly
    out.append(np.tile([999999999999999.0, -999999999999999.0, 0.5], 342)[:CHUNK])
    out.append(np.tile([99999999999999.9, -0.1], 513)[:CHUNK])
    return out


def _edge_chunks_f32():
    rng = np.random.default_rng(9)
    out = []
    for v in _edge_chunks_f64()[:6]:  # integer-valued, exact in binary32
        out.append(v.astype(np.float32))
    bits = rng.integers(0, 1 << 32, CHUNK, dtype=np.uint64).astype(np.uint32)
    bits[0] = np.uint32(0x7FC00001)
    out.append(bits.view(np.float32))
    for k in (0, 1, 7, 8, 14, 15, 16, 29, 30):
        v = np.zeros(CHUNK, np.float32)
        v[300] = np.float32(2.0 ** k)
        out.append(v)
    for e in (1.5, 0.1, 999999.0, 99999.9, 1.234567, 3.4028235e38, 1e-10, 1.17549435e-38):
        v = np.round(rng.normal(0, 5, CHUNK), 1).astype(np.float32)
        v[11] = np.float32(e)
        out.append(v)
    return out


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_edge_chunks(codec, orc, dt):
    """The oracle's edge chunks back to back in one stream (the scheme tie
    lambda = 16 / 17, one and all non-zero bytes, the all-dense worst case,
    every bit width edge, the worked values of Alg. 2 inside chunks), plus a
    partial last chunk: byte-identical streams, bit-exact round trip."""
    parts = _edge_chunks_f64() if dt == "f64" else _edge_chunks_f32()
    x = np.concatenate(parts + [parts[3][:100]])
    xd = torch.from_numpy(x).cuda()
    s = codec.compress(xd)
    assert s.cpu().numpy().tobytes() == orc.compress(x)
    y = codec.decompress(s)
    assert torch.equal(y.view(torch.uint8), xd.view(torch.uint8))


def test_batch_plan_more_chunks_than_waves(codec, orc):
    """A tuned, graph-captured batch plan over 14 series of about 1,000
    chunks each (14,000 chunks, more than the 4,096 waves the device holds at
    once, so waves take many chunks each), replayed three times: every
    series' stream equals the oracle's, and the decompression plan gives
    every bit back."""
    from paper_2511_04140_amd import workloads as W
    rng = np.random.default_rng(21)
    xs = []
    for i in range(14):
        n = int(rng.integers(900 * CHUNK, 1100 * CHUNK)) + int(rng.integers(0, CHUNK))
        if i % 3 == 0:
            xs.append(W.sensor_f64(n, seed=400 + i))
        elif i % 3 == 1:
            xs.append(W.decimal_f64(n, seed=400 + i, places=int(rng.integers(0, 7))))
        else:
            xs.append(W.decimal_f32(n, seed=400 + i, places=int(rng.integers(0, 5))))
    total = sum((x.size + CHUNK - 1) // CHUNK for x in xs)
    _log(f"[batch-big] {len(xs)} series, {total} chunks")
    assert total > 4096 * 3
    xd = [torch.from_numpy(x).cuda() for x in xs]
    plan = codec.plan_compress(xd, tune=True, graph=True)
    with ThreadPoolExecutor(_threads()) as ex:
        want = list(ex.map(orc.compress, xs))
    for rep in range(3):
        torch.zeros(1 << 20, device="cuda").sum().item()  # eager work between replays
        streams = plan.run()
        for i, (s, w) in enumerate(zip(streams, want)):
            assert s.cpu().numpy().tobytes() == w, f"replay {rep}: series {i} differs"
    dplan = codec.plan_decompress(streams, [x.size for x in xs], [t.dtype for t in xd], tune=True, graph=True)
    for rep in range(2):
        ys = dplan.run()
        for x, y in zip(xd, ys):
            assert torch.equal(y.view(torch.uint8), x.view(torch.uint8)), f"replay {rep}"
    plan.close()
    dplan.close()


def test_batch_of_10000_series(codec, orc):
    """The 10,000-series batch of the batched measurement (lengths
    log-uniform on [1,024, 369,000] values, 60 % float64, 0-6 decimal places
    per series, about 4 GB) through one tuned, graph-captured compression
    plan and one decompression plan, writing into one device buffer each as
    the measurement does: every series' stream equals the oracle's byte for
    byte, and every series comes back bit for bit."""
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    xs = W.batch_series()
    tdt = lambda x: torch.float64 if x.dtype == np.float64 else torch.float32
    align = lambda v: (v + 255) // 256 * 256
    in_off, out_off, bounds = [], [], []
    ti = to = 0
    for x in xs:
        in_off.append(ti)
        ti += align(x.nbytes)
        bounds.append(C.compress_bound(x.size, tdt(x)))
        out_off.append(to)
        to += align(bounds[-1])
    _log(f"[batch-10000] {len(xs)} series, {sum(x.nbytes for x in xs) / 1e9:.3f} GB")
    host = np.zeros(ti, np.uint8)
    for x, o in zip(xs, in_off):
        host[o:o + x.nbytes] = x.view(np.uint8)
    xin = torch.from_numpy(host).cuda()
    del host
    xv = [xin[o:o + x.nbytes].view(tdt(x)) for x, o in zip(xs, in_off)]
    out = torch.zeros(to, dtype=torch.uint8, device="cuda")
    ov = [out[o:o + b] for o, b in zip(out_off, bounds)]
    plan = codec.plan_compress(xv, outs=ov, tune=True, graph=True)
    streams = plan.run()
    lens = [s.numel() for s in streams]
    got = out.cpu().numpy()
    _log(f"[batch-10000] plan {plan.info()['form']}, streams {sum(lens):,} bytes; oracle")

    def check(i):
        w = orc.compress(xs[i])
        g = got[out_off[i]:out_off[i] + lens[i]].tobytes()
        return None if g == w else f"series {i} ({xs[i].size} values, {xs[i].dtype}) differs from the oracle"

    with ThreadPoolExecutor(_threads()) as ex:
        for err in ex.map(check, range(len(xs))):
            assert err is None, err
    yin = torch.zeros_like(xin)
    yv = [yin[o:o + x.nbytes].view(tdt(x)) for x, o in zip(xs, in_off)]
    dplan = codec.plan_decompress(streams, [x.size for x in xs], [tdt(x) for x in xs], outs=yv, tune=True,
                                  graph=True)
    dplan.run()
    assert torch.equal(yin, xin), "round trip of the batch"
    _log("[batch-10000] every series equals the oracle's stream and round-trips")
    plan.close()
    dplan.close()
    del xin, out, yin
    torch.cuda.empty_cache()

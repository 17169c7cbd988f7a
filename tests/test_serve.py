"""Serving loop (falcon_server): continuous batching with HBM-budget
admission.  Each request's result must be the same alone and in the mix:
compressed streams byte-identical to the oracle's stream of that input
alone, decompressed values bit-identical to the original."""
import sys
import time

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
    c = C.Codec(0)
    yield c
    c.close()


def _payloads(seed, count, max_values=300_000):
    """Log-uniform sizes, both dtypes, sensor-like content."""
    from paper_2511_04140_amd import workloads as W
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(1), np.log(max_values)))) if i > 1 else i
        x = W.sensor_f64(n, seed=seed * 100 + i) if n else np.zeros(0)
        if i % 2:
            x = x.astype(np.float32)
        out.append(np.ascontiguousarray(x))
    return out


def _drain(srv, expect, timeout_s=60.0, release=True, keep=None):
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < expect:
        assert time.time() < t_end, f"only {len(got)} of {expect} completions"
        for c in srv.poll(wait_ms=20):
            got[c["tag"]] = c
            if keep is not None:
                keep(c)
            if release:
                srv.release(c)
    return got


def _check_mix(codec, orc, srv, xs, streams):
    """Submits compress requests for every xs and decompress requests for
    every (stream, x); checks every result against the input alone."""
    xd = [torch.from_numpy(x).cuda() for x in xs]
    sd = [torch.from_numpy(np.frombuffer(s, np.uint8).copy()).cuda() for s in streams]
    torch.cuda.synchronize()
    results = {}

    def keep(c):
        if c["status"] == 0:
            tag = c["tag"]
            dt = torch.uint8 if tag < 10_000 else (torch.float64 if xs[tag - 10_000].dtype == np.float64
                                                  else torch.float32)
            results[tag] = srv.view(c, dt).cpu().numpy().copy()

    for i in range(len(xs)):  # interleave both kinds
        srv.submit_compress(xd[i], tag=i)
        srv.submit_decompress(sd[i], xs[i].size, xd[i].dtype, tag=10_000 + i)
    got = _drain(srv, 2 * len(xs), keep=keep)
    for tag, c in got.items():
        assert c["status"] == 0, (tag, c)
    for i, x in enumerate(xs):
        assert results[i].tobytes() == streams[i], f"compress request {i} (n={x.size}, {x.dtype})"
        y = results[10_000 + i]
        assert np.array_equal(y.view(np.uint8), x.view(np.uint8)), f"decompress request {i}"
    return got


@pytest.mark.parametrize("lanes,max_batch", [(4, 256), (1, 1), (2, 8)], ids=["batched", "fifo", "small"])
def test_results_same_alone_and_in_the_mix(codec, orc, lanes, max_batch):
    from paper_2511_04140_amd import codec as C
    xs = _payloads(31, 60)
    streams = [orc.compress(x) for x in xs]
    # alone: the one-series device calls give the same bytes
    for x, s in zip(xs[:6], streams[:6]):
        assert codec.compress(torch.from_numpy(x).cuda()).cpu().numpy().tobytes() == s
    srv = C.Server(codec, hbm_budget=256 << 20, lanes=lanes, max_batch=max_batch)
    _log(f"[serve] lanes={lanes} max_batch={max_batch}: {len(xs)} compress + {len(xs)} decompress")
    got = _check_mix(codec, orc, srv, xs, streams)
    lat = sorted(c["complete_us"] - c["submit_us"] for c in got.values())
    _log(f"[serve] latency p50 {lat[len(lat) // 2]:.0f} us, max {lat[-1]:.0f} us")
    assert srv.in_flight() == 0
    srv.close()


def test_admission_by_budget(codec, orc):
    """Outputs far larger in total than the pool: requests wait for
    releases and all complete; one larger than the whole pool fails."""
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    budget = 4 << 20
    srv = C.Server(codec, hbm_budget=budget, lanes=3, max_batch=4)
    xs = [W.sensor_f64(100_000 + 1000 * i, seed=40 + i) for i in range(40)]   # ~0.8 MB bound each
    xd = [torch.from_numpy(x).cuda() for x in xs]
    torch.cuda.synchronize()
    big = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")          # bound > 4 MiB
    srv.submit_compress(big, tag=999)
    for i, t in enumerate(xd):
        srv.submit_compress(t, tag=i)
    outs = {}
    live = []
    t_end = time.time() + 60
    while len(outs) < len(xs) + 1:
        assert time.time() < t_end
        for c in srv.poll(wait_ms=20):
            if c["tag"] == 999:
                assert c["status"] == 5 and c["d_out"] is None  # out of memory
                outs[999] = None
                continue
            assert c["status"] == 0
            live.append(c)
            outs[c["tag"]] = srv.view(c).cpu().numpy().tobytes()
        # release all but the newest output so admission can proceed (with
        # one live output of at most 1.12 MB the 4 MiB pool always has a
        # hole that fits the largest request)
        while len(live) > 1:
            srv.release(live.pop(0))
    for c in live:
        srv.release(c)
    for i, x in enumerate(xs):
        assert outs[i] == orc.compress(x), i
    srv.close()


def test_corrupt_request_fails_alone(codec, orc):
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    xs = [W.walk_f64(5000 + 100 * i, seed=60 + i) for i in range(6)]
    streams = [np.frombuffer(orc.compress(x), np.uint8).copy() for x in xs]
    bad = streams[2].copy()
    nc = (xs[2].size + 1024) // 1025
    sizes = bad[32:32 + 4 * nc].view(np.uint32)
    bad[32 + 4 * nc + int(sizes[0]) + 10] = 70   # bit width above 64 in chunk 1
    streams[2] = bad
    sd = [torch.from_numpy(s).cuda() for s in streams]
    torch.cuda.synchronize()
    srv = C.Server(codec, hbm_budget=64 << 20, lanes=1, max_batch=16)
    for i, s in enumerate(sd):
        srv.submit_decompress(s, xs[i].size, torch.float64, tag=i)
    vals = {}
    got = _drain(srv, len(xs), keep=lambda c: vals.__setitem__(c["tag"], srv.view(c, torch.float64).cpu().numpy()
                                                                 if c["status"] == 0 else None))
    for i in range(len(xs)):
        if i == 2:
            assert got[i]["status"] == C.ERR_CORRUPT_STREAM
        else:
            assert got[i]["status"] == 0
            assert np.array_equal(vals[i].view(np.uint8), xs[i].view(np.uint8))
    srv.close()


def test_batches_overlap_on_the_device(codec, orc):
    """Continuous batching overlaps work on the device: with four lanes and
    one request per batch, some batch starts on one lane (device clock, HIP
    events) before a batch on another lane has ended.  Every result is still
    the oracle's."""
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    xs = [W.sensor_f64(2_000_000 + 1000 * i, seed=700 + i) for i in range(16)]
    xd = [torch.from_numpy(x).cuda() for x in xs]
    srv = C.Server(codec, hbm_budget=1 << 30, lanes=4, max_batch=1)
    keep = {}
    for i, x in enumerate(xd):
        srv.submit_compress(x, tag=i)
    got = _drain(srv, len(xd), release=False)
    for i, x in enumerate(xs):
        c = got[i]
        assert c["status"] == 0 and c["lane"] >= 0 and 0 <= c["dev_start_us"] < c["dev_end_us"]
        assert srv.view(c)[: c["out_len"]].cpu().numpy().tobytes() == orc.compress(x), i
        keep[i] = c
    spans = sorted((c["dev_start_us"], c["dev_end_us"], c["lane"]) for c in keep.values())
    overlaps = [(a, b) for a in spans for b in spans
                if a[2] != b[2] and a[0] < b[0] < a[1]]
    _log(f"[serve] {len(overlaps)} overlapping batch pairs on different lanes; spans {spans[:6]}")
    assert overlaps, "no batch started while another lane's batch was still running"
    assert len({c["lane"] for c in keep.values()}) > 1
    for c in keep.values():
        srv.release(c)
    srv.close()

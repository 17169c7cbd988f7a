"""Host -> host pipeline (Sec. 3.1: Alg. 1's event-driven scheduler, and the
Sync-Based and Pre-Allocation schedulers it is compared with, on HIP streams).

The pipeline's stream must be byte-identical to the oracle's and to the
device-resident call's for every scheduler and geometry (streams, batch
size), with pinned and pageable buffers, and decompression through the
pipeline must give back every bit.  Batches of 1 or 3 chunks over tens of
chunks make many batches complete out of launch order, which is what the
placement order of Alg. 1 has to get right.
"""
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
    c = C.Codec(0)
    yield c
    c.close()


def _host(x, pinned):
    t = torch.from_numpy(np.ascontiguousarray(x))
    return t.pin_memory() if pinned else t.clone()


def _inputs():
    from paper_2511_04140_amd import workloads as W
    rng = np.random.default_rng(77)
    spec = rng.choice(np.array([0x8000000000000000, 0x7FF0000000000000, 0x7FF8000000000123,
                                0x0000000000000001], np.uint64), 300).view(np.float64)
    sensor = W.sensor_f64(37 * 1025 + 11, seed=9)
    sensor[rng.integers(0, sensor.size, 300)] = spec
    return [
        ("sensor_f64", sensor),
        ("walk_f64_exact_chunks", W.walk_f64(24 * 1025, seed=1)),
        ("mixed_f32", W.mixed_f32(41 * 1025 + 600, seed=3, side=64)),
        ("one_value", np.array([3.25])),
    ]


@pytest.mark.parametrize("streams,batch", [(1, 4096), (3, 1), (4, 3), (4, 1024), (4, 2048), (16, 2), (16, 4096)])
@pytest.mark.parametrize("pinned", [True, False], ids=["pinned", "pageable"])
@pytest.mark.parametrize("sched", ["event", "sync", "prealloc"])
def test_pipeline_matches_oracle_and_device(codec, orc, streams, batch, pinned, sched):
    codec.set_pipeline(streams, batch)
    codec.set_scheduler(sched)
    for name, x in _inputs():
        _log(f"[pipeline] {name} n={x.size} streams={streams} batch={batch} pinned={pinned} sched={sched}")
        want = orc.compress(x)
        s = codec.compress_host(_host(x, pinned))
        assert s.is_pinned() == pinned
        got = s.numpy().tobytes()
        assert got == want, f"{name}: pipeline stream differs from oracle ({len(got)} vs {len(want)} bytes)"
        dev = codec.compress(torch.from_numpy(np.ascontiguousarray(x)).cuda()).cpu().numpy().tobytes()
        assert dev == got
        y = codec.decompress_host(_host(np.frombuffer(want, np.uint8).copy(), pinned)).numpy()
        assert y.dtype == x.dtype and np.array_equal(y.view(np.uint8), x.view(np.uint8)), name


def test_pipeline_empty_and_small_buffers(codec, orc):
    from paper_2511_04140_amd import codec as C
    codec.set_pipeline(4, 2)
    codec.set_scheduler("event")
    with pytest.raises(KeyError):
        codec.set_scheduler("round-robin")
    from paper_2511_04140_amd.codec import lib
    assert lib().falcon_set_pipeline_scheduler(codec._ctx, 3) == C.ERR_INVALID_ARG
    x = np.zeros(0, np.float32)
    s = codec.compress_host(torch.from_numpy(x))
    assert s.numpy().tobytes() == orc.compress(x)
    y = codec.decompress_host(s.clone())
    assert y.numel() == 0 and y.dtype == torch.float32
    x = np.arange(5000, dtype=np.float64) / 8
    t = torch.from_numpy(x)
    with pytest.raises(C.FalconError) as e:
        codec.compress_host(t, out=torch.empty(100, dtype=torch.uint8))
    assert e.value.status == C.ERR_BUFFER_TOO_SMALL
    s = codec.compress_host(t)
    with pytest.raises(C.FalconError) as e:
        codec.decompress_host(s, out=torch.empty(10, dtype=torch.float64))
    assert e.value.status == C.ERR_BUFFER_TOO_SMALL


def test_pipeline_rejects_corrupt_streams(codec, orc):
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    codec.set_pipeline(3, 2)
    x = W.walk_f64(9 * 1025 + 5, seed=4)
    good = np.frombuffer(orc.compress(x), np.uint8).copy()
    nc = 10
    sizes = good[32:32 + 4 * nc].view(np.uint32)
    # (1) a size outside the possible range: caught on the host
    bad = good.copy()
    bad[32:36] = np.frombuffer(np.uint32(5).tobytes(), np.uint8)
    with pytest.raises(C.FalconError) as e:
        codec.decompress_host(torch.from_numpy(bad))
    assert e.value.status == C.ERR_CORRUPT_STREAM
    # (2) a bit width above 64 inside chunk 7: caught by the decoder on the GPU
    off = 32 + 4 * nc + int(sizes[:7].sum())
    bad = good.copy()
    bad[off + 10] = 65
    with pytest.raises(C.FalconError) as e:
        codec.decompress_host(torch.from_numpy(bad))
    assert e.value.status == C.ERR_CORRUPT_STREAM
    # the pipeline still works afterwards
    y = codec.decompress_host(torch.from_numpy(good)).numpy()
    assert np.array_equal(y.view(np.uint8), x.view(np.uint8))


@pytest.mark.parametrize("pinned", [True, False], ids=["pinned", "pageable"])
def test_pipeline_full_size_sensor_f64(codec, pinned):
    """The 2 GiB float64 workload host -> host with the default geometry
    (4 streams, 2048-chunk batches): the stream of every scheduler equals the
    device-resident one and decompresses to the input."""
    from paper_2511_04140_amd import workloads as W
    codec.set_pipeline()
    x = W.sensor_f64(1 << 28, seed=2)
    xh = _host(x, pinned)
    dev = codec.compress(xh.cuda())
    for sched in ("event", "sync", "prealloc"):
        _log(f"[pipeline] full-size sensor_f64 pinned={pinned} sched={sched}")
        codec.set_scheduler(sched)
        s = codec.compress_host(xh)
        assert s.numel() == dev.numel()
        assert torch.equal(s.cuda(), dev), sched
    codec.set_scheduler("event")
    del dev
    y = codec.decompress_host(s)
    assert torch.equal(y.view(torch.uint8), xh.view(torch.uint8))

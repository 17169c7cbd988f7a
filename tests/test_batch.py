"""Many series in one launch: batch calls and plans (tuned, HIP graph).

Every series' stream must be byte-identical to the oracle's stream of that
series alone, whatever the launch form (split per dtype or mixed), the
workgroup size and grid the autotuner picks, and however often a captured
graph is replayed; decompression of a batch gives back every bit.
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


def _series(seed, count, max_chunks=40, dtypes=(np.float64, np.float32)):
    """Series of uneven lengths (0, 1, exact chunk multiples, ragged), both
    dtypes, decimals 0..6 per series, some with outliers and specials."""
    from paper_2511_04140_amd import workloads as W
    rng = np.random.default_rng(seed)
    out = []
    fixed = [0, 1, 1025, 2050, 64 * 1025, 65 * 1025 + 3]
    for i in range(count):
        n = fixed[i] if i < len(fixed) else int(rng.integers(1, max_chunks * 1025))
        dt = dtypes[i % len(dtypes)]
        d = int(rng.integers(0, 7))
        if dt == np.float64:
            x = W.decimal_f64(n, seed=seed * 1000 + i, places=d)
            if i % 5 == 3 and n > 10:
                x = W.sensor_f64(n, seed=seed * 1000 + i)
        else:
            x = W.decimal_f32(n, seed=seed * 1000 + i, places=min(d, 4))
            if i % 7 == 5 and n > 10:
                x[rng.integers(0, n, 3)] = np.array([np.nan, -0.0, np.inf], np.float32)
        out.append(np.ascontiguousarray(x))
    return out


def _check_streams(orc, xs, streams):
    for i, (x, s) in enumerate(zip(xs, streams)):
        got = s.cpu().numpy().tobytes()
        want = orc.compress(x)
        assert got == want, f"series {i} (n={x.size}, {x.dtype}): {len(got)} vs {len(want)} bytes"


def test_batch_compress_and_decompress_mixed_dtypes(codec, orc):
    xs = _series(11, 60)
    _log(f"[batch] {len(xs)} series, {sum(x.size for x in xs)} values")
    xd = [torch.from_numpy(x).cuda() for x in xs]
    streams = codec.compress_batch(xd)
    _check_streams(orc, xs, streams)
    ys = codec.decompress_batch(streams, [x.size for x in xs], [t.dtype for t in xd])
    for x, y in zip(xs, ys):
        assert np.array_equal(y.cpu().numpy().view(np.uint8), x.view(np.uint8))


@pytest.mark.parametrize("dtypes", [(np.float64,), (np.float32,)], ids=["f64", "f32"])
def test_batch_one_dtype(codec, orc, dtypes):
    xs = _series(12, 25, dtypes=dtypes)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    streams = codec.compress_batch(xd)
    _check_streams(orc, xs, streams)
    ys = codec.decompress_batch(streams, [x.size for x in xs], [t.dtype for t in xd])
    for x, y in zip(xs, ys):
        assert np.array_equal(y.cpu().numpy().view(np.uint8), x.view(np.uint8))


def test_batch_single_and_empty_series(codec, orc):
    for xs in ([np.zeros(0)], [np.zeros(0, np.float32), np.zeros(0)], [np.arange(7.0)]):
        xd = [torch.from_numpy(x).cuda() for x in xs]
        streams = codec.compress_batch(xd)
        _check_streams(orc, xs, streams)
        ys = codec.decompress_batch(streams, [x.size for x in xs], [t.dtype for t in xd])
        for x, y in zip(xs, ys):
            assert np.array_equal(y.cpu().numpy().view(np.uint8), x.view(np.uint8))


def test_plan_tuned_graph_replays(codec, orc):
    """A tuned, graph-captured compression plan replayed several times with
    eager work in between; new contents of the same buffers compress to the
    oracle's streams of the new contents."""
    xs = _series(13, 40)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    plan = codec.plan_compress(xd, tune=True, graph=True)
    info = plan.info()
    _log(f"[batch] plan info {info}")
    assert info["graph"] == 1 and (info["candidates"] >= 8 or info["from_cache"] == 1)
    for rep in range(3):
        streams = plan.run()
        _check_streams(orc, xs, streams)
        torch.cuda.synchronize()
        _ = (xd[1] * 2).sum().item()  # eager work between replays
    xs2 = _series(14, 40)
    xs2 = [np.resize(b, a.size).astype(a.dtype) for a, b in zip(xs, xs2)]
    for t, x in zip(xd, xs2):
        t.copy_(torch.from_numpy(x))
    streams = plan.run()
    _check_streams(orc, xs2, streams)
    # decompression plan over the streams just made
    dplan = codec.plan_decompress([s.clone() for s in streams], [x.size for x in xs2],
                                  [t.dtype for t in xd], tune=True, graph=True)
    for rep in range(2):
        ys = dplan.run()
        for x, y in zip(xs2, ys):
            assert np.array_equal(y.cpu().numpy().view(np.uint8), x.view(np.uint8))
    dplan.close()
    plan.close()


def test_plan_untuned_matches(codec, orc):
    xs = _series(15, 20)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    plan = codec.plan_compress(xd, tune=False, graph=False)
    _check_streams(orc, xs, plan.run())
    plan.close()


def test_batch_rejects_corrupt_and_mismatched(codec, orc):
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    xs = [W.walk_f64(9 * 1025 + 5, seed=4), W.decimal_f32(3000, seed=5, places=2)]
    streams = [torch.from_numpy(np.frombuffer(orc.compress(x), np.uint8).copy()).cuda() for x in xs]
    counts, dts = [x.size for x in xs], [torch.float64, torch.float32]
    ys = codec.decompress_batch(streams, counts, dts)
    for x, y in zip(xs, ys):
        assert np.array_equal(y.cpu().numpy().view(np.uint8), x.view(np.uint8))
    # a bit width above 64 in chunk 3 of the first series
    bad = streams[0].clone()
    sizes = bad[32:32 + 40].cpu().numpy().view(np.uint32)
    bad[32 + 40 + int(sizes[:3].sum()) + 10] = 65
    with pytest.raises(C.FalconError) as e:
        codec.decompress_batch([bad, streams[1]], counts, dts)
    assert e.value.status == C.ERR_CORRUPT_STREAM
    # a value count that disagrees with the stream header
    with pytest.raises(C.FalconError) as e:
        codec.decompress_batch(streams, [counts[0] - 1, counts[1]], dts)
    assert e.value.status == C.ERR_CORRUPT_STREAM
    # a dtype that disagrees with the stream header
    with pytest.raises(C.FalconError) as e:
        codec.decompress_batch(streams[1:], counts[1:], [torch.float64])
    assert e.value.status == C.ERR_CORRUPT_STREAM
    # still fine afterwards
    ys = codec.decompress_batch(streams, counts, dts)
    assert np.array_equal(ys[1].cpu().numpy().view(np.uint8), xs[1].view(np.uint8))


def test_single_pass_batch_and_plan(orc):
    """The work-queue form over many series (look-back stopping at each
    series' first chunk): a one-shot batch call on a context whose form is
    the single pass, and an untuned graph plan forced to it, replayed with
    eager work in between; every stream equals the oracle's."""
    from paper_2511_04140_amd import codec as C
    c = C.Codec(0, form="single_pass")
    xs = _series(17, 50)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    _check_streams(orc, xs, c.compress_batch(xd))
    plan = c.plan_compress(xd, tune=False, graph=True, single_pass=True)
    assert plan.info()["form"] == 1
    for rep in range(3):
        _check_streams(orc, xs, plan.run())
        _ = (xd[1] * 2).sum().item()
    plan.close()
    c.close()


def test_tuning_record_by_shape_class(codec, orc):
    """A second tuned plan of the same shape class (same dtypes, chunk and
    series counts within the same powers of two) takes the recorded
    geometry without timing, and still gives the oracle's streams."""
    xs = _series(18, 30)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    p1 = codec.plan_compress(xd, tune=True, graph=False)
    i1 = p1.info()
    p2 = codec.plan_compress(xd, tune=True, graph=False)
    i2 = p2.info()
    assert i2["from_cache"] == 1 and i2["candidates"] == 0
    assert (i2["split"], i2["waves_per_group"], i2["grid_percent"], i2["form"]) == \
        (i1["split"], i1["waves_per_group"], i1["grid_percent"], i1["form"])
    _check_streams(orc, xs, p2.run())
    p1.close()
    p2.close()

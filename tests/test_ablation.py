"""GPU parity of the ablation variants of Sec. 5.4.2 (Fig. 12b).

falcon_compress_variant must give the oracle's stream byte for byte under
every variant, on inputs spanning several chunks, ragged tails, special
values and decimal data where Elf's decimal places differ from Alg. 2's.
ELF and DENSE streams decode with the ordinary decompressor; a SPARSE stream
decodes when its chunks stay within the format's chunk bound and is reported
corrupt otherwise.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

VARIANTS = ("falcon", "elf", "sparse", "dense")


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


def _inputs():
    from paper_2511_04140_amd import workloads as W
    rng = np.random.default_rng(21)
    sensor = W.sensor_f64(23 * 1025 + 301, seed=4)
    sensor[rng.integers(0, sensor.size, 40)] = np.array([np.nan, np.inf, -0.0, 5e-324])[rng.integers(0, 4, 40)]
    two_places = np.rint(rng.uniform(-20, 20, 9 * 1025 + 5) * 100) / 100  # 1.11-like values
    worst = np.where(np.arange(3 * 1025) % 2 == 0, 0.0, 2.0)
    worst[::1025] = np.nan                      # every chunk all-sparse worst case
    worst32 = worst.astype(np.float32)
    return [
        ("sensor_f64", sensor),
        ("two_places_f64", two_places),
        ("walk_f64", W.walk_f64(17 * 1025, seed=5)),
        ("decimal_f64_6", W.decimal_f64(5 * 1025 + 1, seed=6, places=6)),
        ("mixed_f32", W.mixed_f32(29 * 1025 + 640, seed=7, side=32)),
        ("decimal_f32_2", W.decimal_f32(7 * 1025 + 100, seed=8, places=2)),
        ("sparse_worst_f64", worst),
        ("sparse_worst_f32", worst32),
        ("one_value", np.array([1.11])),
        ("empty_f32", np.zeros(0, np.float32)),
    ]


@pytest.mark.parametrize("variant", VARIANTS)
def test_variant_matches_oracle(codec, orc, variant):
    from paper_2511_04140_amd import codec as C
    for name, x in _inputs():
        _log(f"[ablation] {variant} {name} n={x.size}")
        want = orc.compress(x, variant)
        xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        got = codec.compress_variant(xd, variant).cpu().numpy().tobytes()
        assert got == want, f"{variant} {name}: {len(got)} vs {len(want)} bytes"
        if variant == "falcon":
            assert got == codec.compress(xd).cpu().numpy().tobytes()
        nc = (x.size + 1024) // 1025
        sizes = np.frombuffer(want[32:32 + 4 * nc], np.uint32)
        chunk_max = 11 + 8 + 64 * 128 if x.dtype == np.float64 else 7 + 4 + 32 * 128
        s = torch.from_numpy(np.frombuffer(want, np.uint8).copy()).cuda()
        if sizes.size == 0 or sizes.max() <= chunk_max:
            y = codec.decompress(s).cpu().numpy()
            assert np.array_equal(y.view(np.uint8), x.view(np.uint8)), (variant, name)
        else:
            assert variant == "sparse"
            with pytest.raises(C.FalconError) as e:
                codec.decompress(s)
            assert e.value.status == C.ERR_CORRUPT_STREAM


def test_elf_changes_the_two_place_data(codec, orc):
    """On values with two decimals, the trial test overestimates some
    decimal places (as 1.11 -> 3), so chunk headers differ from Alg. 2's."""
    x = _inputs()[1][1]
    xd = torch.from_numpy(x).cuda()
    a = codec.compress(xd).cpu().numpy().tobytes()
    b = codec.compress_variant(xd, "elf").cpu().numpy().tobytes()
    assert a != b and len(b) > len(a)


def test_variant_arguments(codec):
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd.codec import lib
    x = torch.arange(3000, dtype=torch.float64, device="cuda") / 4
    with pytest.raises(KeyError):
        codec.compress_variant(x, "elf*")
    assert lib().falcon_compress_bound_variant(3000, 2, 4) == 0
    cap = lib().falcon_compress_bound_variant(3000, 2, 2)
    assert cap == 32 + 3 * (4 + 11 + 8 + 64 * 144)
    small = torch.empty(lib().falcon_compress_bound(3000, 2), dtype=torch.uint8, device="cuda")
    with pytest.raises(C.FalconError) as e:
        codec.compress_variant(x, "sparse", out=small)
    assert e.value.status == C.ERR_BUFFER_TOO_SMALL
    s = codec.compress_variant(x, "dense", out=small)
    y = codec.decompress(s)
    assert torch.equal(y, x)

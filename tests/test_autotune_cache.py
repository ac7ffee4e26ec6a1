"""Lane choice of the batch autotuner from cached timings (no GPU needed)."""
import json

from paper_2302_13680_amd import autotune, binding


class _Ctx:
    def __init__(self, n, N, precision=binding.SMG_F32):
        self.n, self.N, self.precision = n, N, precision


def _write(path, entries):
    with open(path, "w") as fh:
        json.dump(entries, fh)


def test_choice_respects_batch_samples_per_lane(tmp_path):
    cache = tmp_path / "tune.json"
    # N=128 is fastest with 32 lanes in isolation (4 samples per lane), but the
    # batch also holds N=16, and ceil(128/64) = 2 samples per lane is possible
    _write(cache, {
        "127x128:f32:gfx950": {"best": 32, "us": {"64": 11.0, "32": 10.0, "16": 12.0}},
        "63x16:f32:gfx950": {"best": 8, "us": {"16": 3.0, "8": 2.5}},
        "255x64:f32:gfx950": {"best": 32, "us": {"64": 9.0, "32": 8.0, "16": 9.5}},
    })
    ctxs = [_Ctx(127, 128), _Ctx(63, 16), _Ctx(255, 64)]
    lanes, _ = autotune.tune(ctxs, str(cache))
    assert lanes == [64, 8, 32]
    assert max(-(-c.N // w) for c, w in zip(ctxs, lanes)) == 2


def test_single_small_instance_keeps_fastest(tmp_path):
    cache = tmp_path / "tune.json"
    _write(cache, {"31x8:f64:gfx950": {"best": 8, "us": {"8": 1.0}}})
    lanes, _ = autotune.tune([_Ctx(31, 8, binding.SMG_F64)], str(cache))
    assert lanes == [8]

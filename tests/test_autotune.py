"""Tile-shape autotuner: size classes, cache lookup order (user cache, then
the packaged table, then 64 x 64), the architecture fallback, and the table
written from a benchmark line.  The GPU test times real candidates."""
import json

import pytest
import torch

from paper_1608_04431_amd import autotune


def test_size_class():
    assert autotune.size_class(1, 1) == "64"
    assert autotune.size_class(64, 10) == "64"
    assert autotune.size_class(65, 10) == "128"
    assert autotune.size_class(100, 4096) == "4096"
    assert autotune.size_class(4097, 3) == "8192"
    assert autotune.size_class(32768, 32768) == "32768"


def test_lookup_order_and_fallback(tmp_path, monkeypatch):
    packaged = tmp_path / "packaged.json"
    packaged.write_text(json.dumps({"gfx950": {"512": {"tile": [32, 64]}},
                                    "gfx950|batch": {"512": {"tile": [48, 64]}}}))
    monkeypatch.setattr(autotune, "PACKAGED", str(packaged))
    user = tmp_path / "user.json"
    t = autotune.Tuner(path=str(user))
    t.key = "Some GPU|gfx950"
    assert t.tile_for(300, 500) == (32, 64)                # packaged, by architecture
    assert t.tile_for(300, 500, batch=True) == (48, 64)
    assert t.tile_for(3000, 10) == (32, 64)                # nearest tuned class (512)
    assert t.tile_for(3000, 10, batch=True) == (48, 64)
    t.user = {"Some GPU|gfx950": {"512": {"tile": [64, 32]}}}
    assert t.tile_for(300, 500) == (64, 32)                # user cache first
    assert t.tile_for(300, 500, batch=True) == (48, 64)    # batch keeps its own entry
    t.save()
    assert json.loads(user.read_text()) == t.user
    # per-call shapes where an entry has them; the shared shape otherwise
    t.user = {"Some GPU|gfx950": {"512": {"tile": [64, 32], "tile_fwd": [64, 44], "tile_adj": [48, 48]}}}
    assert t.tile_for(300, 500, kind="fwd") == (64, 44)
    assert t.tile_for(300, 500, kind="adj") == (48, 48)
    assert t.tile_for(300, 500) == (64, 32)
    t.user = {"Some GPU|gfx950": {"512": {"tile": [64, 32]}}}
    assert t.tile_for(300, 500, kind="fwd") == (64, 32)
    t.key = "Other|gfx942"
    assert t.tile_for(300, 500) == autotune.DEFAULT_TILE   # nothing for the architecture


def test_nearest_class(tmp_path, monkeypatch):
    """A size class with no entry takes the nearest tuned class in powers of
    two (the larger on a tie); the user's cache first at equal distance."""
    packaged = tmp_path / "packaged.json"
    packaged.write_text(json.dumps({"gfx950": {"8192": {"tile": [64, 40]}, "32768": {"tile": [64, 32]},
                                               "128": {"tile": [32, 32]}}}))
    monkeypatch.setattr(autotune, "PACKAGED", str(packaged))
    t = autotune.Tuner(path=str(tmp_path / "user.json"))
    t.key = "Some GPU|gfx950"
    assert t.tile_for(44001, 53688) == (64, 32)     # 65536 -> 32768
    assert t.tile_for(1 << 20, 5) == (64, 32)
    assert t.tile_for(16384, 100) == (64, 32)       # 16384: 8192 and 32768 tie -> the larger
    assert t.tile_for(3000, 3000) == (64, 40)       # 4096 -> 8192
    assert t.tile_for(200, 100) == (32, 32)         # 256 -> 128
    assert t.tile_for(8192, 8192) == (64, 40)       # exact
    t.user = {"Some GPU|gfx950": {"16384": {"tile": [48, 64]}}}
    assert t.tile_for(30000, 7) == (64, 32)         # exact packaged entry beats a near user one
    assert t.tile_for(10000, 7) == (48, 64)         # exact user entry
    t.user = {"Some GPU|gfx950": {"65536": {"tile": [48, 64]}}}
    assert t.tile_for(100000, 100) == (48, 64)      # 131072: the user's 65536 is nearer than 32768
    assert t.tile_for(16384, 100) == (64, 32)       # 16384: 32768 (distance 1) before 65536 (2)
    t.user = {"Some GPU|gfx950": {"8192": {"tile": [48, 64]}}}
    assert t.tile_for(3000, 3000) == (48, 64)       # 4096 -> 8192, the user's entry first


def test_table_from_bench():
    bench = {"config": {"rows": 32768, "cols": 32768},
             "tile_sweep_ms_per_step": {"64x64": 30.0, "64x48": 29.0},
             "tile_sweep_ms_fwd": {"64x64": 16.0, "64x48": 17.0},
             "tile_sweep_ms_adj": {"64x64": 14.0, "64x48": 12.0},
             "batched": {"tuning_ms": {"256": {"64x64": 2.0, "32x32": 1.5}},
                         "tuning_single_ms": {"256": {"64x64": 0.5, "32x32": 0.4}}}}
    t = autotune.table_from_bench(bench, "gfx950")
    assert t["gfx950"]["32768"]["tile"] == [64, 48]
    assert t["gfx950"]["32768"]["tile_fwd"] == [64, 64]
    assert t["gfx950"]["32768"]["tile_adj"] == [64, 48]
    assert t["gfx950"]["256"]["tile"] == [32, 32]
    assert t["gfx950|batch"]["256"]["tile"] == [32, 32]


def test_packaged_table_is_valid():
    data = json.load(open(autotune.PACKAGED))
    for key, table in data.items():
        if key == "source":
            continue
        for cls, entry in table.items():
            for k in ("tile", "tile_fwd", "tile_adj"):
                if k in entry:
                    th, tw = entry[k]
                    assert 1 <= th <= 64 and 1 <= tw <= 64, (key, cls, k)


@pytest.mark.gpu
def test_tune_on_device(tmp_path):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    import oracle
    import synth
    import paper_1608_04431_amd as d8
    d8._lib.load()
    z = synth.dem(300, 200, seed=12, lambda0=64)
    dirs = torch.from_numpy(oracle.d8(z)).cuda()
    w = torch.from_numpy(synth.uniform(z.shape, 13)).cuda()
    t = autotune.Tuner(path=str(tmp_path / "tiles.json"))
    times = t.tune(dirs, w, w, candidates=((64, 64), (32, 32)), reps=1)
    assert set(times) == {(64, 64), (32, 32)} and all(v > 0 for v in times.values())
    assert t.tile_for(300, 200) == min(times, key=times.get)
    entry = json.load(open(tmp_path / "tiles.json"))[t.key]["512"]
    assert entry["tile"] and tuple(entry["tile_fwd"]) in times and tuple(entry["tile_adj"]) in times
    assert t.tile_for(300, 200, kind="adj") == tuple(entry["tile_adj"])
    samples = [(dirs, w, w), (dirs[:100].contiguous(), w[:100].contiguous(), w[:100].contiguous())]
    bt = t.tune_batch(samples, candidates=((64, 64), (32, 32)), reps=1)
    assert set(bt) == {(64, 64), (32, 32)}
    assert t.tile_for(300, 200, batch=True) == min(bt, key=bt.get)

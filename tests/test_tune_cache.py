"""Host logic of the tuner cache (no GPU): entries are keyed by ISA and
compute-unit count; per-mode lanes fall back to the exact configuration's;
an exact search keeps the per-mode entries it does not redo."""
import json

from paper_2206_13574_amd import tune


def test_best_config_and_mode_lanes(monkeypatch, tmp_path):
    cache = tmp_path / "tune_cache.json"
    cache.write_text(json.dumps({"gfx950x256|w": dict(lanes=256, groups=0, dir_log2_max=17, list_cap=1 << 16,
                                                       dir_factor=16, lanes_heuristic=64, lanes_learned=128)}))
    monkeypatch.setattr(tune, "_CACHE", str(cache))
    monkeypatch.setattr(tune, "_device_name", lambda: "gfx950x256")
    assert tune.best_config("w") == dict(lanes=256, groups=0, dir_log2_max=17, list_cap=1 << 16, dir_factor=16)
    assert tune.best_lanes("w", "heuristic") == 64 and tune.best_lanes("w", "learned") == 128
    # no entry: the defaults, and the exact lanes for the pruning modes
    assert tune.best_config("other") == tune.DEFAULT
    assert tune.best_lanes("other", "learned") == tune.DEFAULT["lanes"]
    # another device: nothing cached applies
    monkeypatch.setattr(tune, "_device_name", lambda: "gfx942x304")
    assert tune.best_lanes("w", "heuristic") == tune.DEFAULT["lanes"]


def test_shipped_cache_has_the_bench_workload():
    c = json.loads(open(tune._CACHE).read())
    e = c["gfx950x256|cfg2"]
    assert e["lanes"] in (64, 128, 256, 512)
    assert e["lanes_heuristic"] in (64, 128, 256, 512) and e["lanes_learned"] in (64, 128, 256, 512)

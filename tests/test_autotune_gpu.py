"""The native autotuner (rl_autotune) times the kernel shapes on probes,
checks that none of them changes the counts, and its table round-trips
through the JSON cache: a cache written by the same library version is applied without
probing, one written by another library version is ignored."""
import json
import time

import pytest

from paper_1406_0559_amd import autotune
from paper_1406_0559_amd import raylens as rl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_tune_save_load_apply(tmp_path):
    ctx = rl.Context(0)
    path = str(tmp_path / "t.json")
    # a small budget: the first classes are tuned, the rest keep defaults
    table = autotune.tune(ctx, path, budget_ms=8000)
    assert table["library"] == rl.rl_version() and table["arch"].startswith("gfx")
    assert "fp32c/1" in table["entries"]
    for key, ent in table["entries"].items():
        prec, cls = key.split("/")
        assert ent["candidates"] >= 1 and ent["best_ms"] <= ent["worst_ms"]
        assert ctx.get_tuning(prec, int(cls)) == ent["shape"]
    assert table["entries"]["fp32c/1"]["candidates"] >= 5
    # a fresh context picks the table up from the cache without probing
    fresh = rl.Context(0)
    t0 = time.perf_counter()
    fresh.autotune(path, 0)
    assert time.perf_counter() - t0 < 2.0
    for key, ent in table["entries"].items():
        prec, cls = key.split("/")
        assert fresh.get_tuning(prec, int(cls)) == ent["shape"]
    assert autotune.apply(rl.Context(0), autotune.load(path))
    # another build's cache is neither applied nor accepted as budget-0 input
    other = json.load(open(path))
    other["library"] = "other"
    bad = str(tmp_path / "other.json")
    json.dump(other, open(bad, "w"))
    assert not autotune.apply(fresh, other)
    with pytest.raises(rl.RaylensError):
        fresh.autotune(bad, 0)

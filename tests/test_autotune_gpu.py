"""The autotuner times every kernel shape on a probe, checks that none of
them changes the counts, and its table round-trips through the JSON cache."""
import pytest

from paper_1406_0559_amd import autotune
from paper_1406_0559_amd import raylens as rl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_tune_save_load_apply(tmp_path):
    ctx = rl.Context(0)
    table = autotune.tune(ctx, precisions=("fp32c", "fp64"), classes=(0,), reps=1,
                          target_evals=2e9, min_rays=1 << 20)
    for key in ("fp32c/0", "fp64/0"):
        ent = table["entries"][key]
        assert ent["candidates"] >= 12 and ent["best_ms"] <= ent["worst_ms"]
    path = str(tmp_path / "t.json")
    autotune.save(table, path)
    back = autotune.load(path)
    fresh = rl.Context(0)
    assert autotune.apply(fresh, back)
    assert fresh.get_tuning("fp32c", 0) == table["entries"]["fp32c/0"]["shape"]
    back["library"] = "other"
    assert not autotune.apply(fresh, back)

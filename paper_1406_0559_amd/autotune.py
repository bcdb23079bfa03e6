"""Autotuner for the ray-shooting kernel shapes: a thin wrapper of the
library's native tuner, rl_autotune.

For each precision and tuning class (lens-count class, with or without
masses) the native tuner times the supported kernel shapes (rays per lane,
LDS lens tile, waves per workgroup, sub-map binning) on probe maps with HIP
events and keeps the fastest; for the batched persistent launch it also picks
the number of ray cells per work item. No shape changes a result bit (cells
and compensation blocks are constants of the grid), and the tuner checks that
on its probes: every candidate must reproduce the first candidate's counts
exactly.

The table is cached as JSON keyed by device architecture and library build
(rl_version), and applied to a context with `apply` (or by rl_autotune itself
when it finds a matching cache).
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional

from . import raylens as rl

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning_gfx950.json")
DEFAULT_BUDGET_MS = 600_000


def tune(ctx: "rl.Context", path: Optional[str] = None, budget_ms: int = DEFAULT_BUDGET_MS) -> Dict:
    """Probes every class within budget_ms, applies the result to ctx and
    writes the table to `path` (a temporary file if None). Returns the table."""
    import tempfile

    out = path
    tmpdir = None
    if out is None:
        tmpdir = tempfile.mkdtemp()
        out = os.path.join(tmpdir, "tuning.json")
    if os.path.exists(out):
        os.remove(out)          # a fresh table, not the cached one
    try:
        ctx.autotune(out, budget_ms)
        return load(out)
    finally:
        if tmpdir is not None:
            if os.path.exists(out):
                os.remove(out)
            os.rmdir(tmpdir)


def save(table: Dict, path: str = DEFAULT_CACHE) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def load(path: str = DEFAULT_CACHE) -> Optional[Dict]:
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def apply(ctx: "rl.Context", table: Optional[Dict]) -> bool:
    """Sets every cached shape on the context. Returns False if there is no
    table or it was made for another library build."""
    if not table or table.get("library") != rl.rl_version():
        return False
    for key, ent in table["entries"].items():
        prec, cls = key.split("/")
        ctx.set_tuning(prec, int(cls), **ent["shape"])
    return True


def tuned_context(device: int = 0, path: str = DEFAULT_CACHE) -> "rl.Context":
    """A context with the cached table applied (defaults if there is none)."""
    ctx = rl.Context(device)
    apply(ctx, load(path))
    return ctx


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description="time the kernel shapes and write the cache")
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--budget-ms", type=int, default=DEFAULT_BUDGET_MS)
    a = ap.parse_args()
    c = rl.Context(0)
    t = tune(c, a.out, a.budget_ms)
    for k, v in t["entries"].items():
        print(k, v["shape"], f"{v['probe_evals_per_s']:.3e} evals/s", f"{v['candidates']} candidates",
              flush=True)
    print("complete" if t.get("complete") else "budget reached before every class was tuned", flush=True)

"""Autotuner for the ray-shooting kernel shapes.

For each precision and lens-count class the tuner times every supported
kernel shape (rays per lane, LDS lens tile, waves per workgroup, sub-map
binning) on a probe map with HIP events on the launch stream and keeps the
fastest; for the batched persistent launch it also picks the number of ray
cells per work item. No shape changes a result bit (cells and compensation
blocks are constants of the grid), and the tuner checks that on its probes:
every candidate must reproduce the first candidate's counts exactly.

The table is cached as JSON keyed by device architecture and library
version, and applied to a context with `apply`.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time
from typing import Dict, Optional

import numpy as np

from . import inputs
from . import raylens as rl

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning_gfx950.json")
CLASS_PROBE_LENSES = {0: 400, 1: 2624, 2: 16000}


def candidates(precision: str):
    """Binning always goes through the LDS sub-map here: global-only binning
    is within a per cent in time but moves ~20x more bytes to memory (one
    device-scope atomic per binned ray instead of one per touched pixel)."""
    rays = [(4, 4), (2, 8), (8, 2), (4, 8), (8, 4)] if precision == "fp32c" else [(4, 4)]
    for (rx, ry), tile, waves, sub in itertools.product(rays, (128, 256, 512, 1024), (1, 2, 4),
                                                       (1, 2)):
        yield dict(rays_x=rx, rays_y=ry, lens_tile=tile, waves=waves, submap=sub)


# a probe must keep every SIMD busy for many rounds of waves, or the tail of
# the launch decides the ranking: >= 16 rounds of 256 CUs x 4 SIMDs x 3 waves
MIN_PROBE_RAYS = 16 * 256 * 4 * 3 * 1024


def probe_spec(n_lens: int, precision: str, target_evals: float,
               min_rays: int = MIN_PROBE_RAYS) -> inputs.MapSpec:
    """A GERLUMPH-like probe (kappa = 0.41, gamma = 0.38, 25 R_E window) with
    n_lens unit lenses and enough rays for ~target_evals evaluations (at
    least min_rays)."""
    base = inputs.config_gerlumph()
    rays = max(min_rays, int(target_evals / max(n_lens, 1)))
    n2 = int(math.sqrt(rays * base.h2 / base.h1))
    n1 = max(64, rays // max(n2, 1))
    R = math.sqrt(n_lens / base.kappa_star)
    return inputs.MapSpec(name=f"probe-{n_lens}", kappa=base.kappa, gamma=base.gamma, s=0.0,
                          n1=n1, n2=max(16, n2), h1=base.h1, h2=base.h2, p1=1024, p2=1024,
                          W1=25.0, W2=25.0, n_lens=n_lens, disc_radius=R, masses="unit", seed=99)


def _time(fn, reps, torch, stream):
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def tune(ctx: "rl.Context", precisions=("fp32c", "fp64"), classes=(0, 1, 2), reps: int = 2,
         target_evals: float = 2e11, verbose: bool = False,
         min_rays: int = MIN_PROBE_RAYS) -> Dict:
    """Times every candidate shape; returns the table (and leaves it applied)."""
    import torch

    stream = torch.cuda.current_stream()
    table = {"arch": torch.cuda.get_device_properties(0).gcnArchName.split(":")[0],
             "library": rl.rl_version(), "created": time.strftime("%Y-%m-%d %H:%M:%S"),
             "entries": {}}
    for prec in precisions:
        for cls in classes:
            n = CLASS_PROBE_LENSES[cls]
            te = target_evals if prec == "fp32c" else target_evals / 4
            spec = probe_spec(n, prec, te, min_rays)
            f = spec.lenses()
            L = rl.DeviceLenses(f.x1, f.x2, f.m)
            counts, esc = ctx.new_map(spec)
            ref = None
            results = []
            for cand in candidates(prec):
                ctx.set_tuning(prec, cls, item_cells=16, **cand)

                def run():
                    counts.zero_()
                    esc.zero_()
                    ctx.shoot(L, spec, prec, counts, esc, stream=stream)

                ms = _time(run, reps, torch, stream)
                got = counts.clone()
                if ref is None:
                    ref = got
                elif not torch.equal(ref, got):
                    raise RuntimeError(f"kernel shape {cand} changed the counts of {spec.name}")
                results.append((ms, cand))
                if verbose:
                    print(f"{prec} class {cls} {cand}: {ms:.3f} ms", flush=True)
            results.sort(key=lambda t: t[0])
            best_ms, best = results[0]
            # work-item size for the batched launch, with the best shape
            item_best, item_ms = 16, None
            maps = [probe_spec(max(200, n // 4), prec, te / 4, min_rays // 4),
                    probe_spec(n, prec, te / 4, min_rays // 4),
                    probe_spec(min(20000, n * 3), prec, te / 4, min_rays // 4)]
            fields = [m.lenses() for m in maps]
            Ls = [rl.DeviceLenses(x.x1, x.x2, x.m) for x in fields]
            outs = [ctx.new_map(m) for m in maps]
            for item in (4, 16, 64):
                ctx.set_tuning(prec, cls, item_cells=item, **best)

                def runb():
                    for c, e in outs:
                        c.zero_()
                        e.zero_()
                    ctx.shoot_batch([(Lb, m, c, e) for Lb, m, (c, e) in zip(Ls, maps, outs)], prec,
                                    stream=stream)

                ms = _time(runb, reps, torch, stream)
                if item_ms is None or ms < item_ms:
                    item_best, item_ms = item, ms
            entry = dict(best, item_cells=item_best)
            ctx.set_tuning(prec, cls, **entry)
            table["entries"][f"{prec}/{cls}"] = {
                "shape": entry, "probe": spec.name, "probe_evals": spec.evals, "best_ms": best_ms,
                "probe_evals_per_s": spec.evals / (best_ms / 1e3),
                "worst_ms": results[-1][0], "candidates": len(results), "batch_item_ms": item_ms,
                "top5": [dict(c, ms=m) for m, c in results[:5]]}
    return table


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
    table or it was made for another library version."""
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

    ap = argparse.ArgumentParser(description="time every kernel shape and write the cache")
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--evals", type=float, default=2e11)
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args()
    c = rl.Context(0)
    t = tune(c, reps=a.reps, target_evals=a.evals, verbose=a.v)
    save(t, a.out)
    for k, v in t["entries"].items():
        print(k, v["shape"], f"{v['probe_evals_per_s']:.3e} evals/s", flush=True)

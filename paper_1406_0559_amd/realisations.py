"""Realisation batches: mean MPD and spread over seeded lens fields.

Section 4's meanMPD tool shows, for one (kappa, gamma, s), the MPDs of 15
maps that differ only in the random positions of the microlenses, their mean
and standard deviation. Here the realisations are shot in one batched
persistent launch, binned in log10(mu / |mu_th|) on the device, and reduced
to the mean and sample standard deviation per bin on the device.
"""
from __future__ import annotations

import dataclasses
from typing import Dict

from . import raylens as rl


def realisation_specs(base, n: int = 15, seed0: int = 1000):
    return [dataclasses.replace(base, seed=seed0 + r, name=f"{base.name}-r{r:02d}") for r in range(n)]


def mean_mpd(ctx: "rl.Context", base, n: int = 15, nbins: int = 100, log_lo: float = -1.5,
             log_hi: float = 1.5, precision: str = "fp32c", seed0: int = 1000,
             stream=None) -> Dict:
    import torch

    specs = realisation_specs(base, n, seed0)
    fields = [s.lenses() for s in specs]
    Ls = [rl.DeviceLenses(f.x1, f.x2, f.m) for f in fields]
    maps = [ctx.new_map(s) for s in specs]
    ctx.shoot_batch([(L, s, c, e) for L, s, (c, e) in zip(Ls, specs, maps)], precision, stream=stream)
    # |mu_th| = |1 / ((1 - kappa)^2 - gamma^2)|, the macro-magnification that
    # Section 4's MPD tools measure mu against, from the library's map
    # statistics (every realisation shares kappa and gamma)
    mu_th = abs(ctx.stats(maps[0][0], maps[0][1], specs[0], stream=stream)["mu_th"])
    bins = torch.zeros((n, nbins + 2), dtype=torch.int64, device=maps[0][0].device)
    for r, (s, (c, _)) in enumerate(zip(specs, maps)):
        ctx.mpd(c, s, mu_th, log_lo, log_hi, nbins, bins=bins[r], stream=stream)
    mean, std = ctx.mpd_moments(bins, base.p1 * base.p2, stream=stream)
    return {"specs": specs, "fields": fields, "counts": [c for c, _ in maps],
            "escaped": [e for _, e in maps], "bins": bins, "mean": mean, "std": std,
            "mu_th": mu_th, "edges": (log_lo, log_hi, nbins)}

"""Whole full-size maps against the FP64 oracle, in the benchmark's launch
configuration (the tuned shapes of the cached table).

The oracle's whole maps of the GERLUMPH-like workload (30000^2 rays, 2624
lenses), the mixed-mass workload (20000^2 rays, 11560 lenses) and the 64 maps
of the batched workload (200-20000 lenses, 1024^2 maps) take about an hour on
8 host cores, so tests/golden/make_full_map_digests.py ran them once and
stored, per map, the sha256 of the count map, its binned and escaped counts,
16 band sums, and the number of rays whose oracle position lies within delta
of a pixel edge for a ladder of delta (tests/golden/full_map_digests.json).

Bars (Section 2.1, eq. 1 and 4; Appendix A on summation order):
  * FP64 path: the whole count map has the oracle's digest, bit for bit;
  * FP32-compensated path: per-ray |dy| <= 1e-4 Einstein radii on 64 evenly
    spaced and 16 seeded ray rows (rays within 0.015 of a lens reported
    apart), the mean magnification within 1e-3 of the oracle's, and the count
    bound: sum |N_ij - N_oracle_ij| <= 2 x (rays within max |dy| of a pixel
    edge), with max |dy| taken from the sampled rows and rounded up to the
    ladder, and again at delta = 1e-4;
  * the batch: every map of one persistent launch equals that map shot
    alone, bit for bit.
The oracle map in the count bound is the GPU's FP64 map of the same test,
used only after its digest has matched the oracle's.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_1406_0559_amd import inputs
from paper_1406_0559_amd import raylens as rl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DIGESTS = os.path.join(HERE, "golden", "full_map_digests.json")
TOL_Y = 1e-4
TOL_MEAN_MU = 1e-3
NEAR_LENS = 0.015


def digests():
    with open(DIGESTS) as fh:
        return json.load(fh)["maps"]


@pytest.fixture(scope="module")
def bench_ctx():
    """A context in bench.py's launch configuration: the tuned shapes of the
    cached table, applied the way bench.py applies them."""
    from paper_1406_0559_amd import autotune
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = rl.Context(0)
    try:
        c.autotune(autotune.DEFAULT_CACHE, 0)
    except rl.RaylensError:
        pass                      # no table for this library version: defaults, as in bench.py
    yield c
    c.close()


def sha(counts_np):
    return hashlib.sha256(np.ascontiguousarray(counts_np, "<i4").tobytes()).hexdigest()


def check_digest(counts_np, escaped, d, what):
    band = d["band_rows"]
    sums = [int(counts_np[k:k + band].sum(dtype=np.int64)) for k in range(0, counts_np.shape[0], band)]
    bad = [k for k, (a, b) in enumerate(zip(sums, d["band_sums"])) if a != b]
    assert not bad, f"{what}: band sums differ in bands {bad}"
    assert int(counts_np.sum(dtype=np.int64)) == d["binned"] and escaped == d["escaped"], what
    assert sha(counts_np) == d["sha256"], f"{what}: count map differs from the oracle's"


def sample_rows(n2, seed):
    even = np.linspace(0, n2 - 1, 64).astype(int)
    rnd = np.random.default_rng(seed).integers(0, n2, 16)
    return sorted(set(int(r) for r in np.concatenate([even, rnd])))


def per_ray_errors(ctx, L, spec, f, rows):
    """FP64 positions bit-identical and FP32 errors on the given rows; returns
    the largest FP32 |dy| over in-window rays away from lenses."""
    worst = 0.0
    lo1, lo2 = spec.w1 - 0.5 * spec.W1 - 1.0, spec.w2 - 0.5 * spec.W2 - 1.0
    for r in rows:
        o1, o2, _, rmin = oracle.ray_positions(f.x1, f.x2, f.m, spec.kappa, spec.gamma, spec.s,
                                               spec.n1, spec.n2, spec.c1, spec.c2, spec.h1,
                                               spec.h2, r, r + 1)
        g1, g2 = ctx.ray_positions(L, spec, "fp64", r, r + 1)
        assert (g1.cpu().numpy().view(np.int64) == o1.view(np.int64)).all(), f"{spec.name} row {r}"
        assert (g2.cpu().numpy().view(np.int64) == o2.view(np.int64)).all(), f"{spec.name} row {r}"
        y1, y2 = ctx.ray_positions(L, spec, "fp32c", r, r + 1)
        err = np.hypot(y1.cpu().numpy() - o1, y2.cpu().numpy() - o2)
        inwin = (o1 >= lo1) & (o1 < lo1 + spec.W1 + 2.0) & (o2 >= lo2) & (o2 < lo2 + spec.W2 + 2.0)
        far = inwin & (rmin >= NEAR_LENS)
        over = far & ~(err <= TOL_Y)
        assert not over.any(), f"{spec.name} row {r}: {int(over.sum())} rays over {TOL_Y}"
        if far.any():
            worst = max(worst, float(err[far].max()))
    return worst


def count_bound(d, max_dy):
    """2 x rays within delta of a pixel edge, delta the smallest ladder entry
    at or above max_dy (and at 1e-4)."""
    deltas = d["edge_deltas"]
    k = next(i for i, v in enumerate(deltas) if v >= max_dy)
    return deltas[k], 2 * d["rays_near_edge"][k], 2 * d["rays_near_edge"][deltas.index(TOL_Y)]


def check_fp32_against(c32_np, e32, c64_np, d, max_dy, spec, what):
    s32 = int(c32_np.sum(dtype=np.int64))
    assert s32 + e32 == spec.rays, f"{what}: ray conservation"
    assert abs(s32 - d["binned"]) / max(1, d["binned"]) <= TOL_MEAN_MU, f"{what}: mean mu"
    diff = int(np.abs(c32_np.astype(np.int64) - c64_np.astype(np.int64)).sum())
    delta, bound, bound_tol = count_bound(d, max_dy)
    assert diff <= bound, f"{what}: sum |dN| = {diff} > {bound} (delta {delta})"
    assert diff <= bound_tol
    return diff, delta, bound


@pytest.mark.parametrize("key,make", [("gerlumph", inputs.config_gerlumph),
                                      ("mixed", inputs.config_mixed)], ids=["gerlumph", "mixed"])
def test_full_size_map_against_the_oracle(bench_ctx, key, make):
    ctx = bench_ctx
    d = digests()[key]
    spec = make()
    assert d["name"] == spec.name and d["rays"] == spec.rays
    f = spec.lenses()
    L = rl.DeviceLenses(f.x1, f.x2, f.m)
    c64, e64 = ctx.shoot(L, spec, "fp64")
    c64_np = c64.cpu().numpy()
    check_digest(c64_np, int(e64.item()), d, f"{spec.name} FP64")
    print(f"  {spec.name}: FP64 map equals the oracle's", flush=True)
    max_dy = per_ray_errors(ctx, L, spec, f, sample_rows(spec.n2, 17))
    c32, e32 = ctx.shoot(L, spec, "fp32c")
    diff, delta, bound = check_fp32_against(c32.cpu().numpy(), int(e32.item()), c64_np, d, max_dy,
                                            spec, f"{spec.name} FP32")
    print(f"  {spec.name}: FP32 max |dy| {max_dy:.2e} on 80 rows; sum |dN| {diff} <= {bound} "
          f"(delta {delta:g}); {diff / d['binned']:.2e} of the binned rays", flush=True)


def test_batch_workload_against_the_oracle(bench_ctx):
    """The 64 maps of the batched workload: FP32 batch == each map alone; FP64
    batch == the oracle's maps; FP32 maps within the count bound."""
    ctx = bench_ctx
    dig = digests()
    maps = inputs.config_batch()
    fields = [m.lenses() for m in maps]
    Ls = [rl.DeviceLenses(f.x1, f.x2, f.m) for f in fields]
    out32 = [ctx.new_map(m) for m in maps]
    out64 = [ctx.new_map(m) for m in maps]
    ctx.shoot_batch([(L, m, c, e) for L, m, (c, e) in zip(Ls, maps, out32)], "fp32c")
    ctx.shoot_batch([(L, m, c, e) for L, m, (c, e) in zip(Ls, maps, out64)], "fp64")
    torch.cuda.synchronize()
    worst = 0.0
    for k, (m, f, L) in enumerate(zip(maps, fields, Ls)):
        d = dig[f"batch-{k:02d}"]
        assert d["name"] == m.name and d["rays"] == m.rays
        c64_np = out64[k][0].cpu().numpy()
        check_digest(c64_np, int(out64[k][1].item()), d, f"{m.name} FP64 batch")
        a, ea = ctx.shoot(L, m, "fp32c")
        c32_np = out32[k][0].cpu().numpy()
        assert (a.cpu().numpy() == c32_np).all() and int(ea.item()) == int(out32[k][1].item()), \
            f"{m.name}: FP32 batch differs from the map shot alone"
        rows = [int(r) for r in np.linspace(0, m.n2 - 1, 3)]
        max_dy = per_ray_errors(ctx, L, m, f, rows)
        worst = max(worst, max_dy)
        check_fp32_against(c32_np, int(out32[k][1].item()), c64_np, d, max_dy, m, f"{m.name} FP32")
    print(f"  64 batch maps: FP64 equal to the oracle's, FP32 batch == alone, max |dy| {worst:.2e}",
          flush=True)

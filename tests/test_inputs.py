"""Checks of the seeded input generators (lens fields, mass spectrum, workloads)."""
import math

import numpy as np
from scipy import stats

from paper_1406_0559_amd import inputs


def test_uniform_disc_is_uniform_in_area():
    rng = np.random.default_rng(0)
    x, y = inputs.uniform_disc(50000, 3.0, rng)
    r = np.hypot(x, y)
    assert r.max() <= 3.0
    # P(r < t) = (t/R)^2 for a uniform disc
    assert stats.kstest((r / 3.0) ** 2, "uniform").pvalue > 1e-3
    theta = np.arctan2(y, x)
    assert stats.kstest((theta + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3


def test_salpeter_masses_follow_the_power_law_and_have_unit_mean():
    """dN/dm ~ m^-2.35 on [0.1, 1], rescaled to mean 1. Dividing by the sample
    maximum (within O(1/n) of the upper bound 1) undoes the rescaling well
    enough for a KS test against the analytic CDF."""
    rng = np.random.default_rng(1)
    m = inputs.salpeter_masses(40000, rng)
    assert abs(m.mean() - 1.0) < 1e-12
    e = 1.0 - 2.35
    cdf = lambda v: (np.clip(v, 0.1, 1.0) ** e - 0.1 ** e) / (1.0 ** e - 0.1 ** e)
    raw = m / m.max()
    assert stats.kstest(raw, cdf).pvalue > 1e-4
    # the analytic mean on [0.1, 1] is ~0.2234, so unit-mean masses span ~[0.45, 4.5]
    assert 0.40 < m.min() < 0.50 and 4.0 < m.max() < 4.6


def test_workload_geometry_matches_the_stated_configs():
    c1 = inputs.config_small()
    assert (c1.n1, c1.n2, c1.n_lens, c1.p1) == (1024, 1024, 200, 256)
    assert abs(c1.disc_radius - 22.36) < 0.01
    c2 = inputs.config_gerlumph()
    assert c2.n_lens == 2624 and c2.evals == 30000 * 30000 * 2624
    c3 = inputs.config_mixed()
    assert c3.n_lens == 11560 and c3.masses == "salpeter"
    f = c3.lenses()
    assert f.m is not None and abs(f.m.mean() - 1.0) < 1e-12
    assert np.hypot(f.x1, f.x2).max() <= 170.0


def test_batch_workload():
    maps = inputs.config_batch()
    assert len(maps) == 64
    assert all(200 <= m.n_lens <= 20000 for m in maps)
    kept = inputs.macro_grid()
    assert len(kept) == 57   # 7 of the 64 (kappa, gamma) cells sit on |1-kappa| = gamma
    for m in maps:
        assert abs(abs(1 - m.kappa) - m.gamma) >= 0.05
        assert 3.0e7 < m.rays < 4.6e7
        assert m.p1 == 1024 and m.W1 == 25.0


def test_generators_are_seeded():
    a = inputs.lens_field(100, 5.0, "salpeter", 7)
    b = inputs.lens_field(100, 5.0, "salpeter", 7)
    assert (a.x1 == b.x1).all() and (a.m == b.m).all()
    r1 = inputs.serve_requests(20, rate=2.0, seed=3)
    r2 = inputs.serve_requests(20, rate=2.0, seed=3)
    assert [r.spec.n_lens for r in r1] == [r.spec.n_lens for r in r2]
    assert all(500 <= r.spec.n_lens <= 50000 for r in r1)
    assert all(r1[i].arrival < r1[i + 1].arrival for i in range(19))


def test_realisation_base_geometry():
    b = inputs.config_realisation_base()
    assert (b.kappa, b.gamma, b.s, b.p1, b.p2, b.W1) == (0.41, 0.38, 0.0, 1024, 1024, 25.0)
    mu_th = abs(1.0 / ((1.0 - b.kappa) ** 2 - b.gamma ** 2))
    n_avg = b.n1 * b.n2 / (4.0 * b.h1 * b.h2) * (b.W1 / b.p1) ** 2
    assert abs(n_avg * mu_th - 30.0) < 0.5           # ~30 lensed rays per pixel
    assert abs(b.disc_radius ** 2 * b.kappa_star - b.n_lens) < 1e-6 * b.n_lens

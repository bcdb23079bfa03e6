"""Seeded synthetic inputs for ray-shooting workloads.

This module only *generates inputs*: lens fields, ray grids, map windows and
request streams. It holds none of the method's arithmetic (no lens equation,
no binning, no normalisation), imports nothing else from this package and
nothing from the oracle, so both the HIP path and the oracle can be fed the
very same arrays.

Shapes follow the paper's workloads (Vernardos & Fluke 2014): ~1e9 rays per
map and N_* ~ 1e3-1e5 point lenses (Section 2.1), lenses spread uniformly in a
disc of area A with N_* = kappa_* A / (pi <M>) (eq. 3, Fig. 1), maps of
4096^2-10000^2 pixels spanning 24-25 Einstein radii (Table "datasets"). The
GERLUMPH maps and lens positions themselves are not used; these seeded fields
stand in for them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class LensField:
    """Point lenses on the lens plane; lengths in Einstein radii of <M>,
    masses in units of <M> (m is None for unit masses)."""
    x1: np.ndarray
    x2: np.ndarray
    m: Optional[np.ndarray]

    @property
    def n(self) -> int:
        return int(self.x1.size)


@dataclasses.dataclass
class MapSpec:
    """One magnification-map job: macro model (kappa, gamma, s), ray grid and
    source-plane window. Rays sit at the centres of an n1 x n2 grid of cells
    covering [c1-h1, c1+h1) x [c2-h2, c2+h2)."""
    name: str
    kappa: float
    gamma: float
    s: float
    n1: int
    n2: int
    h1: float
    h2: float
    p1: int
    p2: int
    W1: float
    W2: float
    c1: float = 0.0
    c2: float = 0.0
    w1: float = 0.0
    w2: float = 0.0
    n_lens: int = 0
    disc_radius: float = 0.0
    masses: str = "unit"          # "unit" or "salpeter"
    seed: int = 0

    @property
    def kappa_star(self) -> float:
        return (1.0 - self.s) * self.kappa

    @property
    def rays(self) -> int:
        return self.n1 * self.n2

    @property
    def evals(self) -> int:
        return self.n1 * self.n2 * self.n_lens

    def lenses(self) -> LensField:
        return lens_field(self.n_lens, self.disc_radius, self.masses, self.seed)


def uniform_disc(n: int, radius: float, rng: np.random.Generator):
    """n points uniform in a disc of the given radius centred at the origin."""
    r = radius * np.sqrt(rng.random(n))
    t = 2.0 * np.pi * rng.random(n)
    return r * np.cos(t), r * np.sin(t)


def salpeter_masses(n: int, rng: np.random.Generator, lo: float = 0.1, hi: float = 1.0,
                    slope: float = 2.35) -> np.ndarray:
    """Masses with dN/dm proportional to m^-slope on [lo, hi], drawn by inverse CDF
    and rescaled so that the sample mean is exactly 1 (masses in units of <M>)."""
    if n == 0:
        return np.zeros(0)
    e = 1.0 - slope
    u = rng.random(n)
    m = (lo ** e + u * (hi ** e - lo ** e)) ** (1.0 / e)
    return m / m.mean()


def lens_field(n: int, radius: float, masses: str = "unit", seed: int = 0) -> LensField:
    rng = np.random.default_rng(seed)
    x1, x2 = uniform_disc(n, radius, rng)
    if masses == "unit":
        m = None
    elif masses == "salpeter":
        m = salpeter_masses(n, rng)
    else:
        raise ValueError(f"unknown mass model {masses!r}")
    return LensField(np.ascontiguousarray(x1), np.ascontiguousarray(x2), m)


def lenses_for_disc(kappa_star: float, radius: float) -> int:
    """N_* = kappa_* A / (pi <M>) with A = pi R^2 and <M> = 1 (eq. 3)."""
    return int(round(kappa_star * radius * radius))


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------

def config_small() -> MapSpec:
    """Small all-compact field: kappa_*=0.4, gamma=0.3, 200 unit lenses in a disc
    of radius sqrt(200/0.4); 1024^2 rays over half-widths 8.0 x 2.67; 256^2 map
    over 4 x 4 Einstein radii."""
    return MapSpec(name="small-fp64", kappa=0.4, gamma=0.3, s=0.0,
                   n1=1024, n2=1024, h1=8.0, h2=2.67, p1=256, p2=256, W1=4.0, W2=4.0,
                   n_lens=200, disc_radius=math.sqrt(200 / 0.4), masses="unit", seed=1)


def config_gerlumph() -> MapSpec:
    """GERLUMPH-like map: kappa=0.41 all compact, gamma=0.38, 2624 unit lenses in
    a disc of radius 80; 30000^2 rays over half-widths 65 x 14.2; 4096^2 map over
    25 x 25 Einstein radii (~45 rays per pixel)."""
    return MapSpec(name="gerlumph-30000sq-2624", kappa=0.41, gamma=0.38, s=0.0,
                   n1=30000, n2=30000, h1=65.0, h2=14.2, p1=4096, p2=4096, W1=25.0, W2=25.0,
                   n_lens=2624, disc_radius=80.0, masses="unit", seed=2)


def config_mixed() -> MapSpec:
    """Mixed masses plus smooth matter near the critical line: kappa=0.8, s=0.5,
    gamma=0.3; kappa_* R^2 = 11560 lenses with a Salpeter-like spectrum on
    [0.1, 1] rescaled to mean 1, disc radius 170; 20000^2 rays over half-widths
    137 x 27.5; 4096^2 map over 25 x 25."""
    return MapSpec(name="mixed-20000sq-11560", kappa=0.8, gamma=0.3, s=0.5,
                   n1=20000, n2=20000, h1=137.0, h2=27.5, p1=4096, p2=4096, W1=25.0, W2=25.0,
                   n_lens=lenses_for_disc(0.4, 170.0), disc_radius=170.0, masses="salpeter",
                   seed=3)


def scaled(spec: MapSpec, ray_factor: float = 1.0, pixel_factor: float = 1.0,
           lens_factor: float = 1.0, name: Optional[str] = None) -> MapSpec:
    """The same geometry with fewer rays / pixels / lenses (for quick checks).
    The lens disc keeps its radius; its density scales with lens_factor."""
    n1 = max(1, int(round(spec.n1 * ray_factor)))
    n2 = max(1, int(round(spec.n2 * ray_factor)))
    p1 = max(1, int(round(spec.p1 * pixel_factor)))
    p2 = max(1, int(round(spec.p2 * pixel_factor)))
    nl = int(round(spec.n_lens * lens_factor))
    return dataclasses.replace(spec, n1=n1, n2=n2, p1=p1, p2=p2, n_lens=nl,
                               name=name or f"{spec.name}-scaled")


def macro_grid(n: int = 8, kappa_range=(0.1, 1.2), gamma_range=(0.0, 1.0), skip: float = 0.05):
    """The (kappa, gamma) grid of the batched workload, without the cells that
    sit on the critical line | |1-kappa| - gamma | < skip."""
    ks = np.linspace(kappa_range[0], kappa_range[1], n)
    gs = np.linspace(gamma_range[0], gamma_range[1], n)
    kept = []
    for k in ks:
        for g in gs:
            if abs(abs(1.0 - k) - g) < skip:
                continue
            kept.append((float(k), float(g)))
    return kept


def _survey_geometry(kappa: float, gamma: float, s: float, pixels: int, width: float,
                     mean_count: float, margin: float, corner_margin: float,
                     n_min: int, n_max: int, seed: int, name: str,
                     n_lens: Optional[int] = None) -> MapSpec:
    """Ray region, ray count and lens disc for a survey map.

    The ray rectangle is the window mapped back through the mean macro model
    (convergence kappa, shear gamma), grown by `margin`; the ray count gives a
    lensed mean of `mean_count` rays per pixel; the lens disc covers the ray
    rectangle's corner grown by `corner_margin`, with N clamped to [n_min, n_max].
    """
    a1 = abs(1.0 - kappa - gamma)
    a2 = abs(1.0 - kappa + gamma)
    h1 = margin * 0.5 * width / a1
    h2 = margin * 0.5 * width / a2
    mu_th = abs(1.0 / ((1.0 - kappa) ** 2 - gamma ** 2))
    unlensed_per_pixel = mean_count / mu_th
    pix_area = (width / pixels) ** 2
    rays_total = unlensed_per_pixel * 4.0 * h1 * h2 / pix_area
    # isotropic ray spacing: n1 / n2 = h1 / h2
    n2 = max(1, int(round(math.sqrt(rays_total * h2 / h1))))
    n1 = max(1, int(round(rays_total / n2)))
    kstar = (1.0 - s) * kappa
    if n_lens is None:
        corner = corner_margin * math.hypot(h1, h2)
        n_lens = int(min(max(round(kstar * corner * corner), n_min), n_max))
    radius = math.sqrt(n_lens / kstar) if kstar > 0 else 0.0
    return MapSpec(name=name, kappa=kappa, gamma=gamma, s=s, n1=n1, n2=n2, h1=h1, h2=h2,
                   p1=pixels, p2=pixels, W1=width, W2=width, n_lens=n_lens,
                   disc_radius=radius, masses="unit", seed=seed)


def config_batch(n_maps: int = 64, pixels: int = 1024, seed0: int = 4) -> List[MapSpec]:
    """Batched workload: maps with (kappa, gamma) on an 8 x 8 grid in
    [0.1, 1.2] x [0, 1] without the critical-line cells, s cycling through
    {0, 0.5, 0.9}, unit-mass uniform disc fields of 200-20000 lenses, 1024^2
    maps over 25 Einstein radii, ray grids sized for ~30 rays per pixel."""
    cells = macro_grid()
    s_values = (0.0, 0.5, 0.9)
    out = []
    for i in range(n_maps):
        k, g = cells[i % len(cells)]
        s = s_values[i % len(s_values)]
        out.append(_survey_geometry(k, g, s, pixels, 25.0, 30.0, 1.1, 1.2, 200, 20000,
                                    seed0 + i, f"batch-{i:02d}"))
    return out


def config_realisation_base(pixels: int = 1024) -> MapSpec:
    """Base map of the realisation batches (Section 4's meanMPD tool: maps that
    differ only in the random lens positions): the GERLUMPH-like macro model
    (kappa = 0.41, gamma = 0.38, s = 0) on a 1024^2 map over 25 Einstein radii,
    ~30 lensed rays per pixel, unit masses; realisations vary the seed."""
    return _survey_geometry(0.41, 0.38, 0.0, pixels, 25.0, 30.0, 1.1, 1.2, 200, 20000, 6,
                            "realisation-base")


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float      # seconds after the start of the stream
    spec: MapSpec


def serve_requests(n: int = 1000, rate: float = 1.0, seed: int = 5,
                   sizes=(1024, 2048, 4096), n_lens_range=(500, 50000),
                   size_scale: float = 1.0) -> List[Request]:
    """Poisson stream of map requests: (kappa, gamma, s) uniform over the batched
    workload's grid, map sizes uniform over `sizes`, lens counts uniform in
    `n_lens_range`, ~30 lensed rays per pixel. `size_scale` shrinks every map
    (pixels and rays) for quick runs."""
    rng = np.random.default_rng(seed)
    cells = macro_grid()
    s_values = (0.0, 0.5, 0.9)
    t = 0.0
    out = []
    for rid in range(n):
        t += float(rng.exponential(1.0 / rate))
        k, g = cells[int(rng.integers(len(cells)))]
        s = s_values[int(rng.integers(len(s_values)))]
        p = int(sizes[int(rng.integers(len(sizes)))])
        p = max(16, int(round(p * size_scale)))
        nl = int(rng.integers(n_lens_range[0], n_lens_range[1] + 1))
        spec = _survey_geometry(k, g, s, p, 25.0, 30.0, 1.1, 1.2, nl, nl, seed + 1000 + rid,
                                f"req-{rid:04d}", n_lens=nl)
        out.append(Request(rid, t, spec))
    return out


WORKLOADS = {
    "small-fp64": config_small,
    "gerlumph-30000sq-2624": config_gerlumph,
    "mixed-20000sq-11560": config_mixed,
}

"""Pins of the oracle's magnification probability distributions (MPDs).

Section 3.2.1 defines a map's MPD as the frequency of each magnification value
divided by the number of pixels; Section 4's tools bin it (100 bins by
default, up to 400) against the macro-magnification mu_th and form
probability sums P(mu < mu_lim) and P(mu > mu_lim), which add up to one.
The checks below compare the oracle with closed forms (uniform sheet, point
lens), the mass-sheet transformation, and an independent evaluation that
takes log10 of each pixel's magnification directly.
"""
import math

import numpy as np
import pytest

import oracle


def uniform_sheet_map(kappa_s, gamma, n1, n2, p1, p2, W1, W2):
    a1 = 1.0 - kappa_s - gamma
    a2 = 1.0 - kappa_s + gamma
    h1 = 1.2 * 0.5 * W1 / abs(a1)
    h2 = 1.2 * 0.5 * W2 / abs(a2)
    counts, esc = oracle.shoot(np.zeros(0), np.zeros(0), None, kappa_s, gamma, 1.0, n1, n2, 0.0,
                               0.0, h1, h2, p1, p2, 0.0, 0.0, W1, W2)
    return counts, (a1, a2, h1, h2)


def per_axis_pixel_counts(a, h, n, p, W):
    """Rays of one axis per pixel for the linear map y = a x: pixel k holds the
    x in [lo_k, hi_k) / a (half-open after mapping), counted on the grid."""
    x = -h + (np.arange(n) + 0.5) * (2.0 * h / n)
    y = a * x
    edges = -0.5 * W + np.arange(p + 1) * (W / p)
    return np.array([np.count_nonzero((y >= edges[k]) & (y < edges[k + 1])) for k in range(p)])


def test_totals_add_to_one():
    rng = np.random.default_rng(3)
    counts = rng.poisson(20.0, size=(64, 48)).astype(np.int32)
    counts[0, 0] = 0
    counts[1, 1] = 5000
    h = oracle.count_histogram(counts, int(counts.max()) + 1)
    assert h.sum() == counts.size
    assert (h == np.bincount(counts.ravel(), minlength=h.size)).all()
    bins = oracle.mpd(counts, 20.0, 1.0, -1.0, 1.0, 100)
    assert bins.sum() == counts.size and bins.size == 102
    lo, hi = oracle.probability_sums(counts, 20.0, 1.25)
    assert lo + hi == counts.size
    clipped = oracle.count_histogram(counts, 30)
    assert clipped[-1] == np.count_nonzero(counts >= 29) and clipped.sum() == counts.size


@pytest.mark.parametrize("kappa_s,gamma", [(0.4, 0.2), (0.3, 0.9)])
def test_uniform_sheet_histogram_is_the_product_of_axis_counts(kappa_s, gamma):
    """No point lenses: every pixel's count is n1(ix) * n2(iy), so the
    frequency of each count value is fixed by the per-axis counts alone."""
    p1, p2, W1, W2, n1, n2 = 40, 30, 3.0, 2.0, 1100, 900
    counts, (a1, a2, h1, h2) = uniform_sheet_map(kappa_s, gamma, n1, n2, p1, p2, W1, W2)
    c1 = per_axis_pixel_counts(a1, h1, n1, p1, W1)
    c2 = per_axis_pixel_counts(a2, h2, n2, p2, W2)
    expect = np.bincount(np.outer(c2, c1).ravel(), minlength=int(counts.max()) + 1)
    got = oracle.count_histogram(counts, int(counts.max()) + 1)
    assert (got == expect).all()
    assert np.count_nonzero(got) <= 4      # each axis count is one of two neighbours


def test_identity_map_mpd_is_a_single_bin():
    """kappa = gamma = 0, no lenses: mu = 1 in every pixel, so the whole MPD sits
    in the bin that contains log10(mu / mu_th) = 0."""
    n, h, p, W = 1024, 2.0, 256, 4.0
    counts, _ = oracle.shoot(np.zeros(0), np.zeros(0), None, 0.0, 0.0, 0.0, n, n, 0.0, 0.0, h, h,
                             p, p, 0.0, 0.0, W, W)
    navg = oracle.n_avg(n, n, h, h, p, p, W, W)
    bins = oracle.mpd(counts, navg, 1.0, -0.95, 1.05, 100)    # edges at -0.95 + 0.02 k
    assert bins[1 + 47] == p * p and bins.sum() == p * p      # log 1 = 0 lies in [-0.01, 0.01)
    lo, hi = oracle.probability_sums(counts, navg, 1.25)
    assert (lo, hi) == (p * p, 0)
    lo, hi = oracle.probability_sums(counts, navg, 1.0)         # mu < 1 is false everywhere
    assert (lo, hi) == (0, p * p)


def test_point_lens_high_magnification_fraction():
    """One unit lens centred on the window: P(mu > mu0) is the fraction of the
    window where the point-lens mu(u) = (u^2+2)/(u sqrt(u^2+4)) exceeds mu0,
    i.e. pi u0^2 / W^2 with mu(u0) = mu0 (up to pixel averaging and lattice
    noise)."""
    n, h, p, W = 3000, 2.6, 128, 4.0
    counts, _ = oracle.shoot(np.array([0.0]), np.array([0.0]), None, 0.0, 0.0, 0.0, n, n, 0.0, 0.0,
                             h, h, p, p, 0.0, 0.0, W, W)
    navg = oracle.n_avg(n, n, h, h, p, p, W, W)
    for mu0 in (1.5, 3.0):
        # mu(u) = mu0  <=>  u^2 = 2 (mu0 / sqrt(mu0^2 - 1) - 1)
        u0 = math.sqrt(2.0 * (mu0 / math.sqrt(mu0 * mu0 - 1.0) - 1.0))
        lo, hi = oracle.probability_sums(counts, navg, mu0)
        frac = hi / counts.size
        expect = math.pi * u0 * u0 / (W * W)
        assert abs(frac - expect) / expect < 0.03, (mu0, frac, expect)


def test_mass_sheet_equivalent_maps_have_the_same_mpd():
    """Maps related by the mass-sheet rescaling (the 'equivalent maps' of
    Section 2.2) have the same MPD in mu / mu_th: with a = 1 - kappa_s,
    mu = mu' / a^2 and mu_th = mu_th' / a^2."""
    rng = np.random.default_rng(9)
    n_l = 40
    r = 5.0 * np.sqrt(rng.random(n_l))
    t = 2 * np.pi * rng.random(n_l)
    x1, x2 = r * np.cos(t), r * np.sin(t)
    kappa, s, gamma = 0.7, 0.5, 0.25
    ks = s * kappa
    kst = kappa - ks
    a = 1.0 - ks
    sa = math.sqrt(a)
    N1, N2, h1, h2, p, W = 900, 700, 3.0, 2.2, 48, 2.0
    c, _ = oracle.shoot(x1, x2, None, kappa, gamma, s, N1, N2, 0.0, 0.0, h1, h2, p, p, 0.0, 0.0, W, W)
    cp, _ = oracle.shoot(sa * x1, sa * x2, None, kst / a, gamma / a, 0.0, N1, N2, 0.0, 0.0, sa * h1,
                         sa * h2, p, p, 0.0, 0.0, W / sa, W / sa)
    mu_th = 1.0 / ((1.0 - kappa) ** 2 - gamma ** 2)
    mu_thp = 1.0 / ((1.0 - kst / a) ** 2 - (gamma / a) ** 2)
    assert abs(mu_thp / mu_th - a * a) < 1e-12
    na = oracle.n_avg(N1, N2, h1, h2, p, p, W, W)
    nap = oracle.n_avg(N1, N2, sa * h1, sa * h2, p, p, W / sa, W / sa)
    b = oracle.mpd(c, na, abs(mu_th), -1.0, 1.0, 40)
    bp = oracle.mpd(cp, nap, abs(mu_thp), -1.0, 1.0, 40)
    assert np.abs(b - bp).sum() <= 2 * np.abs(c.astype(np.int64) - cp).sum() + 2


def test_mpd_against_direct_log10_binning():
    """An independent evaluation: log10(N / (N_avg mu_ref)) per pixel, binned with
    numpy; pixels within 1e-9 of an edge (none here) would be ambiguous."""
    rng = np.random.default_rng(4)
    counts = rng.integers(0, 400, size=(90, 70)).astype(np.int32)
    navg, mu_ref, lo, hi, nb = 11.37, 2.71, -1.3, 1.45, 137
    bins = oracle.mpd(counts, navg, mu_ref, lo, hi, nb)
    c = counts.ravel().astype(np.float64)
    with np.errstate(divide="ignore"):
        x = np.log10(c / (navg * mu_ref))
    edges = lo + np.arange(nb + 1) * ((hi - lo) / nb)
    finite = np.isfinite(x)
    assert np.min(np.abs(x[finite][:, None] - edges[None, :])) > 1e-9
    idx = np.where(finite, np.searchsorted(edges, x, side="right"), 0)
    expect = np.bincount(idx, minlength=nb + 2)
    assert (bins == expect).all()


def test_invalid_arguments():
    c = np.zeros((2, 2), np.int32)
    with pytest.raises(ValueError):
        oracle.mpd(c, 0.0, 1.0, -1, 1, 10)
    with pytest.raises(ValueError):
        oracle.mpd(c, 1.0, 1.0, 1, -1, 10)
    with pytest.raises(ValueError):
        oracle.count_histogram(np.array([-1], np.int32), 4)
    with pytest.raises(ValueError):
        oracle.probability_sums(c, -2.0, 1.0)


def test_bin_edges_are_half_open():
    """Thresholds that are exact integers (N_avg mu_ref 10^0 = 10 and 10^1 = 100):
    a pixel on a lower edge belongs to that bin, one on the top edge overflows."""
    counts = np.array([[9, 10, 99, 100, 0, 55]], np.int32)
    thr = oracle.mpd_thresholds(10.0, 1.0, 0.0, 1.0, 1)
    assert thr[0] == 10.0 and thr[1] == 100.0
    bins = oracle.mpd(counts, 10.0, 1.0, 0.0, 1.0, 1)
    assert bins.tolist() == [2, 3, 1]


# ---------------------------------------------------------------------------
# MPDs of maps of real magnifications (finite-source maps)
# ---------------------------------------------------------------------------

def test_mpd_values_against_searchsorted():
    """The bin of a value is the number of thresholds at or below it: the
    insertion point of the value to the right of equal thresholds, which
    numpy's searchsorted gives independently of the oracle's scan."""
    rng = np.random.default_rng(41)
    mu = 10.0 ** rng.uniform(-2.5, 2.5, size=20000)
    thr = oracle.mpd_thresholds(1.0, 3.7, -1.5, 1.5, 100)
    mu[:101] = thr                                        # exactly on every edge
    mu[101:202] = np.nextafter(thr, -np.inf)              # just below every edge
    got = oracle.mpd_values(mu, 3.7, -1.5, 1.5, 100)
    expect = np.bincount(np.searchsorted(thr, mu, side="right"), minlength=102)
    assert (got == expect).all()
    assert got.sum() == mu.size


def test_mpd_values_thresholds_are_mu_ref_times_powers_of_ten():
    """With n_avg = 1 the edges are mu_ref 10^(lo + k (hi - lo) / nbins); the
    bin of log10(mu / mu_ref) = lo + (k + 1/2) (hi - lo) / nbins is k."""
    mu_ref, lo, hi, nb = 4.91, -1.5, 1.5, 100
    thr = oracle.mpd_thresholds(1.0, mu_ref, lo, hi, nb)
    k = np.arange(nb)
    np.testing.assert_allclose(thr, mu_ref * 10.0 ** (lo + np.arange(nb + 1) * (hi - lo) / nb), rtol=1e-14)
    mids = mu_ref * 10.0 ** (lo + (k + 0.5) * (hi - lo) / nb)
    got = oracle.mpd_values(mids, mu_ref, lo, hi, nb)
    assert (got[1:-1] == 1).all() and got[0] == 0 and got[-1] == 0


def test_mpd_values_special_values():
    """NaN and -inf are below every edge (underflow), +inf above (overflow);
    zeros and negative values underflow; a constant map fills one bin."""
    mu = np.array([np.nan, -np.inf, -1.0, 0.0, np.inf, 1e300])
    got = oracle.mpd_values(mu, 1.0, -1.0, 1.0, 10)
    assert got[0] == 4 and got[-1] == 2 and got.sum() == 6
    c = np.full((30, 40), 2.0)
    got = oracle.mpd_values(c, 1.0, -1.0, 1.0, 10)      # log10 2 = 0.301 lies in [0.2, 0.4)
    assert got[1 + 6] == 1200 and got.sum() == 1200

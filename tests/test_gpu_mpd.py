"""MPDs on the GPU against the oracle: the count histogram, the binned MPD and
the probability sums bit for bit (every bin decision is an FP64 comparison of
an integer count with a threshold computed the same way on both sides), and
the realisation mean and spread against numpy."""
import numpy as np
import pytest

import oracle
from paper_1406_0559_amd import inputs
from paper_1406_0559_amd import raylens as rl
from paper_1406_0559_amd import realisations

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = rl.Context(0)
    yield c
    c.close()


def spec_of(p1, p2, n1=1000, n2=1000, h=2.0, W=4.0):
    return inputs.MapSpec(name="mpd", kappa=0.5, gamma=0.2, s=0.0, n1=n1, n2=n2, h1=h, h2=h,
                          p1=p1, p2=p2, W1=W, W2=W)


def check_all(ctx, counts_np, spec, n_avg, mu_ref):
    counts = torch.from_numpy(np.ascontiguousarray(counts_np, np.int32)).cuda()
    nv = int(counts_np.max()) + 1
    for n_values in (nv, max(2, nv // 3), 1):
        h = ctx.count_histogram(counts, spec, n_values).cpu().numpy()
        assert (h == oracle.count_histogram(counts_np, n_values)).all()
    # 255 bins (256 thresholds) is the longest list that travels with the
    # launch, 256 bins the shortest one read from device memory
    for lo, hi, nb in ((-1.0, 1.0, 100), (-1.5, 1.5, 400), (0.0, 1.0, 1), (-3.0, 2.0, 4096),
                       (-1.0, 1.0, 255), (-1.0, 1.0, 256)):
        b = ctx.mpd(counts, spec, mu_ref, lo, hi, nb, n_avg=n_avg).cpu().numpy()
        assert (b == oracle.mpd(counts_np, n_avg, mu_ref, lo, hi, nb)).all(), (lo, hi, nb)
    edge = 100.0 / n_avg          # the quotient of a count present in the maps
    for mu_lim in (0.3 * mu_ref, 1.25 * mu_ref, 3.0 * mu_ref, 1.0, 0.0, -1.0, np.inf, -np.inf,
                   edge, np.nextafter(edge, np.inf), np.nextafter(edge, -np.inf)):
        got = ctx.probability_sums(counts, spec, mu_lim, n_avg=n_avg)
        assert got == oracle.probability_sums(counts_np, n_avg, mu_lim), mu_lim


def test_probability_sums_extreme_counts(ctx):
    """Negative counts (an overflowed pixel) and the int32 limits: the count
    threshold taken on the host covers the whole int32 range."""
    spec = spec_of(67, 3)
    rng = np.random.default_rng(13)
    c = rng.integers(0, 300, size=(3, 67)).astype(np.int32)
    c[0, :6] = [np.iinfo(np.int32).min, -5, -1, np.iinfo(np.int32).max, 2**30, 0]
    counts = torch.from_numpy(c).cuda()
    for n_avg in (10.0, 7.3, 1e-300, 1e300):
        for mu_lim in (-1e9, -0.5, 0.0, 1.0, 29.9, 1e8, 3e8, np.inf, -np.inf, 5e-324):
            got = ctx.probability_sums(counts, spec, mu_lim, n_avg=n_avg)
            assert got == oracle.probability_sums(c, n_avg, mu_lim), (n_avg, mu_lim)


def test_random_and_adversarial_counts(ctx):
    rng = np.random.default_rng(12)
    spec = spec_of(301, 257)
    c = rng.poisson(25.0, size=(257, 301)).astype(np.int32)
    c[0, :6] = [0, 10, 100, 1000, 9999, 123456]     # values on integer thresholds, large tail
    c[5, 5] = 20000
    check_all(ctx, c, spec, 10.0, 1.0)               # thresholds 10^k are exact integers here
    check_all(ctx, c, spec, 7.3, 2.9)


def test_shot_map_mpd_matches_the_oracle(ctx):
    spec = inputs.config_small()
    f = spec.lenses()
    L = rl.DeviceLenses(f.x1, f.x2, f.m)
    counts, esc = ctx.shoot(L, spec, "fp32c")
    navg = rl.rl_n_avg(rl.grid_of(spec), rl.window_of(spec))
    mu_th = abs(1.0 / ((1.0 - spec.kappa) ** 2 - spec.gamma ** 2))
    check_all(ctx, counts.cpu().numpy(), spec, navg, mu_th)


def test_full_size_map_mpd(ctx):
    """The 4096^2 map of the GERLUMPH-like workload: histogram and 100-bin MPD."""
    spec = inputs.config_gerlumph()
    f = spec.lenses()
    L = rl.DeviceLenses(f.x1, f.x2, f.m)
    counts, esc = ctx.shoot(L, spec, "fp32c")
    cn = counts.cpu().numpy()
    navg = rl.rl_n_avg(rl.grid_of(spec), rl.window_of(spec))
    mu_th = abs(1.0 / ((1.0 - spec.kappa) ** 2 - spec.gamma ** 2))
    h = ctx.count_histogram(counts, spec, int(cn.max()) + 1).cpu().numpy()
    assert (h == np.bincount(cn.ravel(), minlength=h.size)).all()
    b = ctx.mpd(counts, spec, mu_th, -1.5, 1.5, 100, n_avg=navg).cpu().numpy()
    assert (b == oracle.mpd(cn, navg, mu_th, -1.5, 1.5, 100)).all()
    assert b.sum() == spec.p1 * spec.p2
    lo, hi = ctx.probability_sums(counts, spec, 1.25 * mu_th, n_avg=navg)
    assert (lo, hi) == oracle.probability_sums(cn, navg, 1.25 * mu_th)


def test_realisations_mean_and_spread(ctx):
    base = inputs.scaled(inputs.config_small(), ray_factor=0.5, pixel_factor=0.5, name="real")
    out = realisations.mean_mpd(ctx, base, n=5, nbins=60, log_lo=-1.0, log_hi=1.0)
    bins = out["bins"].cpu().numpy()
    navg = rl.rl_n_avg(rl.grid_of(base), rl.window_of(base))
    for r, (c, s) in enumerate(zip(out["counts"], out["specs"])):
        assert (bins[r] == oracle.mpd(c.cpu().numpy(), navg, out["mu_th"], -1.0, 1.0, 60)).all()
        # each realisation equals the same map shot alone
        f = out["fields"][r]
        alone, _ = ctx.shoot(rl.DeviceLenses(f.x1, f.x2, f.m), s, "fp32c")
        assert torch.equal(alone, c)
    p = bins / float(base.p1 * base.p2)
    assert np.allclose(out["mean"].cpu().numpy(), p.mean(axis=0), rtol=1e-12, atol=1e-15)
    assert np.allclose(out["std"].cpu().numpy(), p.std(axis=0, ddof=1), rtol=1e-10, atol=1e-14)
    assert len({s.seed for s in out["specs"]}) == 5


@pytest.mark.parametrize("p1,p2", [(517, 131), (4096, 64)])
def test_mpd_of_real_maps_matches_the_oracle(ctx, p1, p2):
    """rl_mpd_values against the oracle, bit for bit: magnifications over five
    decades with values exactly on every bin edge and one ulp below, zeros,
    negatives, +-inf and NaN; edges from the launch argument (up to 255 bins)
    and from device memory (256 and 4096 bins); an unaligned map start."""
    rng = np.random.default_rng(p1 + p2)
    spec = spec_of(p1, p2)
    n = p1 * p2
    mu_ref = 4.91
    mu = 10.0 ** rng.uniform(-2.5, 2.5, size=n)
    thr = oracle.mpd_thresholds(1.0, mu_ref, -1.5, 1.5, 100)
    mu[:101] = thr
    mu[101:202] = np.nextafter(thr, -np.inf)
    mu[202:208] = [0.0, -1.0, np.inf, -np.inf, np.nan, 1e308]
    rng.shuffle(mu)
    flat = torch.empty(n + 1, dtype=torch.float64, device="cuda")
    flat[1:] = torch.from_numpy(mu).cuda()
    for dev_mu in (torch.from_numpy(mu).cuda(), flat[1:]):         # aligned, and 8 bytes off
        for lo, hi, nb in ((-1.5, 1.5, 100), (-1.0, 1.0, 255), (-1.0, 1.0, 256), (-3.0, 2.0, 4096),
                           (0.0, 1.0, 1)):
            got = ctx.mpd_values(dev_mu, spec, mu_ref, lo, hi, nb).cpu().numpy()
            assert (got == oracle.mpd_values(mu, mu_ref, lo, hi, nb)).all(), (lo, hi, nb)


def test_mpd_of_a_finite_source_map(ctx):
    """The MPD of a convolved map (the product stored for every convolution):
    a count map convolved with a Gaussian source, as magnification, binned on
    the GPU and by the oracle from the same values."""
    spec = spec_of(1024, 512)
    rng = np.random.default_rng(8)
    M = torch.from_numpy(rng.poisson(30.0, size=(512, 1024)).astype(np.int32)).cuda()
    k = ctx.source_kernel(spec, "gaussian", 0.1)
    mu = ctx.convolve(M, k, spec, n_avg=30.0)
    got = ctx.mpd_values(mu, spec, 1.0, -1.0, 1.0, 100).cpu().numpy()
    assert (got == oracle.mpd_values(mu.cpu().numpy(), 1.0, -1.0, 1.0, 100)).all()
    assert got.sum() == 1024 * 512 and got[0] == 0 and got[-1] == 0

"""Finite-source maps on the GPU against the oracle (Section 2.4, eq. 6):
source kernels to 1e-13 relative, FFT convolutions to 1e-12 of the map's
largest value (both FP64; the FFTs differ only in rounding order)."""
import numpy as np
import pytest

from oracle import convolve as ocv
from paper_1406_0559_amd import inputs
from paper_1406_0559_amd import raylens as rl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = rl.Context(0)
    yield c
    c.close()


def spec_of(p1, p2, W1=4.0, W2=4.0):
    return inputs.MapSpec(name="conv", kappa=0.5, gamma=0.2, s=0.0, n1=10, n2=10, h1=1.0, h2=1.0,
                          p1=p1, p2=p2, W1=W1, W2=W2)


@pytest.mark.parametrize("shape,radius,hole", [("uniform", 0.237, 0.0), ("gaussian", 0.311, 0.0),
                                               ("power", 0.419, 0.05), ("uniform", 0.013, 0.0)])
def test_source_kernel_matches_the_oracle(ctx, shape, radius, hole):
    spec = spec_of(128, 64, 4.0, 3.0)
    k = ctx.source_kernel(spec, shape, radius, hole).cpu().numpy()
    ref = ocv.source_kernel(shape, spec.p1, spec.p2, spec.W1 / spec.p1, spec.W2 / spec.p2, radius, hole)
    assert np.abs(k - ref).max() <= 1e-13 * ref.max()
    assert abs(k.sum() - 1.0) < 1e-12


def subsample_table(shape, radius, hole, pix1, pix2, n1, n2, s=8):
    """The profile tabulated at the 8 x 8 sub-sample points of pixels -n .. n
    on each axis (ascending, as profile files store them), FP32."""
    off = (np.arange(s) + 0.5) / s - 0.5
    x = ((np.arange(-n1, n1 + 1)[:, None] + off[None, :]).ravel() * pix1).astype(np.float32)
    y = ((np.arange(-n2, n2 + 1)[:, None] + off[None, :]).ravel() * pix2).astype(np.float32)
    X, Y = np.meshgrid(x.astype(np.float64), y.astype(np.float64))
    return x, y, ocv.brightness(shape, np.hypot(X, Y), radius, hole).astype(np.float32)


@pytest.mark.parametrize("shape,radius,hole", [("uniform", 0.237, 0.0), ("gaussian", 0.311, 0.0),
                                               ("power", 0.419, 0.05)])
def test_table_kernel_matches_the_oracle_and_the_analytic_kernel(ctx, shape, radius, hole):
    """A profile tabulated at the analytic kernel's sub-sample points: the
    GPU table kernel equals the oracle's to rounding of the normalisation and
    the analytic kernel to FP32 precision of the table."""
    spec = spec_of(128, 64, 4.0, 3.0)
    pix1, pix2 = spec.W1 / spec.p1, spec.W2 / spec.p2
    n1, n2 = int(np.ceil(radius / pix1)), int(np.ceil(radius / pix2))
    x, y, b = subsample_table(shape, radius, hole, pix1, pix2, n1, n2)
    k = ctx.source_kernel_table(spec, x, y, b).cpu().numpy()
    ref = ocv.table_kernel(x, y, b, spec.p1, spec.p2, pix1, pix2)
    assert np.abs(k - ref).max() <= 1e-13 * ref.max()
    assert abs(k.sum() - 1.0) < 1e-12
    ana = ctx.source_kernel(spec, shape, radius, hole).cpu().numpy()
    assert np.abs(k - ana).max() <= 1e-6 * ana.max()


@pytest.mark.parametrize("seed,nx,ny,p1,p2", [(1, 37, 53, 64, 48), (2, 1, 1, 16, 16), (3, 300, 7, 256, 30),
                                              (4, 1000, 1000, 1024, 1024)])
def test_table_kernel_of_unordered_tables(ctx, seed, nx, ny, p1, p2):
    """Positions in random order, some exactly on pixel edges (pix = 1/32 and
    1/64, so the edges are FP32 numbers), repeated positions and zero
    brightness: the same pixels as the oracle (bit-exact zero pattern) and its
    per-pixel sums to rounding."""
    rng = np.random.default_rng(seed)
    spec = spec_of(p1, p2, p1 / 32.0, p2 / 64.0)
    pix1, pix2 = spec.W1 / spec.p1, spec.W2 / spec.p2
    hx, hy = min(p1 // 2 - 1, 9), min(p2 // 2 - 1, 9)
    x = rng.uniform(-hx * pix1, hx * pix1, nx)
    y = rng.uniform(-hy * pix2, hy * pix2, ny)
    x[: nx // 4] = (rng.integers(-hx, hx, nx // 4) + 0.5) * pix1      # on box edges
    y[: ny // 4] = (rng.integers(-hy, hy, ny // 4) + 0.5) * pix2
    if nx > 3:
        x[-1] = x[-2]
    b = rng.exponential(1.0, (ny, nx))
    b[rng.random((ny, nx)) < 0.2] = 0.0
    b.flat[0] = 1.0
    x, y, b = x.astype(np.float32), y.astype(np.float32), b.astype(np.float32)
    k = ctx.source_kernel_table(spec, x, y, b).cpu().numpy()
    ref = ocv.table_kernel(x, y, b, p1, p2, pix1, pix2)
    assert np.array_equal(k != 0, ref != 0)
    assert np.abs(k - ref).max() <= 1e-13 * ref.max()
    assert abs(k.sum() - 1.0) < 1e-12


def test_table_kernel_of_a_paper_sized_grid(ctx):
    """A regular grid of the size the disc profiles are stored on (1000 to
    3000 points per axis), ascending: hundreds of samples per pixel, summed in
    a different order than the oracle's, equal to rounding."""
    spec = spec_of(512, 512, 8.0, 8.0)
    x = np.linspace(-0.31, 0.31, 1500).astype(np.float32)
    y = np.linspace(-0.27, 0.27, 1200).astype(np.float32)
    X, Y = np.meshgrid(x.astype(np.float64), y.astype(np.float64))
    b = ocv.brightness("power", np.hypot(X, Y), 0.3, 0.02).astype(np.float32)
    k = ctx.source_kernel_table(spec, x, y, b).cpu().numpy()
    ref = ocv.table_kernel(x, y, b, 512, 512, 8.0 / 512, 8.0 / 512)
    assert np.array_equal(k != 0, ref != 0)
    assert np.abs(k - ref).max() <= 1e-13 * ref.max()
    assert abs(k.sum() - 1.0) < 1e-12


def test_table_kernel_at_the_largest_axis(ctx):
    """RL_MAX_TABLE_AXIS samples on one axis (random order), two on the other;
    one more sample is refused before any work."""
    rng = np.random.default_rng(21)
    spec = spec_of(128, 64, 4.0, 2.0)
    n = rl.RL_MAX_TABLE_AXIS
    x = rng.uniform(-0.5, 0.5, n).astype(np.float32)
    y = np.array([-0.01, 0.02], np.float32)
    b = rng.exponential(1.0, (2, n)).astype(np.float32)
    k = ctx.source_kernel_table(spec, x, y, b).cpu().numpy()
    ref = ocv.table_kernel(x, y, b, 128, 64, 4.0 / 128, 2.0 / 64)
    assert np.array_equal(k != 0, ref != 0)
    assert np.abs(k - ref).max() <= 1e-13 * ref.max()
    x1 = np.zeros(n + 1, np.float32)
    with pytest.raises(rl.RaylensError):
        ctx.source_kernel_table(spec, x1, y, np.ones((2, n + 1), np.float32))


def test_convolution_with_a_table_kernel(ctx):
    """The table kernel feeds the convolution like the analytic one."""
    rng = np.random.default_rng(11)
    spec = spec_of(256, 256)
    x, y, b = subsample_table("gaussian", 0.2, 0.0, 4.0 / 256, 4.0 / 256, 13, 13)
    counts = torch.from_numpy(rng.poisson(50.0, (256, 256)).astype(np.int32)).cuda()
    k = ctx.source_kernel_table(spec, x, y, b)
    out = ctx.convolve(counts, k, spec, 50.0).cpu().numpy()
    ref = ocv.convolve(counts.cpu().numpy(), ocv.table_kernel(x, y, b, 256, 256, 4.0 / 256, 4.0 / 256), 50.0)
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


# Powers of two, mixed radices (2, 3, 4, 5), odd sides, rows longer than 4096
# (the 160 KiB LDS class) and columns longer than 5120 (the split pass); then
# every side of the three-pass path (256 .. 8192 and 10000) along each axis,
# and the full 10000^2 map of the high-resolution GERLUMPH datasets.
@pytest.mark.parametrize("p1,p2", [(2, 2), (16, 8), (64, 256), (1024, 512), (3, 5), (30, 12),
                                   (100, 250), (375, 81), (1000, 600), (6000, 16), (64, 6000),
                                   (2048, 10), (10240, 8), (256, 8192), (8192, 256), (512, 2048),
                                   (4096, 1024), (2048, 4096), (256, 256), (10000, 256),
                                   (256, 10000), (10000, 10000)])
def test_convolution_matches_the_oracle(ctx, p1, p2):
    rng = np.random.default_rng(p1 + p2)
    spec = spec_of(p1, p2)
    M = rng.integers(0, 1000, size=(p2, p1)).astype(np.int32)
    K = rng.random((p2, p1))
    K /= K.sum()
    out = ctx.convolve(torch.from_numpy(M).cuda(), torch.from_numpy(K).cuda(), spec, n_avg=3.7)
    ref = ocv.convolve(M, K, 3.7)
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


def test_delta_kernel_and_flux(ctx):
    rng = np.random.default_rng(5)
    spec = spec_of(256, 128)
    M = rng.integers(0, 5000, size=(128, 256)).astype(np.int32)
    K = np.zeros((128, 256))
    K[0, 0] = 1.0
    out = ctx.convolve(torch.from_numpy(M).cuda(), torch.from_numpy(K).cuda(), spec).cpu().numpy()
    assert np.abs(out - M).max() < 1e-8
    k = ctx.source_kernel(spec, "gaussian", 0.2)
    out = ctx.convolve(torch.from_numpy(M).cuda(), k, spec).cpu().numpy()
    assert abs(out.sum() - M.sum()) < 1e-9 * M.sum()


@pytest.mark.parametrize("p1,p2", [(512, 256), (256, 8192), (10000, 256)])
def test_kernels_with_zero_row_pairs(ctx, p1, p2):
    """Kernels that are zero on most rows, as source profiles are beyond
    their radius: nonzero rows alone, in pairs, straddling a pair boundary,
    the last row, and negative zeros elsewhere; then an all-zero kernel."""
    rng = np.random.default_rng(p1 * 7 + p2)
    spec = spec_of(p1, p2)
    M = rng.integers(0, 1000, size=(p2, p1)).astype(np.int32)
    K = np.full((p2, p1), -0.0)
    for r in (0, 1, 5, 6, 7, 64, p2 // 2 + 1, p2 - 2, p2 - 1):
        K[r] = rng.random(p1) * (rng.random(p1) < 0.3)
    K[3, p1 - 1] = 1e-300                      # a lone tiny value keeps its pair
    K /= K.sum()
    out = ctx.convolve(torch.from_numpy(M).cuda(), torch.from_numpy(K).cuda(), spec, n_avg=2.0)
    ref = ocv.convolve(M, K, 2.0)
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    zero = np.zeros((p2, p1))
    out = ctx.convolve(torch.from_numpy(M).cuda(), torch.from_numpy(zero).cuda(), spec, n_avg=2.0)
    assert not out.cpu().numpy().any()


def test_kernel_support_changing_between_calls():
    """Pass A leaves rows of the kernel's spectrum that are known to hold
    zeros from the previous call alone: a fresh context convolves with
    kernels whose nonzero rows move from call to call (and an all-zero, a
    dense kernel, and a call with other sides in between, which resets what
    is known), every result against the oracle."""
    c = rl.Context(0)
    try:
        rng = np.random.default_rng(23)
        p1, p2 = 512, 256

        def kernel(rows):
            K = np.zeros((p2, p1))
            for r in rows:
                K[r] = rng.random(p1)
            return K / K.sum() if K.any() else K

        dense = rng.random((p2, p1))
        dense /= dense.sum()
        seq = [kernel((0, 1, 2)), kernel((100, 101, 150)), kernel((0, 1, 2)), np.zeros((p2, p1)),
               kernel((0, p2 - 1)), "other", kernel((100, 101, 150)), dense, kernel((7,)),
               kernel((0, 1, 2))]
        spec = spec_of(p1, p2)
        for K in seq:
            if isinstance(K, str):
                spec_o = spec_of(256, 512)
                Mo = rng.integers(0, 900, size=(512, 256)).astype(np.int32)
                Ko = rng.random((512, 256))
                Ko /= Ko.sum()
                out = c.convolve(torch.from_numpy(Mo).cuda(), torch.from_numpy(Ko).cuda(), spec_o, n_avg=2.0)
                ref = ocv.convolve(Mo, Ko, 2.0)
                assert np.abs(out.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
                continue
            M = rng.integers(0, 900, size=(p2, p1)).astype(np.int32)
            out = c.convolve(torch.from_numpy(M).cuda(), torch.from_numpy(K).cuda(), spec, n_avg=2.0)
            ref = ocv.convolve(M, K, 2.0)
            tol = 1e-12 * max(np.abs(ref).max(), 1.0)
            assert np.abs(out.cpu().numpy() - ref).max() <= tol
    finally:
        c.close()


def test_finite_source_map_of_the_full_size_workload(ctx):
    """The 4096^2 GERLUMPH-like map convolved with a Gaussian disc of radius
    0.2 Einstein radii (1e16 cm for R_Ein = 5e16 cm), as magnification."""
    spec = inputs.config_gerlumph()
    f = spec.lenses()
    counts, _ = ctx.shoot(rl.DeviceLenses(f.x1, f.x2, f.m), spec, "fp32c")
    navg = rl.rl_n_avg(rl.grid_of(spec), rl.window_of(spec))
    k = ctx.source_kernel(spec, "gaussian", 0.2)
    mu = ctx.convolve(counts, k, spec, n_avg=navg).cpu().numpy()
    ref = ocv.convolve(counts.cpu().numpy(), k.cpu().numpy(), navg)
    assert np.abs(mu - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(mu.mean() - counts.sum().item() / counts.numel() / navg) < 1e-9
    # smoothing: the convolved map varies less than the point-source map
    assert mu.std() < (counts.cpu().numpy() / navg).std()


def test_convolution_of_a_10000sq_map_at_sampled_pixels(ctx):
    """A 10000^2 map (the GERLUMPH high-resolution size) with a uniform disc:
    sampled pixels against the defining sum, flux against the map's."""
    rng = np.random.default_rng(77)
    spec = spec_of(10000, 10000, 25.0, 25.0)
    M = rng.poisson(40.0, size=(10000, 10000)).astype(np.int32)
    M[5000:5100, 5000:5100] += 3000            # a caustic-like bright patch
    k = ctx.source_kernel(spec, "uniform", 0.05)
    mu = ctx.convolve(torch.from_numpy(M).cuda(), k, spec, n_avg=40.0).cpu().numpy()
    pts = [(int(a), int(b)) for a, b in rng.integers(0, 10000, size=(200, 2))]
    pts += [(0, 0), (9999, 9999), (0, 9999), (5000, 5000), (5099, 5099), (4990, 5010)]
    ref = ocv.convolve_at(M, k.cpu().numpy(), pts, 40.0)
    got = np.array([mu[j, i] for j, i in pts])
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(mu.sum() * 40.0 - M.sum(dtype=np.int64)) < 1e-9 * M.sum(dtype=np.int64)


@pytest.mark.parametrize("p1,p2", [(512, 256), (4096, 512), (256, 10000), (300, 120)])
def test_batch_equals_single_calls(p1, p2):
    """rl_convolve_batch (the map's transforms once, then each kernel) gives
    the same bits as one rl_convolve per kernel: source profiles of several
    sizes, a dense kernel and a zero kernel, on the power-of-two path and on
    the general path (300 x 120, one five-pass convolution per kernel); the
    first result also against the oracle."""
    c = rl.Context(0)
    try:
        rng = np.random.default_rng(p1 + 3 * p2)
        spec = spec_of(p1, p2)
        M = torch.from_numpy(rng.integers(0, 900, size=(p2, p1)).astype(np.int32)).cuda()
        dense = rng.random((p2, p1))
        dense /= dense.sum()
        kernels = [c.source_kernel(spec, "gaussian", 0.05), c.source_kernel(spec, "uniform", 0.11),
                   torch.from_numpy(dense).cuda(), torch.zeros((p2, p1), dtype=torch.float64, device="cuda"),
                   c.source_kernel(spec, "power", 0.08, 0.01)]
        outs = c.convolve_batch(M, kernels, spec, n_avg=2.5)
        torch.cuda.synchronize()
        for q, k in enumerate(kernels):
            one = c.convolve(M, k, spec, n_avg=2.5)
            assert torch.equal(outs[q], one), q
        ref = ocv.convolve(M.cpu().numpy(), kernels[0].cpu().numpy(), 2.5)
        assert np.abs(outs[0].cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
        # a zero kernel convolves to exact zeros on both paths (the general one
        # packs M + i 2^e K into one transform and takes the kernel's zero norm
        # as the factor on the way out)
        assert not outs[3].cpu().numpy().any()
    finally:
        c.close()


def test_cached_twiddles_across_calls():
    """A fresh context convolves sides in the order A, A, B, A, C (C larger,
    so the scratch is reallocated), A: the stage-twiddle tables are reused
    only while the sides and the scratch buffer are the same, and every call
    gives the same bits as the first call for its sides."""
    c = rl.Context(0)
    try:
        rng = np.random.default_rng(17)
        sides = {"A": (512, 256), "B": (300, 120), "C": (2048, 1024)}
        data = {}
        for name, (p1, p2) in sides.items():
            M = rng.integers(0, 900, size=(p2, p1)).astype(np.int32)
            K = rng.random((p2, p1))
            K /= K.sum()
            data[name] = (spec_of(p1, p2), torch.from_numpy(M).cuda(), torch.from_numpy(K).cuda(),
                          ocv.convolve(M, K, 2.5))
        first = {}
        for name in ["A", "A", "B", "A", "C", "A"]:
            spec, M, K, ref = data[name]
            out = c.convolve(M, K, spec, n_avg=2.5).cpu().numpy()
            assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max(), name
            if name in first:
                assert np.array_equal(out, first[name]), name
            first.setdefault(name, out)
    finally:
        c.close()

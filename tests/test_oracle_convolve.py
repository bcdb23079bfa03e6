"""Pins of the oracle's finite-source convolution (Section 2.4, eq. 6)."""
import math

import numpy as np
import pytest

from oracle import convolve as cv


def test_fft_convolution_equals_the_defining_sum():
    rng = np.random.default_rng(1)
    M = rng.integers(0, 50, size=(32, 48)).astype(np.float64)
    for shape, R in (("uniform", 2.5), ("gaussian", 3.0), ("power", 4.0)):
        K = cv.source_kernel(shape, 48, 32, 1.0, 1.0, R)
        assert np.allclose(cv.convolve(M, K), cv.convolve_direct(M, K), rtol=0, atol=1e-10)


def test_delta_kernel_is_the_identity_and_flux_is_conserved():
    rng = np.random.default_rng(2)
    M = rng.integers(0, 1000, size=(64, 64)).astype(np.float64)
    K = np.zeros_like(M)
    K[0, 0] = 1.0
    assert np.allclose(cv.convolve(M, K), M, rtol=0, atol=1e-9)
    K = cv.source_kernel("gaussian", 64, 64, 1.0, 1.0, 6.0)
    C = cv.convolve(M, K)
    assert abs(C.sum() - M.sum()) < 1e-8 * M.sum()
    assert abs(cv.convolve(M, K, n_avg=4.0).sum() - M.sum() / 4.0) < 1e-8 * M.sum()


def test_shift_equivariance():
    rng = np.random.default_rng(3)
    M = rng.random((32, 32))
    K = cv.source_kernel("power", 32, 32, 1.0, 1.0, 3.0, hole=0.5)
    a = np.roll(cv.convolve(M, K), (3, -5), axis=(0, 1))
    b = cv.convolve(np.roll(M, (3, -5), axis=(0, 1)), K)
    assert np.allclose(a, b, atol=1e-12)


def test_uniform_kernel_weights_match_disc_area():
    """A large uniform disc: the kernel is ~1/(pi R^2) inside and 0 outside, and
    its number of touched pixels matches the disc area up to the rim."""
    R = 20.0
    K = cv.source_kernel("uniform", 128, 128, 1.0, 1.0, R)
    assert abs(K.sum() - 1.0) < 1e-12
    assert abs(K[0, 0] * math.pi * R * R - 1.0) < 0.01
    full = np.count_nonzero(K > 0.999 * K[0, 0])
    assert abs(full - math.pi * R * R) < 2 * math.pi * R
    assert K[0, 25] == 0.0 and K[25, 0] == 0.0


def test_profile_shapes():
    r = np.array([0.0, 0.5, 1.0, 2.0, 2.999, 3.0, 4.0])
    u = cv.brightness("uniform", r, 3.0)
    assert u.tolist() == [1, 1, 1, 1, 1, 0, 0]
    g = cv.brightness("gaussian", r, 3.0)
    assert g[0] == 1.0 and abs(g[3] - math.exp(-2.0)) < 1e-15 and g[5] == 0.0
    p = cv.brightness("power", r, 3.0)
    assert abs(p[0] - (0.03 / 3.0) ** -0.75) < 1e-12           # flat inside the core r < R/100
    assert abs(p[1] - (0.5 / 3.0) ** -0.75) < 1e-12
    assert abs(p[4] / p[3] - (2.999 / 2.0) ** -0.75) < 1e-12
    h = cv.brightness("uniform", r, 3.0, hole=1.0)
    assert h.tolist() == [0, 0, 1, 1, 1, 0, 0]


def test_invalid():
    with pytest.raises(ValueError):
        cv.source_kernel("uniform", 16, 16, 1.0, 1.0, 10.0)
    with pytest.raises(ValueError):
        cv.brightness("cone", 1.0, 2.0)


def test_convolve_at_agrees_with_the_direct_sum():
    rng = np.random.default_rng(8)
    M = rng.integers(0, 100, size=(24, 36)).astype(np.int32)
    K = cv.source_kernel("power", 36, 24, 0.1, 0.1, 0.35, 0.05)
    full = cv.convolve_direct(M, K, 2.0)
    pts = [(0, 0), (23, 35), (5, 30), (12, 0)]
    assert np.allclose(cv.convolve_at(M, K, pts, 2.0), [full[j, i] for j, i in pts], rtol=1e-14)


def _signed(n):
    """Signed offsets of the wrapped indices 0..n-1 (n - k stands for -k)."""
    k = np.arange(n)
    return np.where(k <= n // 2, k, k - n)


@pytest.mark.parametrize("shape", ["uniform", "gaussian", "power"])
@pytest.mark.parametrize("pix1,pix2,R,hole", [(1.0, 1.0, 3.3, 0.0), (0.7, 1.3, 4.1, 0.0),
                                               (1.0, 1.0, 5.2, 1.7), (0.25, 0.4, 2.05, 0.0)])
def test_source_kernel_is_centred_on_pixel_zero(shape, pix1, pix2, R, hole):
    """A circular profile centred on pixel (0, 0) (Section 2.4: the kernel is the
    binned profile; centred, the convolved map is not shifted): the kernel is
    unchanged under x1 -> -x1 and x2 -> -x2 separately, its centroid in wrapped
    pixel offsets is (0, 0), and without a hole its largest value sits at
    (0, 0). A kernel whose sub-samples or pixels are offset breaks all three."""
    p1, p2 = 40, 36
    K = cv.source_kernel(shape, p1, p2, pix1, pix2, R, hole)
    flip1 = K[:, (-np.arange(p1)) % p1]
    flip2 = K[(-np.arange(p2)) % p2, :]
    assert np.allclose(K, flip1, rtol=1e-13, atol=1e-16)
    assert np.allclose(K, flip2, rtol=1e-13, atol=1e-16)
    s1, s2 = _signed(p1), _signed(p2)
    assert abs(float(np.sum(K * s1[None, :]))) < 1e-13
    assert abs(float(np.sum(K * s2[:, None]))) < 1e-13
    if hole == 0.0:
        assert K[0, 0] == K.max()
    # the support reaches ceil(R / pix) pixels from the centre on each side
    n1, n2 = int(np.ceil(R / pix1)), int(np.ceil(R / pix2))
    nz_b, nz_a = np.nonzero(K)
    assert np.abs(s1[nz_a]).max() <= n1 and np.abs(s2[nz_b]).max() <= n2


def test_convolution_with_an_offset_delta_shifts_the_map():
    """Eq. 6 is a convolution, not a correlation: a unit kernel at offset (b, a)
    moves every pixel by (+b, +a), C[j, i] = M[j - b, i - a] (wrapped)."""
    rng = np.random.default_rng(5)
    M = rng.integers(0, 1000, size=(24, 40)).astype(np.float64)
    K = np.zeros_like(M)
    K[3, 5] = 1.0
    want = np.roll(M, (3, 5), axis=(0, 1))
    assert np.allclose(cv.convolve(M, K), want, rtol=0, atol=1e-9)
    assert np.array_equal(cv.convolve_direct(M, K), want)
    assert np.array_equal(cv.convolve_at(M.astype(np.int32), K, [(0, 0), (7, 39)]),
                          [want[0, 0], want[7, 39]])


def test_fft_convolution_with_an_asymmetric_kernel_equals_the_defining_sum():
    rng = np.random.default_rng(6)
    M = rng.integers(0, 50, size=(30, 20)).astype(np.float64)
    K = np.zeros_like(M)
    K[:4, :3] = rng.random((4, 3))
    K[-2:, -1] = rng.random(2)
    assert np.allclose(cv.convolve(M, K, 3.0), cv.convolve_direct(M, K, 3.0), rtol=0, atol=1e-10)


# ---------------------------------------------------------------------------
# Kernels of tabulated profiles (profile.bin)
# ---------------------------------------------------------------------------

def subsample_table(shape, radius, hole, pix1, pix2, n1, n2, s=8):
    """A profile tabulated at the sub-sample points that source_kernel
    averages over, pixels -n .. n on each axis: float32 positions, as the
    files store them."""
    off = (np.arange(s) + 0.5) / s - 0.5
    x = ((np.arange(-n1, n1 + 1)[:, None] + off[None, :]).ravel() * pix1).astype(np.float32)
    y = ((np.arange(-n2, n2 + 1)[:, None] + off[None, :]).ravel() * pix2).astype(np.float32)
    X, Y = np.meshgrid(x.astype(np.float64), y.astype(np.float64))
    b = cv.brightness(shape, np.hypot(X, Y), radius, hole).astype(np.float32)
    return x, y, b


@pytest.mark.parametrize("shape,R,hole", [("uniform", 3.3, 0.0), ("gaussian", 4.1, 0.0), ("power", 5.2, 0.7)])
def test_table_kernel_at_the_subsample_points_is_the_analytic_kernel(shape, R, hole):
    """Tabulated at the points where source_kernel samples the profile, a
    profile binned by table_kernel gives source_kernel's kernel: each pixel
    holds the same 64 samples, summed instead of averaged, and both kernels
    are normalised (to float32 precision of the tabulated brightness)."""
    pix1, pix2, p1, p2 = 1.0, 0.8, 48, 40
    n1, n2 = int(math.ceil(R / pix1)), int(math.ceil(R / pix2))
    x, y, b = subsample_table(shape, R, hole, pix1, pix2, n1, n2)
    got = cv.table_kernel(x, y, b, p1, p2, pix1, pix2)
    ref = cv.source_kernel(shape, p1, p2, pix1, pix2, R, hole)
    assert np.abs(got - ref).max() <= 1e-6 * ref.max()
    assert abs(got.sum() - 1.0) < 1e-12


def test_table_kernel_of_one_sample_is_a_delta():
    K = cv.table_kernel([0.0], [0.0], [5.0], 16, 8, 1.0, 1.0)
    assert K[0, 0] == 1.0 and K.sum() == 1.0
    # off-centre sample: pixel (floor(x / pix + 1/2), ...), wrapped
    K = cv.table_kernel([-1.49], [2.51], [2.0], 16, 8, 1.0, 1.0)
    assert K[3, 16 - 1] == 1.0 and K.sum() == 1.0


def test_table_kernel_box_edges_are_half_open():
    """A sample exactly on a box edge x = (i + 1/2) pix belongs to pixel i + 1."""
    K = cv.table_kernel([0.5, -0.5], [0.0], [1.0, 3.0], 8, 8, 1.0, 1.0)
    assert K[0, 1] == 0.25 and K[0, 0] == 0.75


def test_table_kernel_of_a_source_too_large_is_refused():
    with pytest.raises(ValueError):
        cv.table_kernel([-5.0, 5.0], [0.0], [1.0, 1.0], 8, 8, 1.0, 1.0)

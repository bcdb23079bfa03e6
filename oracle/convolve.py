"""Finite-source maps: convolution of a map with a source profile (oracle).

Vernardos & Fluke 2014, Section 2.4: the projected source profile is binned
in pixels of the map's pixel size and padded with zeros to the map's size,
which gives the convolution kernel K; the convolved map is
C = M * K = F^-1[F(M) F(K)] (eq. 6). Section 3.1 lists the profile shapes
(uniform disc, Gaussian, thin-disc power law, profiles with a central hole)
and defines a profile's size as the radius where its brightness drops to
zero (Table "components": 0.5-50 x 10^15 cm, with R_Ein 1-9 x 10^16 cm).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py). Plain numpy in FP64; the
FFT is numpy's, used as a library step of the definition.

Readings (also listed in the design notes):
  * the kernel is centred on pixel (0, 0) and wraps around, so C is not
    shifted; it is normalised to unit sum, so the mean of C equals the mean
    of M (the convolution redistributes rays, it does not create them);
  * a kernel pixel's value is the mean brightness over an s x s grid of
    sub-samples at the sub-pixel centres (s = 8);
  * uniform: I = 1 for r < R; gaussian: I = exp(-r^2 / (2 sigma^2)) with
    sigma = R / 3, cut at R; power: I = (max(r, r_core) / R)^(-3/4) for r < R
    (the thin-disc temperature slope) with r_core = R / 100; a hole of radius
    r_hole sets I = 0 for r < r_hole in any shape.
"""
import numpy as np

SHAPES = ("uniform", "gaussian", "power")
SUBSAMPLES = 8


def brightness(shape, r, radius, hole=0.0):
    """Profile brightness at distance r (same units as radius)."""
    r = np.asarray(r, dtype=np.float64)
    if shape == "uniform":
        I = np.ones_like(r)
    elif shape == "gaussian":
        sigma = radius / 3.0
        I = np.exp(-(r * r) / (2.0 * sigma * sigma))
    elif shape == "power":
        core = radius / 100.0
        I = (np.maximum(r, core) / radius) ** (-0.75)
    else:
        raise ValueError(f"unknown profile shape {shape!r}")
    return np.where((r < radius) & (r >= hole), I, 0.0)


def source_kernel(shape, p1, p2, pix1, pix2, radius, hole=0.0, subsamples=SUBSAMPLES):
    """Kernel of a circular source of the given radius (map units) on a p2 x p1
    map with pixel sizes pix1 x pix2, centred on pixel (0, 0) with wrap-around,
    normalised to unit sum."""
    if radius <= 0 or pix1 <= 0 or pix2 <= 0:
        raise ValueError("radius and pixel sizes must be > 0")
    n1 = int(np.ceil(radius / pix1))
    n2 = int(np.ceil(radius / pix2))
    if 2 * n1 + 1 > p1 or 2 * n2 + 1 > p2:
        raise ValueError("source larger than the map")
    K = np.zeros((p2, p1), np.float64)
    off = (np.arange(subsamples) + 0.5) / subsamples - 0.5
    for j in range(-n2, n2 + 1):
        for i in range(-n1, n1 + 1):
            x = (i + off)[None, :] * pix1
            y = (j + off)[:, None] * pix2
            K[j % p2, i % p1] = brightness(shape, np.hypot(x, y), radius, hole).mean()
    total = K.sum()
    if not total > 0:
        raise ValueError("empty source kernel")
    return K / total


def table_kernel(x, y, b, p1, p2, pix1, pix2):
    """Kernel of a tabulated profile (the disc profiles of Section 3.1, stored
    as in the disc table of Section 3.2: N_x x values, N_y y values, then N_x
    N_y brightness values, read with x fastest), positions in the map's units:
    each pixel (i, j) around the source centre sums the brightness of the
    samples it holds, sample (x, y) being in pixel (floor(x / pix1 + 1/2),
    floor(y / pix2 + 1/2)); the sums are taken in the table's order (y, then
    x), centred on pixel (0, 0) with wrap-around and normalised to unit sum
    like source_kernel."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64).reshape(len(y), len(x))
    ix = np.floor(x / pix1 + 0.5).astype(np.int64)
    iy = np.floor(y / pix2 + 0.5).astype(np.int64)
    h1, h2 = int(np.abs(ix).max()), int(np.abs(iy).max())
    if 2 * h1 + 1 > p1 or 2 * h2 + 1 > p2:
        raise ValueError("source larger than the map")
    compact = np.zeros((2 * h2 + 1, 2 * h1 + 1), np.float64)
    for ky in range(len(y)):
        for kx in range(len(x)):
            compact[iy[ky] + h2, ix[kx] + h1] += b[ky, kx]
    total = compact.sum()
    if not total > 0:
        raise ValueError("empty source kernel")
    K = np.zeros((p2, p1), np.float64)
    for j in range(-h2, h2 + 1):
        for i in range(-h1, h1 + 1):
            K[j % p2, i % p1] = compact[j + h2, i + h1] / total
    return K


def convolve(counts, kernel, n_avg=1.0):
    """C = F^-1[F(M) F(K)] / n_avg in FP64 (eq. 6); circular."""
    M = np.asarray(counts, dtype=np.float64)
    K = np.asarray(kernel, dtype=np.float64)
    if M.shape != K.shape:
        raise ValueError("map and kernel differ in shape")
    C = np.fft.ifft2(np.fft.fft2(M) * np.fft.fft2(K)).real
    return C / n_avg


def convolve_direct(counts, kernel, n_avg=1.0):
    """The same circular convolution by the defining sum (small maps only):
    C[j, i] = sum over (b, a) of K[b, a] M[(j - b) mod p2, (i - a) mod p1]."""
    M = np.asarray(counts, dtype=np.float64)
    K = np.asarray(kernel, dtype=np.float64)
    C = np.zeros_like(M)
    for b, a in zip(*np.nonzero(K)):
        C += K[b, a] * np.roll(np.roll(M, b, axis=0), a, axis=1)
    return C / n_avg


def convolve_at(counts, kernel, points, n_avg=1.0):
    """C at the given pixels (j, i) by the defining sum over the kernel's
    non-zero entries, for spot checks of large maps:
    C[j, i] = sum over (b, a) of K[b, a] M[(j - b) mod p2, (i - a) mod p1] / n_avg."""
    M = np.asarray(counts)
    K = np.asarray(kernel, dtype=np.float64)
    p2, p1 = M.shape
    nz_b, nz_a = np.nonzero(K)
    w = K[nz_b, nz_a]
    out = []
    for j, i in points:
        vals = M[(j - nz_b) % p2, (i - nz_a) % p1].astype(np.float64)
        out.append(float(np.sum(w * vals)) / n_avg)
    return np.array(out)

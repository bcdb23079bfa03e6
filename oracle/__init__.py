"""Plain FP64 CPU oracle for direct inverse ray-shooting (ctypes wrapper).

Vernardos & Fluke 2014, Section 2.1, eq. 1-4. TEST INFRASTRUCTURE ONLY: the
tests, the smoke check and the CPU-baseline leg of the benchmark are the only
users. It shares no code with the HIP library and imports nothing from it.

All arrays are numpy arrays on the host. Parameters are passed as plain numbers
so that nothing here depends on the library's structures.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB points the wrapper at another build of oracle.c (the
        # mutation tests use it to check that planted mistakes are caught).
        path = os.environ.get("ORACLE_LIB") or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        i64, i32, dbl = C.c_int64, C.c_int32, C.c_double
        vp = C.c_void_p
        L.oracle_ray_positions.argtypes = [vp, vp, vp, i64, dbl, dbl, dbl, i64, i64, dbl, dbl, dbl,
                                           dbl, i64, i64, vp, vp, vp, vp]
        L.oracle_bin.argtypes = [vp, vp, vp, i64, i32, i32, dbl, dbl, dbl, dbl, vp, vp]
        L.oracle_shoot.argtypes = [vp, vp, vp, i64, dbl, dbl, dbl, i64, i64, dbl, dbl, dbl, dbl,
                                   i32, i32, dbl, dbl, dbl, dbl, i64, i64, vp, vp, C.c_int]
        L.oracle_n_avg.argtypes = [i64, i64, dbl, dbl, i32, i32, dbl, dbl]
        L.oracle_n_avg.restype = dbl
        L.oracle_normalise.argtypes = [vp, i64, dbl, vp]
        L.oracle_stats.argtypes = [vp, i64, dbl, dbl, dbl, vp]
        L.oracle_count_histogram.argtypes = [vp, i64, i64, vp]
        L.oracle_mpd_thresholds.argtypes = [dbl, dbl, dbl, dbl, i32, vp]
        L.oracle_mpd.argtypes = [vp, i64, vp, i32, vp]
        L.oracle_mpd_values.argtypes = [vp, i64, vp, i32, vp]
        L.oracle_probability_sums.argtypes = [vp, i64, dbl, dbl, vp, vp]
        L.oracle_codec_encode.argtypes = [vp, i64, vp, vp, vp, vp]
        L.oracle_codec_decode.argtypes = [vp, i64, i32, vp, i64, vp]
        for f in ("oracle_ray_positions", "oracle_bin", "oracle_shoot", "oracle_normalise",
                  "oracle_stats", "oracle_max_threads", "oracle_count_histogram",
                  "oracle_mpd_thresholds", "oracle_mpd", "oracle_mpd_values", "oracle_probability_sums",
                  "oracle_codec_encode", "oracle_codec_decode"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _lens_arrays(x1, x2, m):
    x1 = np.ascontiguousarray(x1, dtype=np.float64)
    x2 = np.ascontiguousarray(x2, dtype=np.float64)
    if x1.shape != x2.shape or x1.ndim != 1:
        raise ValueError("lens coordinate arrays must be 1-D and of equal length")
    if m is not None:
        m = np.ascontiguousarray(m, dtype=np.float64)
        if m.shape != x1.shape:
            raise ValueError("mass array must match the lens coordinates")
    return x1, x2, m


def max_threads():
    return lib().oracle_max_threads()


def ray_positions(x1, x2, m, kappa, gamma, s, n1, n2, c1, c2, h1, h2, row_begin=0, row_end=None):
    """Eq. 1 per ray for rows [row_begin, row_end). Returns (y1, y2, singular, rmin),
    each shaped (rows, n1)."""
    x1, x2, m = _lens_arrays(x1, x2, m)
    if row_end is None:
        row_end = n2
    rows = row_end - row_begin
    shape = (max(rows, 0), n1)
    y1 = np.empty(shape, np.float64)
    y2 = np.empty(shape, np.float64)
    sing = np.empty(shape, np.uint8)
    rmin = np.empty(shape, np.float64)
    rc = lib().oracle_ray_positions(_p(x1), _p(x2), _p(m), x1.size, kappa, gamma, s, n1, n2,
                                    c1, c2, h1, h2, row_begin, row_end,
                                    _p(y1), _p(y2), _p(sing), _p(rmin))
    if rc != 0:
        raise ValueError("oracle_ray_positions: invalid arguments")
    return y1, y2, sing, rmin


def bin_positions(y1, y2, p1, p2, w1, w2, W1, W2, singular=None, counts=None):
    """Bins given positions. Returns (counts[p2, p1] int32, escaped)."""
    y1 = np.ascontiguousarray(y1, dtype=np.float64).ravel()
    y2 = np.ascontiguousarray(y2, dtype=np.float64).ravel()
    if y1.shape != y2.shape:
        raise ValueError("y1 and y2 differ in size")
    if singular is not None:
        singular = np.ascontiguousarray(singular, dtype=np.uint8).ravel()
    if counts is None:
        counts = np.zeros((p2, p1), np.int32)
    esc = np.zeros(1, np.int64)
    rc = lib().oracle_bin(_p(y1), _p(y2), _p(singular), y1.size, p1, p2, w1, w2, W1, W2,
                          _p(counts), _p(esc))
    if rc != 0:
        raise ValueError("oracle_bin: invalid arguments")
    return counts, int(esc[0])


def shoot(x1, x2, m, kappa, gamma, s, n1, n2, c1, c2, h1, h2, p1, p2, w1, w2, W1, W2,
          row_begin=0, row_end=None, nthreads=0, counts=None):
    """Eq. 1 + binning for rows [row_begin, row_end). Returns (counts[p2, p1], escaped)."""
    x1, x2, m = _lens_arrays(x1, x2, m)
    if row_end is None:
        row_end = n2
    if counts is None:
        counts = np.zeros((p2, p1), np.int32)
    esc = np.zeros(1, np.int64)
    rc = lib().oracle_shoot(_p(x1), _p(x2), _p(m), x1.size, kappa, gamma, s, n1, n2, c1, c2,
                            h1, h2, p1, p2, w1, w2, W1, W2, row_begin, row_end,
                            _p(counts), _p(esc), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_shoot: invalid arguments")
    return counts, int(esc[0])


def n_avg(n1, n2, h1, h2, p1, p2, W1, W2):
    return lib().oracle_n_avg(n1, n2, h1, h2, p1, p2, W1, W2)


def normalise(counts, n_avg_value):
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    mu = np.empty(counts.shape, np.float32)
    rc = lib().oracle_normalise(_p(counts), counts.size, n_avg_value, _p(mu))
    if rc != 0:
        raise ValueError("oracle_normalise: invalid arguments")
    return mu


def stats(counts, n_avg_value, kappa, gamma):
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    out = np.zeros(4, np.float64)
    rc = lib().oracle_stats(_p(counts), counts.size, n_avg_value, kappa, gamma, _p(out))
    if rc != 0:
        raise ValueError("oracle_stats: invalid arguments")
    return {"binned": int(out[0]), "mean_count": out[1], "mean_mu": out[2], "mu_th": out[3]}


def count_histogram(counts, n_values):
    """Frequency of each count value (Section 3.2.1's MPD before division by
    the pixel count); values >= n_values - 1 land in the last entry."""
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    hist = np.zeros(int(n_values), np.int64)
    if lib().oracle_count_histogram(_p(counts), counts.size, int(n_values), _p(hist)) != 0:
        raise ValueError("oracle_count_histogram: invalid arguments")
    return hist


def mpd_thresholds(n_avg_value, mu_ref, log_lo, log_hi, nbins):
    thr = np.zeros(int(nbins) + 1, np.float64)
    if lib().oracle_mpd_thresholds(n_avg_value, mu_ref, log_lo, log_hi, int(nbins), _p(thr)) != 0:
        raise ValueError("oracle_mpd_thresholds: invalid arguments")
    return thr


def mpd(counts, n_avg_value, mu_ref, log_lo, log_hi, nbins):
    """Binned MPD in log10(mu / mu_ref): [underflow, nbins bins, overflow]
    pixel counts (divide by the pixel count for probabilities)."""
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    thr = mpd_thresholds(n_avg_value, mu_ref, log_lo, log_hi, nbins)
    bins = np.zeros(int(nbins) + 2, np.int64)
    if lib().oracle_mpd(_p(counts), counts.size, _p(thr), int(nbins), _p(bins)) != 0:
        raise ValueError("oracle_mpd: invalid arguments")
    return bins


def mpd_values(mu, mu_ref, log_lo, log_hi, nbins):
    """Binned MPD of a map of real magnifications (a finite-source map) in
    log10(mu / mu_ref): [underflow, nbins bins, overflow] pixel counts; the
    thresholds are mu_ref 10^edge (mpd_thresholds with n_avg = 1)."""
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    thr = mpd_thresholds(1.0, mu_ref, log_lo, log_hi, nbins)
    bins = np.zeros(int(nbins) + 2, np.int64)
    if lib().oracle_mpd_values(_p(mu), mu.size, _p(thr), int(nbins), _p(bins)) != 0:
        raise ValueError("oracle_mpd_values: invalid arguments")
    return bins


def probability_sums(counts, n_avg_value, mu_lim):
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    lo = np.zeros(1, np.int64)
    hi = np.zeros(1, np.int64)
    if lib().oracle_probability_sums(_p(counts), counts.size, n_avg_value, mu_lim, _p(lo), _p(hi)) != 0:
        raise ValueError("oracle_probability_sums: invalid arguments")
    return int(lo[0]), int(hi[0])


def codec_encode(counts):
    """Indexed map of Appendix B: returns (values, bits, packed uint32 words)."""
    counts = np.ascontiguousarray(counts, dtype=np.int32).ravel()
    values = np.zeros(counts.size, np.int32)
    nd = np.zeros(1, np.int64)
    bits = np.zeros(1, np.int32)
    packed = np.zeros(counts.size, np.uint32)
    if lib().oracle_codec_encode(_p(counts), counts.size, _p(values), _p(nd), _p(bits), _p(packed)) != 0:
        raise ValueError("oracle_codec_encode: invalid arguments")
    b = int(bits[0])
    words = (counts.size * b + 31) // 32
    return values[: int(nd[0])].copy(), b, packed[:words].copy()


def codec_decode(packed, n_pix, bits, values):
    packed = np.ascontiguousarray(packed, dtype=np.uint32)
    values = np.ascontiguousarray(values, dtype=np.int32)
    counts = np.zeros(int(n_pix), np.int32)
    if packed.size < (int(n_pix) * int(bits) + 31) // 32:
        raise ValueError("packed stream too short")
    if lib().oracle_codec_decode(_p(packed), int(n_pix), int(bits), _p(values), values.size,
                                 _p(counts)) != 0:
        raise ValueError("oracle_codec_decode: invalid arguments")
    return counts

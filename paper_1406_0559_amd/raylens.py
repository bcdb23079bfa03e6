"""Thin ctypes binding of the raylens C-ABI (include/raylens.h).

Functions keep the C names (rl_create, rl_shoot, ...) and only marshal
arguments; every step of the computation runs in the HIP library. A missing
library is an error: there is no CPU fallback on this path.

The `Context` class adds torch plumbing (device tensors for the lens field,
count maps and magnification maps; the current torch stream) on top of the
same calls.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libraylens.so")

RL_OK, RL_E_INVALID, RL_E_NOMEM, RL_E_DEVICE, RL_E_BUSY, RL_E_CANCELLED, RL_E_OVERFLOW = range(7)
RL_FP32_COMP, RL_FP64_PLAIN = 0, 1
PRECISIONS = {"fp32c": RL_FP32_COMP, "fp64": RL_FP64_PLAIN}


class RaylensError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"raylens status {status}: {message}")
        self.status = status


class rl_macro(C.Structure):
    _fields_ = [("kappa", C.c_double), ("gamma", C.c_double), ("s", C.c_double)]


class rl_raygrid(C.Structure):
    _fields_ = [("n1", C.c_int64), ("n2", C.c_int64), ("c1", C.c_double), ("c2", C.c_double),
                ("half1", C.c_double), ("half2", C.c_double)]


class rl_window(C.Structure):
    _fields_ = [("p1", C.c_int32), ("p2", C.c_int32), ("c1", C.c_double), ("c2", C.c_double),
                ("width1", C.c_double), ("width2", C.c_double)]


class rl_lenses(C.Structure):
    _fields_ = [("x1", C.c_void_p), ("x2", C.c_void_p), ("m", C.c_void_p), ("n", C.c_int64)]


class rl_stats(C.Structure):
    _fields_ = [("shot", C.c_int64), ("binned", C.c_int64), ("escaped", C.c_int64),
                ("n_avg", C.c_double), ("mean_count", C.c_double), ("mean_mu", C.c_double),
                ("mu_th", C.c_double), ("max_count", C.c_int32)]


class rl_map_desc(C.Structure):
    _fields_ = [("lenses", rl_lenses), ("macro", rl_macro), ("grid", rl_raygrid),
                ("win", rl_window), ("row_begin", C.c_int64), ("row_end", C.c_int64),
                ("d_counts", C.c_void_p), ("d_escaped", C.c_void_p)]


class rl_profile(C.Structure):
    _fields_ = [("shape", C.c_int32), ("radius", C.c_double), ("hole", C.c_double)]


PROFILES = {"uniform": 0, "gaussian": 1, "power": 2}


class rl_tuning(C.Structure):
    _fields_ = [("rays_x", C.c_int32), ("rays_y", C.c_int32), ("lens_tile", C.c_int32),
                ("waves", C.c_int32), ("submap", C.c_int32)]


_lib = None


def load():
    """Opens libraylens.so (built by paper_1406_0559_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1406_0559_amd/build.py "
                           "(or __graft_entry__.build()); there is no fallback")
    # PyTorch ships its own HIP runtime and asks for it as "libamdhip64.so";
    # the library asks for "libamdhip64.so.7". Loading torch first makes the
    # library bind to torch's runtime (same soname), so one runtime owns the
    # streams and device memory that torch hands to the library. Loaded the
    # other way round, the process would hold two runtimes.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "rl_create": [i32, P(vp)],
        "rl_destroy": [vp],
        "rl_n_avg": [P(rl_raygrid), P(rl_window), P(dbl)],
        "rl_shoot": [vp, P(rl_lenses), P(rl_macro), P(rl_raygrid), P(rl_window), C.c_int, i64, i64,
                     vp, vp, vp],
        "rl_shoot_noalloc": [vp, P(rl_lenses), P(rl_macro), P(rl_raygrid), P(rl_window), C.c_int,
                             i64, i64, vp, vp, vp],
        "rl_normalise": [vp, vp, P(rl_window), dbl, vp, vp],
        "rl_stats_get": [vp, vp, vp, P(rl_macro), P(rl_raygrid), P(rl_window), P(rl_stats), vp],
        "rl_bin_positions": [vp, vp, vp, i64, P(rl_window), vp, vp, vp],
        "rl_ray_positions": [vp, P(rl_lenses), P(rl_macro), P(rl_raygrid), C.c_int, i64, i64, vp,
                             vp, vp],
        "rl_shoot_batch": [vp, P(rl_map_desc), i32, C.c_int, vp],
        "rl_count_histogram": [vp, vp, P(rl_window), i64, vp, vp],
        "rl_mpd": [vp, vp, P(rl_window), dbl, dbl, dbl, dbl, i32, vp, vp],
        "rl_mpd_values": [vp, vp, P(rl_window), dbl, dbl, dbl, i32, vp, vp],
        "rl_probability_sums": [vp, vp, P(rl_window), dbl, dbl, P(i64), P(i64), vp],
        "rl_mpd_moments": [vp, vp, i32, i32, i64, vp, vp, vp],
        "rl_codec_encode": [vp, vp, P(rl_window), vp, i64, vp, i64, P(i64), P(i32), vp],
        "rl_codec_decode": [vp, vp, i32, vp, i64, P(rl_window), vp, vp],
        "rl_source_kernel": [vp, P(rl_profile), P(rl_window), vp, vp],
        "rl_source_kernel_table": [vp, vp, i32, vp, i32, vp, P(rl_window), vp, vp],
        "rl_convolve": [vp, vp, vp, P(rl_window), dbl, vp, vp],
        "rl_convolve_batch": [vp, vp, P(vp), i32, P(rl_window), dbl, P(vp), vp],
        "rl_autotune": [vp, C.c_char_p, i32],
        "rl_get_tuning": [vp, C.c_int, i32, P(rl_tuning)],
        "rl_set_tuning": [vp, C.c_int, i32, P(rl_tuning)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.rl_last_error.restype = C.c_char_p
    L.rl_last_error.argtypes = []
    L.rl_version.restype = C.c_char_p
    L.rl_version.argtypes = []
    _lib = L
    return L


def _check(status):
    if status != RL_OK:
        raise RaylensError(status, load().rl_last_error().decode())


# ----------------------------------------------------------------------------
# same-name wrappers (marshalling only)
# ----------------------------------------------------------------------------

def rl_version() -> str:
    return load().rl_version().decode()


def rl_last_error() -> str:
    return load().rl_last_error().decode()


def rl_create(device: int = 0) -> int:
    out = C.c_void_p()
    _check(load().rl_create(device, C.byref(out)))
    return out.value


def rl_destroy(ctx: int) -> None:
    _check(load().rl_destroy(ctx))


def rl_n_avg(grid: rl_raygrid, win: rl_window) -> float:
    out = C.c_double()
    _check(load().rl_n_avg(C.byref(grid), C.byref(win), C.byref(out)))
    return out.value


def rl_shoot(ctx, lenses, macro, grid, win, precision, row_begin, row_end, d_counts, d_escaped,
             stream=None):
    _check(load().rl_shoot(ctx, C.byref(lenses), C.byref(macro), C.byref(grid), C.byref(win),
                           precision, row_begin, row_end, d_counts, d_escaped, stream))


def rl_shoot_noalloc(ctx, lenses, macro, grid, win, precision, row_begin, row_end, d_counts,
                     d_escaped, stream=None):
    _check(load().rl_shoot_noalloc(ctx, C.byref(lenses), C.byref(macro), C.byref(grid),
                                   C.byref(win), precision, row_begin, row_end, d_counts,
                                   d_escaped, stream))


RL_NOALLOC_MAX_LENSES = 131072   # include/raylens.h
RL_MAX_CONVOLVE_BATCH = 4096     # include/raylens.h
RL_MAX_TABLE_AXIS = 16384        # include/raylens.h


def rl_normalise(ctx, d_counts, win, n_avg, d_mu, stream=None):
    _check(load().rl_normalise(ctx, d_counts, C.byref(win), n_avg, d_mu, stream))


def rl_stats_get(ctx, d_counts, d_escaped, macro, grid, win, stream=None, allow_overflow=False):
    st = rl_stats()
    status = load().rl_stats_get(ctx, d_counts, d_escaped, C.byref(macro), C.byref(grid),
                                 C.byref(win), C.byref(st), stream)
    if not (allow_overflow and status == RL_E_OVERFLOW):
        _check(status)
    return st


def rl_bin_positions(ctx, d_y1, d_y2, n, win, d_counts, d_escaped, stream=None):
    _check(load().rl_bin_positions(ctx, d_y1, d_y2, n, C.byref(win), d_counts, d_escaped, stream))


def rl_ray_positions(ctx, lenses, macro, grid, precision, row_begin, row_end, d_y1, d_y2,
                     stream=None):
    _check(load().rl_ray_positions(ctx, C.byref(lenses), C.byref(macro), C.byref(grid), precision,
                                   row_begin, row_end, d_y1, d_y2, stream))


def rl_shoot_batch(ctx, descs: Sequence[rl_map_desc], precision, stream=None):
    arr = (rl_map_desc * len(descs))(*descs)
    _check(load().rl_shoot_batch(ctx, arr, len(descs), precision, stream))


def rl_count_histogram(ctx, d_counts, win, n_values, d_hist, stream=None):
    _check(load().rl_count_histogram(ctx, d_counts, C.byref(win), n_values, d_hist, stream))


def rl_mpd(ctx, d_counts, win, n_avg, mu_ref, log_lo, log_hi, nbins, d_bins, stream=None):
    _check(load().rl_mpd(ctx, d_counts, C.byref(win), n_avg, mu_ref, log_lo, log_hi, nbins, d_bins,
                         stream))


def rl_mpd_values(ctx, d_mu, win, mu_ref, log_lo, log_hi, nbins, d_bins, stream=None):
    _check(load().rl_mpd_values(ctx, d_mu, C.byref(win), mu_ref, log_lo, log_hi, nbins, d_bins, stream))


def rl_probability_sums(ctx, d_counts, win, n_avg, mu_lim, stream=None):
    below = C.c_int64()
    above = C.c_int64()
    _check(load().rl_probability_sums(ctx, d_counts, C.byref(win), n_avg, mu_lim, C.byref(below),
                                      C.byref(above), stream))
    return below.value, above.value


def rl_mpd_moments(ctx, d_bins, n_maps, n_bins, n_pix, d_mean, d_std, stream=None):
    _check(load().rl_mpd_moments(ctx, d_bins, n_maps, n_bins, n_pix, d_mean, d_std, stream))


def rl_codec_encode(ctx, d_counts, win, d_values, values_capacity, d_packed, packed_capacity,
                    stream=None):
    nd = C.c_int64()
    bits = C.c_int32()
    _check(load().rl_codec_encode(ctx, d_counts, C.byref(win), d_values, values_capacity, d_packed,
                                  packed_capacity, C.byref(nd), C.byref(bits), stream))
    return nd.value, bits.value


def rl_codec_decode(ctx, d_packed, bits, d_values, n_distinct, win, d_counts, stream=None):
    _check(load().rl_codec_decode(ctx, d_packed, bits, d_values, n_distinct, C.byref(win), d_counts,
                                  stream))


def rl_source_kernel(ctx, profile, win, d_kernel, stream=None):
    _check(load().rl_source_kernel(ctx, C.byref(profile), C.byref(win), d_kernel, stream))


def rl_source_kernel_table(ctx, h_x, nx, h_y, ny, h_b, win, d_kernel, stream=None):
    _check(load().rl_source_kernel_table(ctx, h_x, nx, h_y, ny, h_b, C.byref(win), d_kernel, stream))


def read_profile_table(path, nx, ny):
    """A tabulated disc profile as the GERLUMPH profile files store it (Section
    3.2, the disc table): FP32 throughout, the N_x x positions, the N_y y
    positions, then the N_x N_y brightness values, read here with x fastest
    and little-endian; N_x and N_y come from the profile's metadata, not from
    this file. Returns (x, y, b) as numpy float32 arrays, b of shape
    (N_y, N_x). Positions are in the profile's physical units: scale them to
    Einstein radii before building a kernel."""
    import numpy as np
    nx, ny = int(nx), int(ny)
    if nx < 1 or ny < 1:
        raise ValueError(f"grid {nx} x {ny}: both sides must be >= 1")
    raw = np.fromfile(path, dtype="<f4")
    if raw.size != nx + ny + nx * ny:
        raise ValueError(f"{path}: {raw.size} values, a {nx} x {ny} grid needs {nx + ny + nx * ny}")
    raw = raw.astype(np.float32)
    return raw[:nx].copy(), raw[nx:nx + ny].copy(), raw[nx + ny:].reshape(ny, nx).copy()


def rl_convolve(ctx, d_counts, d_kernel, win, n_avg, d_out, stream=None):
    _check(load().rl_convolve(ctx, d_counts, d_kernel, C.byref(win), n_avg, d_out, stream))


def rl_convolve_batch(ctx, d_counts, d_kernels, win, n_avg, d_outs, stream=None):
    """d_kernels, d_outs: sequences of device pointers of equal length."""
    n = len(d_kernels)
    ks = (C.c_void_p * n)(*d_kernels)
    os_ = (C.c_void_p * len(d_outs))(*d_outs)
    _check(load().rl_convolve_batch(ctx, d_counts, ks, n, C.byref(win), n_avg, os_, stream))


def rl_autotune(ctx, cache_path=None, budget_ms=0):
    _check(load().rl_autotune(ctx, None if cache_path is None else str(cache_path).encode(), budget_ms))


def rl_get_tuning(ctx, precision, n_class) -> rl_tuning:
    t = rl_tuning()
    _check(load().rl_get_tuning(ctx, precision, n_class, C.byref(t)))
    return t


def rl_set_tuning(ctx, precision, n_class, tuning: rl_tuning):
    _check(load().rl_set_tuning(ctx, precision, n_class, C.byref(tuning)))


# ----------------------------------------------------------------------------
# torch plumbing
# ----------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def macro_of(spec) -> rl_macro:
    return rl_macro(spec.kappa, spec.gamma, spec.s)


def grid_of(spec) -> rl_raygrid:
    return rl_raygrid(spec.n1, spec.n2, spec.c1, spec.c2, spec.h1, spec.h2)


def window_of(spec) -> rl_window:
    return rl_window(spec.p1, spec.p2, spec.w1, spec.w2, spec.W1, spec.W2)


class DeviceLenses:
    """A lens field resident in HBM as FP64 structure-of-arrays tensors."""

    def __init__(self, x1, x2, m=None, device="cuda"):
        torch = _torch()
        self.x1 = torch.as_tensor(x1, dtype=torch.float64).to(device).contiguous()
        self.x2 = torch.as_tensor(x2, dtype=torch.float64).to(device).contiguous()
        self.m = None if m is None else torch.as_tensor(m, dtype=torch.float64).to(device).contiguous()
        if self.x1.shape != self.x2.shape or self.x1.dim() != 1:
            raise ValueError("lens positions must be 1-D tensors of equal length")
        if self.m is not None and self.m.shape != self.x1.shape:
            raise ValueError("masses must match the positions")

    @property
    def n(self):
        return int(self.x1.numel())

    def struct(self, device=None) -> rl_lenses:
        """The C descriptor; with `device` given, the tensors must live there."""
        if device is not None and self.n:
            torch = _torch()
            for name, t in (("x1", self.x1), ("x2", self.x2), ("m", self.m)):
                if t is not None:
                    _dev(t, torch.float64, self.n, f"lens {name}", device)
        return rl_lenses(self.x1.data_ptr() if self.n else None,
                         self.x2.data_ptr() if self.n else None,
                         None if self.m is None else self.m.data_ptr(), self.n)

    def nbytes(self):
        return self.x1.numel() * 8 * (3 if self.m is not None else 2)


def _stream_ptr(stream):
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


class Context:
    """An rl_context plus torch-tensor conveniences."""

    def __init__(self, device: int = 0):
        self.device = device
        self.handle = rl_create(device)

    def close(self):
        if self.handle:
            rl_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_map(self, spec):
        torch = _torch()
        dev = f"cuda:{self.device}"
        counts = torch.zeros((spec.p2, spec.p1), dtype=torch.int32, device=dev)
        escaped = torch.zeros(1, dtype=torch.int64, device=dev)
        return counts, escaped

    def shoot(self, lenses: DeviceLenses, spec, precision="fp32c", counts=None, escaped=None,
              row_begin=0, row_end=None, stream=None):
        if counts is None or escaped is None:
            counts, escaped = self.new_map(spec)
        _check_map_tensors(counts, escaped, spec, self.device)
        rl_shoot(self.handle, lenses.struct(self.device), macro_of(spec), grid_of(spec), window_of(spec),
                 PRECISIONS[precision], row_begin, spec.n2 if row_end is None else row_end,
                 counts.data_ptr(), escaped.data_ptr(), _stream_ptr(stream))
        return counts, escaped

    def shoot_noalloc(self, lenses: DeviceLenses, spec, precision, counts, escaped, row_begin=0,
                      row_end=None, stream=None):
        """rl_shoot_noalloc into caller-made (zeroed) counts and escaped tensors."""
        _check_map_tensors(counts, escaped, spec, self.device)
        rl_shoot_noalloc(self.handle, lenses.struct(self.device), macro_of(spec), grid_of(spec),
                         window_of(spec), PRECISIONS[precision], row_begin,
                         spec.n2 if row_end is None else row_end, counts.data_ptr(),
                         escaped.data_ptr(), _stream_ptr(stream))
        return counts, escaped

    def ray_positions(self, lenses: DeviceLenses, spec, precision="fp32c", row_begin=0,
                      row_end=None, stream=None):
        torch = _torch()
        row_end = spec.n2 if row_end is None else row_end
        rows = row_end - row_begin
        dev = f"cuda:{self.device}"
        y1 = torch.empty((rows, spec.n1), dtype=torch.float64, device=dev)
        y2 = torch.empty((rows, spec.n1), dtype=torch.float64, device=dev)
        rl_ray_positions(self.handle, lenses.struct(self.device), macro_of(spec), grid_of(spec),
                         PRECISIONS[precision], row_begin, row_end, y1.data_ptr(), y2.data_ptr(),
                         _stream_ptr(stream))
        return y1, y2

    def bin_positions(self, y1, y2, spec, counts=None, escaped=None, stream=None):
        torch = _torch()
        if counts is None or escaped is None:
            counts, escaped = self.new_map(spec)
        _check_map_tensors(counts, escaped, spec, self.device)
        y1 = y1.contiguous()
        y2 = y2.contiguous()
        _dev(y1, torch.float64, y1.numel(), "y1", self.device)
        _dev(y2, torch.float64, y1.numel(), "y2", self.device)
        rl_bin_positions(self.handle, y1.data_ptr(), y2.data_ptr(), y1.numel(), window_of(spec),
                         counts.data_ptr(), escaped.data_ptr(), _stream_ptr(stream))
        return counts, escaped

    def normalise(self, counts, spec, n_avg=None, mu=None, stream=None):
        torch = _torch()
        if n_avg is None:
            n_avg = rl_n_avg(grid_of(spec), window_of(spec))
        if mu is None:
            mu = torch.empty((spec.p2, spec.p1), dtype=torch.float32, device=counts.device)
        _dev(counts, torch.int32, spec.p1 * spec.p2, "counts", self.device)
        _dev(mu, torch.float32, spec.p1 * spec.p2, "mu", self.device)
        rl_normalise(self.handle, counts.data_ptr(), window_of(spec), n_avg, mu.data_ptr(),
                     _stream_ptr(stream))
        return mu

    def stats(self, counts, escaped, spec, stream=None):
        _check_map_tensors(counts, escaped, spec, self.device)
        st = rl_stats_get(self.handle, counts.data_ptr(), escaped.data_ptr(), macro_of(spec),
                          grid_of(spec), window_of(spec), _stream_ptr(stream))
        return {f: getattr(st, f) for f, _ in rl_stats._fields_}

    def shoot_batch(self, items, precision="fp32c", stream=None):
        """items: sequence of (DeviceLenses, spec, counts, escaped[, row_begin, row_end])."""
        descs = []
        for it in items:
            lenses, spec, counts, escaped = it[:4]
            rb = it[4] if len(it) > 4 else 0
            re = it[5] if len(it) > 5 else spec.n2
            _check_map_tensors(counts, escaped, spec, self.device)
            descs.append(rl_map_desc(lenses.struct(self.device), macro_of(spec), grid_of(spec), window_of(spec),
                                     rb, re, counts.data_ptr(), escaped.data_ptr()))
        rl_shoot_batch(self.handle, descs, PRECISIONS[precision], _stream_ptr(stream))

    # ---- magnification probability distributions ----------------------------
    def count_histogram(self, counts, spec, n_values, hist=None, stream=None):
        torch = _torch()
        _check_counts(counts, spec, self.device)
        if hist is None:
            hist = torch.zeros(int(n_values), dtype=torch.int64, device=counts.device)
        _dev(hist, torch.int64, int(n_values), "hist", self.device)
        rl_count_histogram(self.handle, counts.data_ptr(), window_of(spec), int(n_values),
                           hist.data_ptr(), _stream_ptr(stream))
        return hist

    def mpd(self, counts, spec, mu_ref, log_lo, log_hi, nbins, n_avg=None, bins=None, stream=None):
        """[underflow, nbins bins of log10(mu / mu_ref) over [log_lo, log_hi), overflow]."""
        torch = _torch()
        _check_counts(counts, spec, self.device)
        if n_avg is None:
            n_avg = rl_n_avg(grid_of(spec), window_of(spec))
        if bins is None:
            bins = torch.zeros(int(nbins) + 2, dtype=torch.int64, device=counts.device)
        _dev(bins, torch.int64, int(nbins) + 2, "bins", self.device)
        rl_mpd(self.handle, counts.data_ptr(), window_of(spec), n_avg, mu_ref, log_lo, log_hi,
               int(nbins), bins.data_ptr(), _stream_ptr(stream))
        return bins

    def mpd_values(self, mu, spec, mu_ref, log_lo, log_hi, nbins, bins=None, stream=None):
        """The binned MPD of a map of real magnifications (e.g. a finite-source
        map from convolve): [underflow, nbins bins, overflow]."""
        torch = _torch()
        _dev(mu, torch.float64, spec.p1 * spec.p2, "mu", self.device)
        if bins is None:
            bins = torch.zeros(int(nbins) + 2, dtype=torch.int64, device=mu.device)
        _dev(bins, torch.int64, int(nbins) + 2, "bins", self.device)
        rl_mpd_values(self.handle, mu.data_ptr(), window_of(spec), mu_ref, log_lo, log_hi, int(nbins),
                      bins.data_ptr(), _stream_ptr(stream))
        return bins

    def probability_sums(self, counts, spec, mu_lim, n_avg=None, stream=None):
        _check_counts(counts, spec, self.device)
        if n_avg is None:
            n_avg = rl_n_avg(grid_of(spec), window_of(spec))
        return rl_probability_sums(self.handle, counts.data_ptr(), window_of(spec), n_avg, mu_lim,
                                   _stream_ptr(stream))

    def mpd_moments(self, bins, n_pix, stream=None):
        """bins: int64 tensor (n_maps, n_bins). Returns (mean, std) float64 tensors."""
        torch = _torch()
        bins = bins.contiguous()
        if bins.dim() != 2:
            raise ValueError("bins must be a 2-D int64 tensor")
        _dev(bins, torch.int64, bins.numel(), "bins", self.device)
        mean = torch.empty(bins.shape[1], dtype=torch.float64, device=bins.device)
        std = torch.empty_like(mean)
        rl_mpd_moments(self.handle, bins.data_ptr(), bins.shape[0], bins.shape[1], int(n_pix),
                       mean.data_ptr(), std.data_ptr(), _stream_ptr(stream))
        return mean, std

    # ---- indexed maps ----------------------------------------------------------
    def encode(self, counts, spec, stream=None):
        """Returns (values int32[n_distinct], bits, packed uint32 words) on the device."""
        torch = _torch()
        _check_counts(counts, spec, self.device)
        nd, bits = rl_codec_encode(self.handle, counts.data_ptr(), window_of(spec), None, 0, None, 0,
                                   _stream_ptr(stream))
        words = (spec.p1 * spec.p2 * bits + 31) // 32
        values = torch.empty(nd, dtype=torch.int32, device=counts.device)
        packed = torch.empty(words, dtype=torch.int32, device=counts.device)   # 32-bit words
        nd2, bits2 = rl_codec_encode(self.handle, counts.data_ptr(), window_of(spec), values.data_ptr(),
                                     nd, packed.data_ptr(), words, _stream_ptr(stream))
        assert (nd2, bits2) == (nd, bits)
        return values, bits, packed

    def decode(self, packed, bits, values, spec, counts=None, stream=None):
        torch = _torch()
        if counts is None:
            counts = torch.empty((spec.p2, spec.p1), dtype=torch.int32, device=packed.device)
        words = (spec.p1 * spec.p2 * int(bits) + 31) // 32
        if packed.dtype not in (torch.int32, torch.uint32):
            raise ValueError("packed must hold 32-bit words")
        _dev(packed, packed.dtype, words, "packed", self.device, exact=False)
        _dev(values, torch.int32, values.numel(), "values", self.device)
        _dev(counts, torch.int32, spec.p1 * spec.p2, "counts", self.device)
        rl_codec_decode(self.handle, packed.data_ptr(), int(bits), values.data_ptr(), values.numel(),
                        window_of(spec), counts.data_ptr(), _stream_ptr(stream))
        return counts

    # ---- finite sources ---------------------------------------------------------
    def source_kernel(self, spec, shape, radius, hole=0.0, kernel=None, stream=None):
        torch = _torch()
        if kernel is None:
            kernel = torch.empty((spec.p2, spec.p1), dtype=torch.float64, device=f"cuda:{self.device}")
        _dev(kernel, torch.float64, spec.p1 * spec.p2, "kernel", self.device)
        rl_source_kernel(self.handle, rl_profile(PROFILES[shape], radius, hole), window_of(spec),
                         kernel.data_ptr(), _stream_ptr(stream))
        return kernel

    def source_kernel_table(self, spec, x, y, b, kernel=None, stream=None):
        """Kernel of a tabulated profile: x[N_x], y[N_y] positions in Einstein
        radii around the source centre, b[N_y, N_x] brightness (x fastest),
        host arrays converted to contiguous FP32."""
        import numpy as np
        torch = _torch()
        x = np.ascontiguousarray(x, dtype=np.float32).ravel()
        y = np.ascontiguousarray(y, dtype=np.float32).ravel()
        b = np.ascontiguousarray(b, dtype=np.float32).ravel()
        if b.size != x.size * y.size:
            raise ValueError(f"brightness holds {b.size} values, not {y.size} x {x.size}")
        if kernel is None:
            kernel = torch.empty((spec.p2, spec.p1), dtype=torch.float64, device=f"cuda:{self.device}")
        _dev(kernel, torch.float64, spec.p1 * spec.p2, "kernel", self.device)
        rl_source_kernel_table(self.handle, x.ctypes.data, x.size, y.ctypes.data, y.size, b.ctypes.data,
                               window_of(spec), kernel.data_ptr(), _stream_ptr(stream))
        return kernel

    def convolve(self, counts, kernel, spec, n_avg=1.0, out=None, stream=None):
        torch = _torch()
        _check_counts(counts, spec, self.device)
        _dev(kernel, torch.float64, spec.p1 * spec.p2, "kernel", self.device)
        if out is None:
            out = torch.empty((spec.p2, spec.p1), dtype=torch.float64, device=counts.device)
        _dev(out, torch.float64, spec.p1 * spec.p2, "out", self.device)
        rl_convolve(self.handle, counts.data_ptr(), kernel.data_ptr(), window_of(spec), n_avg,
                    out.data_ptr(), _stream_ptr(stream))
        return out

    def convolve_batch(self, counts, kernels, spec, n_avg=1.0, outs=None, stream=None):
        """The map convolved with each of `kernels` (rl_convolve_batch)."""
        torch = _torch()
        _check_counts(counts, spec, self.device)
        kernels = list(kernels)
        if not kernels:
            raise ValueError("kernels is empty")
        for q, k in enumerate(kernels):
            _dev(k, torch.float64, spec.p1 * spec.p2, f"kernels[{q}]", self.device)
        if outs is None:
            outs = [torch.empty((spec.p2, spec.p1), dtype=torch.float64, device=counts.device)
                    for _ in kernels]
        outs = list(outs)
        if len(outs) != len(kernels):
            raise ValueError("outs and kernels differ in length")
        for q, o in enumerate(outs):
            _dev(o, torch.float64, spec.p1 * spec.p2, f"outs[{q}]", self.device)
        rl_convolve_batch(self.handle, counts.data_ptr(), [k.data_ptr() for k in kernels], window_of(spec),
                          n_avg, [o.data_ptr() for o in outs], _stream_ptr(stream))
        return outs

    def autotune(self, cache_path=None, budget_ms=0):
        rl_autotune(self.handle, cache_path, budget_ms)

    def get_tuning(self, precision, n_class):
        t = rl_get_tuning(self.handle, PRECISIONS[precision], n_class)
        return {f: getattr(t, f) for f, _ in rl_tuning._fields_}

    def set_tuning(self, precision, n_class, **kw):
        cur = self.get_tuning(precision, n_class)
        cur.update(kw)
        rl_set_tuning(self.handle, PRECISIONS[precision], n_class, rl_tuning(**cur))


def _dev(t, dtype, numel, name, device, exact=True):
    """A contiguous tensor of `dtype` on HIP device `device` with `numel`
    elements (at least `numel` if not exact): anything else is refused before
    its pointer reaches the library."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if not t.is_cuda or (t.device.index if t.device.index is not None else 0) != device:
        raise ValueError(f"{name} must live on cuda:{device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if (t.numel() != numel) if exact else (t.numel() < numel):
        raise ValueError(f"{name} must hold {'' if exact else 'at least '}{numel} elements")
    return t


def _check_map_tensors(counts, escaped, spec, device=0):
    torch = _torch()
    _dev(counts, torch.int32, spec.p1 * spec.p2, "counts", device)
    _dev(escaped, torch.int64, 1, "escaped", device, exact=False)


def _check_counts(counts, spec, device=0):
    _dev(counts, _torch().int32, spec.p1 * spec.p2, "counts", device)


def n_class(n: int) -> int:
    """Lens-count class: 0 (n < 1000), 1 (n < 10000), 2."""
    return 0 if n < 1000 else (1 if n < 10000 else 2)


TUNING_CLASSES = 6


def tuning_class(n: int, masses: bool) -> int:
    """Tuning class of a lens field: its lens-count class, plus 3 with masses."""
    return n_class(n) + (3 if masses else 0)


def spec_tuning_class(spec) -> int:
    return tuning_class(spec.n_lens, spec.masses != "unit")

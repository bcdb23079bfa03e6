"""The C-ABI library on the CPU: it loads, exports every declared symbol, and
rejects invalid arguments before any HIP call (no compute happens here)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_1406_0559_amd import raylens as rl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "raylens.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rl_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = rl.load()
    syms = declared_symbols()
    assert len(syms) >= 13
    for s in syms:
        assert hasattr(lib, s), f"{s} declared in include/raylens.h but not exported"


def test_version_and_context_lifecycle_without_device():
    assert "raylens" in rl.rl_version()
    ctx = rl.rl_create(0)     # makes no HIP call
    assert ctx
    rl.rl_destroy(ctx)
    rl.rl_destroy(None)


def test_invalid_arguments_are_rejected_on_the_host():
    lib = rl.load()
    ctx = rl.rl_create(0)
    try:
        g = rl.rl_raygrid(64, 64, 0.0, 0.0, 1.0, 1.0)
        w = rl.rl_window(16, 16, 0.0, 0.0, 2.0, 2.0)
        m = rl.rl_macro(0.4, 0.3, 0.0)
        L = rl.rl_lenses(None, None, None, 0)
        fake = C.c_void_p(0x1000)   # never dereferenced: validation fails first
        cases = [
            ("n1 = 0", dict(g=rl.rl_raygrid(0, 64, 0.0, 0.0, 1.0, 1.0))),
            ("2^51 rays", dict(g=rl.rl_raygrid(1 << 26, 1 << 25, 0.0, 0.0, 1.0, 1.0))),
            ("2^26 + 1 rays along x1", dict(g=rl.rl_raygrid((1 << 26) + 1, 2, 0.0, 0.0, 1.0, 1.0))),
            ("negative half-width", dict(g=rl.rl_raygrid(64, 64, 0.0, 0.0, -1.0, 1.0))),
            ("nan half-width", dict(g=rl.rl_raygrid(64, 64, 0.0, 0.0, math.nan, 1.0))),
            ("p2 = 0", dict(w=rl.rl_window(16, 0, 0.0, 0.0, 2.0, 2.0))),
            ("zero width", dict(w=rl.rl_window(16, 16, 0.0, 0.0, 0.0, 2.0))),
            ("inf kappa", dict(m=rl.rl_macro(math.inf, 0.3, 0.0))),
            ("nan gamma", dict(m=rl.rl_macro(0.4, math.nan, 0.0))),
            ("negative lens count", dict(L=rl.rl_lenses(None, None, None, -1))),
            ("lenses without positions", dict(L=rl.rl_lenses(None, None, None, 5))),
            ("rows reversed", dict(rb=10, re=5)),
            ("rows past the grid", dict(rb=0, re=65)),
            ("bad precision", dict(prec=7)),
            ("null counts", dict(counts=None)),
        ]
        for fn in (lib.rl_shoot, lib.rl_shoot_noalloc):
            for label, kw in cases:
                st = fn(ctx, C.byref(kw.get("L", L)), C.byref(kw.get("m", m)),
                        C.byref(kw.get("g", g)), C.byref(kw.get("w", w)),
                        kw.get("prec", rl.RL_FP32_COMP), kw.get("rb", 0), kw.get("re", 64),
                        kw.get("counts", fake), fake, None)
                assert st == rl.RL_E_INVALID, label
                assert rl.rl_last_error(), label
        # the no-allocation entry point's lens limit, refused before any HIP call
        big = rl.rl_lenses(fake, fake, None, rl.RL_NOALLOC_MAX_LENSES + 1)
        assert lib.rl_shoot_noalloc(ctx, C.byref(big), C.byref(m), C.byref(g), C.byref(w), 0, 0,
                                    64, fake, fake, None) == rl.RL_E_INVALID
        assert "at most 131072 lenses" in rl.rl_last_error()
        assert lib.rl_shoot_noalloc(None, C.byref(L), C.byref(m), C.byref(g), C.byref(w), 0, 0,
                                    64, fake, fake, None) == rl.RL_E_INVALID
        assert lib.rl_shoot(None, C.byref(L), C.byref(m), C.byref(g), C.byref(w), 0, 0, 64, fake,
                            fake, None) == rl.RL_E_INVALID
        assert lib.rl_normalise(ctx, fake, C.byref(w), 0.0, fake, None) == rl.RL_E_INVALID
        assert lib.rl_normalise(ctx, fake, C.byref(w), math.nan, fake, None) == rl.RL_E_INVALID
        assert lib.rl_bin_positions(ctx, fake, fake, -1, C.byref(w), fake, fake, None) == rl.RL_E_INVALID
        assert lib.rl_bin_positions(ctx, None, fake, 3, C.byref(w), fake, fake, None) == rl.RL_E_INVALID
        assert lib.rl_ray_positions(ctx, C.byref(L), C.byref(m), C.byref(g), 0, 3, 2, fake, fake,
                                    None) == rl.RL_E_INVALID
        assert lib.rl_shoot_batch(ctx, None, 2, 0, None) == rl.RL_E_INVALID
        bad = rl.rl_map_desc(L, m, rl.rl_raygrid(0, 1, 0.0, 0.0, 1.0, 1.0), w, 0, 1, fake.value,
                             fake.value)
        assert lib.rl_shoot_batch(ctx, C.byref(bad), 1, 0, None) == rl.RL_E_INVALID
        assert "map 0" in rl.rl_last_error()
        assert lib.rl_stats_get(ctx, fake, fake, C.byref(m), C.byref(g), C.byref(w), None,
                                None) == rl.RL_E_INVALID
    finally:
        rl.rl_destroy(ctx)


def test_empty_work_is_a_no_op():
    """Zero rows and zero positions return before touching a device."""
    lib = rl.load()
    ctx = rl.rl_create(0)
    try:
        g = rl.rl_raygrid(64, 64, 0.0, 0.0, 1.0, 1.0)
        w = rl.rl_window(16, 16, 0.0, 0.0, 2.0, 2.0)
        m = rl.rl_macro(0.4, 0.3, 0.0)
        L = rl.rl_lenses(None, None, None, 0)
        fake = C.c_void_p(0x1000)
        assert lib.rl_shoot(ctx, C.byref(L), C.byref(m), C.byref(g), C.byref(w), 0, 5, 5, fake,
                            fake, None) == rl.RL_OK
        assert lib.rl_bin_positions(ctx, None, None, 0, C.byref(w), fake, fake, None) == rl.RL_OK
        assert lib.rl_shoot_batch(ctx, None, 0, 0, None) == rl.RL_OK
    finally:
        rl.rl_destroy(ctx)


def test_n_avg_matches_the_oracle_bit_for_bit():
    for (n1, n2, h1, h2, p1, p2, W1, W2) in [(1024, 1024, 8.0, 2.67, 256, 256, 4.0, 4.0),
                                             (30000, 30000, 65.0, 14.2, 4096, 4096, 25.0, 25.0),
                                             (7, 3, 0.3, 1.9, 5, 11, 0.7, 3.3)]:
        a = rl.rl_n_avg(rl.rl_raygrid(n1, n2, 0.0, 0.0, h1, h2), rl.rl_window(p1, p2, 0.0, 0.0, W1, W2))
        b = oracle.n_avg(n1, n2, h1, h2, p1, p2, W1, W2)
        assert a == b


def test_tuning_table_validation():
    ctx = rl.rl_create(0)
    try:
        t = rl.rl_get_tuning(ctx, rl.RL_FP32_COMP, 1)
        assert t.rays_x * t.rays_y in (16, 32)
        for bad in [dict(rays_x=3), dict(lens_tile=100), dict(lens_tile=4096), dict(waves=3),
                    dict(submap=3)]:
            cur = {f: getattr(t, f) for f, _ in rl.rl_tuning._fields_}
            cur.update(bad)
            with pytest.raises(rl.RaylensError):
                rl.rl_set_tuning(ctx, rl.RL_FP32_COMP, 1, rl.rl_tuning(**cur))
        ok = rl.rl_tuning(2, 8, 512, 2, 0)
        rl.rl_set_tuning(ctx, rl.RL_FP32_COMP, 2, ok)
        back = rl.rl_get_tuning(ctx, rl.RL_FP32_COMP, 2)
        assert (back.rays_x, back.rays_y, back.lens_tile, back.waves,
                back.submap) == (2, 8, 512, 2, 0)
        with pytest.raises(rl.RaylensError):   # FP64 path keeps 4 x 4 rays per lane
            rl.rl_set_tuning(ctx, rl.RL_FP64_PLAIN, 0, ok)
        for cls in (-1, rl.TUNING_CLASSES):
            with pytest.raises(rl.RaylensError):
                rl.rl_get_tuning(ctx, rl.RL_FP32_COMP, cls)
        # classes 3-5 (fields with masses) are separate entries
        rl.rl_set_tuning(ctx, rl.RL_FP32_COMP, 5, rl.rl_tuning(4, 8, 256, 4, 1))
        assert rl.rl_get_tuning(ctx, rl.RL_FP32_COMP, 2).rays_y == 8
        assert (rl.rl_get_tuning(ctx, rl.RL_FP32_COMP, 5).rays_x, rl.rl_get_tuning(ctx, rl.RL_FP32_COMP, 5).rays_y) == (4, 8)
        assert rl.tuning_class(999, False) == 0 and rl.tuning_class(10000, True) == 5
    finally:
        rl.rl_destroy(ctx)


def test_autotune_validates_on_the_host(tmp_path):
    lib = rl.load()
    assert lib.rl_autotune(None, None, 0) == rl.RL_E_INVALID
    ctx = rl.rl_create(0)
    try:
        assert lib.rl_autotune(ctx, None, -1) == rl.RL_E_INVALID
        assert "budget" in rl.rl_last_error()
    finally:
        rl.rl_destroy(ctx)


def test_mpd_of_real_maps_validates_on_the_host():
    lib = rl.load()
    ctx = rl.rl_create(0)
    try:
        w = rl.rl_window(64, 64, 0.0, 0.0, 2.0, 2.0)
        fake = C.c_void_p(0x1000)
        bad = [(None, w, 1.0, -1.0, 1.0, 10, fake), (fake, w, 0.0, -1.0, 1.0, 10, fake),
               (fake, w, math.inf, -1.0, 1.0, 10, fake), (fake, w, 1.0, 1.0, -1.0, 10, fake),
               (fake, w, 1.0, -1.0, math.nan, 10, fake), (fake, w, 1.0, -1.0, 1.0, 0, fake),
               (fake, w, 1.0, -1.0, 1.0, 4097, fake), (fake, w, 1.0, -1.0, 1.0, 10, None),
               (fake, rl.rl_window(0, 64, 0.0, 0.0, 2.0, 2.0), 1.0, -1.0, 1.0, 10, fake)]
        for mu, ww, ref, lo, hi, nb, bins in bad:
            assert lib.rl_mpd_values(ctx, mu, C.byref(ww), ref, lo, hi, nb, bins, None) == rl.RL_E_INVALID
    finally:
        rl.rl_destroy(ctx)


def test_binding_constants_match_the_header():
    text = open(os.path.join(ROOT, "include", "raylens.h")).read()
    for name in ("RL_NOALLOC_MAX_LENSES", "RL_MAX_CONVOLVE_BATCH", "RL_MAX_TABLE_AXIS"):
        m = re.search(r"^#define\s+" + name + r"\s+(\d+)", text, flags=re.M)
        assert m, name
        assert int(m.group(1)) == getattr(rl, name), name


def test_header_documents_every_entry_point():
    """Each declaration in the public header is preceded by a comment."""
    text = open(os.path.join(ROOT, "include", "raylens.h")).read()
    for sym in declared_symbols():
        decl = re.search(r"^(?:rl_status|const char\*|void)\s+" + sym + r"\(", text, flags=re.M)
        assert decl, f"{sym}: declaration not found"
        before = text[:decl.start()].rstrip()
        assert "*/" in before[-400:], f"{sym} has no comment"


def test_one_hip_runtime_per_process():
    """Loading the library before torch must not leave two HIP runtimes in the
    process (torch's bundled one and the system one): the binding loads torch
    first so the library binds to torch's runtime."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1406_0559_amd import raylens as rl\n"
            "rl.load()\n"
            "import torch\n"
            "paths = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(paths), sorted(paths))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.split()[0] == "1", out.stdout


def test_mpd_entry_points_validate_on_the_host():
    lib = rl.load()
    ctx = rl.rl_create(0)
    try:
        w = rl.rl_window(16, 16, 0.0, 0.0, 2.0, 2.0)
        fake = C.c_void_p(0x1000)
        lo = C.c_int64()
        hi = C.c_int64()
        assert lib.rl_count_histogram(ctx, fake, C.byref(w), 0, fake, None) == rl.RL_E_INVALID
        assert lib.rl_count_histogram(ctx, None, C.byref(w), 10, fake, None) == rl.RL_E_INVALID
        bad = [(0.0, 1.0, -1.0, 1.0, 10), (1.0, 0.0, -1.0, 1.0, 10), (1.0, 1.0, 1.0, -1.0, 10),
               (1.0, 1.0, -1.0, 1.0, 0), (1.0, 1.0, -1.0, 1.0, 5000), (math.nan, 1.0, -1.0, 1.0, 10),
               (1.0, 1.0, -math.inf, 1.0, 10)]
        for n_avg, mu_ref, a, b, nb in bad:
            assert lib.rl_mpd(ctx, fake, C.byref(w), n_avg, mu_ref, a, b, nb, fake, None) == rl.RL_E_INVALID
        assert lib.rl_probability_sums(ctx, fake, C.byref(w), 1.0, math.nan, C.byref(lo), C.byref(hi),
                                       None) == rl.RL_E_INVALID
        assert lib.rl_probability_sums(ctx, fake, C.byref(w), -1.0, 1.0, C.byref(lo), C.byref(hi),
                                       None) == rl.RL_E_INVALID
        assert lib.rl_mpd_moments(ctx, fake, 0, 10, 100, fake, fake, None) == rl.RL_E_INVALID
        assert lib.rl_mpd_moments(ctx, fake, 3, 10, 0, fake, fake, None) == rl.RL_E_INVALID
    finally:
        rl.rl_destroy(ctx)


def test_codec_entry_points_validate_on_the_host():
    lib = rl.load()
    ctx = rl.rl_create(0)
    try:
        w = rl.rl_window(16, 16, 0.0, 0.0, 2.0, 2.0)
        fake = C.c_void_p(0x1000)
        nd = C.c_int64()
        bits = C.c_int32()
        assert lib.rl_codec_encode(ctx, None, C.byref(w), fake, 1, fake, 1, C.byref(nd), C.byref(bits),
                                   None) == rl.RL_E_INVALID
        assert lib.rl_codec_encode(ctx, fake, C.byref(w), fake, 0, fake, 1, C.byref(nd), C.byref(bits),
                                   None) == rl.RL_E_INVALID
        assert lib.rl_codec_encode(ctx, fake, C.byref(w), fake, 1, fake, 1, None, C.byref(bits),
                                   None) == rl.RL_E_INVALID
        for b in (0, 33):
            assert lib.rl_codec_decode(ctx, fake, b, fake, 4, C.byref(w), fake, None) == rl.RL_E_INVALID
        assert lib.rl_codec_decode(ctx, fake, 4, fake, 0, C.byref(w), fake, None) == rl.RL_E_INVALID
        assert lib.rl_codec_decode(ctx, None, 4, fake, 4, C.byref(w), fake, None) == rl.RL_E_INVALID
    finally:
        rl.rl_destroy(ctx)


def test_convolution_entry_points_validate_on_the_host():
    lib = rl.load()
    ctx = rl.rl_create(0)
    try:
        w = rl.rl_window(64, 64, 0.0, 0.0, 2.0, 2.0)
        fake = C.c_void_p(0x1000)
        for prof in (rl.rl_profile(5, 0.1, 0.0), rl.rl_profile(0, -0.1, 0.0), rl.rl_profile(0, 0.1, -1.0),
                     rl.rl_profile(1, math.nan, 0.0), rl.rl_profile(0, 5.0, 0.0)):
            assert lib.rl_source_kernel(ctx, C.byref(prof), C.byref(w), fake, None) == rl.RL_E_INVALID
        # sides must be products of 2, 3 and 5 in [2, 10240]
        for ww in (rl.rl_window(49, 64, 0.0, 0.0, 2.0, 2.0), rl.rl_window(64, 7, 0.0, 0.0, 2.0, 2.0),
                   rl.rl_window(10368, 2, 0.0, 0.0, 2.0, 2.0), rl.rl_window(1, 64, 0.0, 0.0, 2.0, 2.0),
                   rl.rl_window(2 * 5003, 64, 0.0, 0.0, 2.0, 2.0)):
            assert lib.rl_convolve(ctx, fake, fake, C.byref(ww), 1.0, fake, None) == rl.RL_E_INVALID
        assert lib.rl_convolve(ctx, fake, fake, C.byref(w), 0.0, fake, None) == rl.RL_E_INVALID
        assert lib.rl_convolve(ctx, fake, None, C.byref(w), 1.0, fake, None) == rl.RL_E_INVALID
        # the batch form: counts, sizes, NULL arrays or entries, shared outputs
        V = C.c_void_p
        ks = (V * 3)(0x1000, 0x2000, 0x3000)
        outs = (V * 3)(0x4000, 0x5000, 0x6000)
        same = (V * 3)(0x4000, 0x5000, 0x4000)
        holes = (V * 3)(0x1000, None, 0x3000)
        bad = rl.rl_window(49, 64, 0.0, 0.0, 2.0, 2.0)
        for args in ((fake, ks, 0, w, 1.0, outs), (fake, ks, rl.RL_MAX_CONVOLVE_BATCH + 1, w, 1.0, outs),
                     (fake, None, 3, w, 1.0, outs), (fake, ks, 3, w, 1.0, None), (fake, holes, 3, w, 1.0, outs),
                     (fake, ks, 3, w, 1.0, holes), (fake, ks, 3, w, 1.0, same), (None, ks, 3, w, 1.0, outs),
                     (fake, ks, 3, w, 0.0, outs), (fake, ks, 3, bad, 1.0, outs)):
            c, k, n, ww, na, o = args
            assert lib.rl_convolve_batch(ctx, c, k, n, C.byref(ww), na, o, None) == rl.RL_E_INVALID, args
        assert lib.rl_convolve_batch(ctx, fake, ks, 3, C.byref(w), 1.0, same, None) == rl.RL_E_INVALID
        assert "outputs 0 and 2" in rl.rl_last_error()
        onto_kernel = (V * 3)(0x4000, 0x3000, 0x6000)     # output 1 is kernel 2
        assert lib.rl_convolve_batch(ctx, fake, ks, 3, C.byref(w), 1.0, onto_kernel, None) == rl.RL_E_INVALID
        assert "output 1 is kernel 2" in rl.rl_last_error()
        onto_map = (V * 3)(0x4000, 0x1000, 0x6000)        # output 1 is the map (fake)
        assert lib.rl_convolve_batch(ctx, fake, ks, 3, C.byref(w), 1.0, onto_map, None) == rl.RL_E_INVALID
        # tabulated profiles: axis sizes, positions, brightness, box size
        F = C.c_float
        xs = (F * 3)(-0.02, 0.0, 0.02)
        b9 = (F * 9)(*([1.0] * 9))
        table = lambda x, nx, y, ny, b, ww=w: lib.rl_source_kernel_table(ctx, x, nx, y, ny, b, C.byref(ww),
                                                                         fake, None)
        assert table(xs, 0, xs, 3, b9) == rl.RL_E_INVALID
        assert table(xs, 3, xs, rl.RL_MAX_TABLE_AXIS + 1, b9) == rl.RL_E_INVALID
        assert table(None, 3, xs, 3, b9) == rl.RL_E_INVALID
        assert table(xs, 3, xs, 3, None) == rl.RL_E_INVALID
        for bad_x in ((F * 3)(-0.02, math.nan, 0.02), (F * 3)(-0.02, 0.0, 1.5)):
            assert table(bad_x, 3, xs, 3, b9) == rl.RL_E_INVALID, list(bad_x)
        assert "larger than the map" in rl.rl_last_error()
        for bad_b in ((F * 9)(*([1.0] * 8 + [-1.0])), (F * 9)(*([1.0] * 8 + [math.inf])), (F * 9)(*([0.0] * 9))):
            assert table(xs, 3, xs, 3, bad_b) == rl.RL_E_INVALID, list(bad_b)
        assert "every brightness is 0" in rl.rl_last_error()
    finally:
        rl.rl_destroy(ctx)


def test_binding_refuses_host_tensors_before_any_library_call():
    """Host (CPU) tensors, wrong dtypes and short outputs are refused by the
    binding: their pointers never reach a kernel."""
    import torch
    from paper_1406_0559_amd import inputs
    ctx = rl.Context(0)
    try:
        spec = inputs.MapSpec(name="t", kappa=0.4, gamma=0.3, s=0.0, n1=8, n2=8, h1=1.0, h2=1.0,
                              p1=4, p2=4, W1=2.0, W2=2.0)
        c = torch.zeros((4, 4), dtype=torch.int32)
        e = torch.zeros(1, dtype=torch.int64)
        L = rl.DeviceLenses([0.1], [0.2], device="cpu")
        calls = [
            lambda: ctx.shoot(L, spec, "fp32c", c, e),
            lambda: ctx.normalise(c, spec),
            lambda: ctx.stats(c, e, spec),
            lambda: ctx.count_histogram(c, spec, 8),
            lambda: ctx.mpd(c, spec, 1.0, -1.0, 1.0, 10),
            lambda: ctx.probability_sums(c, spec, 1.0),
            lambda: ctx.encode(c, spec),
            lambda: ctx.convolve(c, torch.zeros((4, 4), dtype=torch.float64), spec),
            lambda: ctx.bin_positions(torch.zeros(3, dtype=torch.float64),
                                      torch.zeros(3, dtype=torch.float64), spec, c, e),
            lambda: ctx.mpd_moments(torch.zeros((2, 3), dtype=torch.int64), 16),
            lambda: ctx.decode(torch.zeros(4, dtype=torch.int32), 4,
                               torch.zeros(2, dtype=torch.int32), spec),
        ]
        for call in calls:
            with pytest.raises(ValueError):
                call()
    finally:
        ctx.close()


def test_profile_table_reader(tmp_path):
    """read_profile_table: FP32 x, y and brightness (x fastest), the grid's
    sides given by the caller; a size that does not match is refused."""
    import numpy as np
    x = np.array([-0.5, 0.0, 0.5], np.float32)
    y = np.array([-1.0, 1.0], np.float32)
    b = np.arange(6, dtype=np.float32).reshape(2, 3)
    f = tmp_path / "profile.bin"
    f.write_bytes(x.astype("<f4").tobytes() + y.astype("<f4").tobytes() + b.astype("<f4").tobytes())
    gx, gy, gb = rl.read_profile_table(f, 3, 2)
    assert np.array_equal(gx, x) and np.array_equal(gy, y) and np.array_equal(gb, b)
    for nx, ny in ((4, 2), (3, 3), (0, 2)):
        with pytest.raises(ValueError):
            rl.read_profile_table(f, nx, ny)

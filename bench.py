#!/usr/bin/env python3
"""Benchmark of the ray-shooting hot path on one MI355X.

Workload (one "step" = one whole magnification map): the GERLUMPH-like map
of 30000 x 30000 rays through 2624 unit point lenses (kappa = 0.41, s = 0,
gamma = 0.38) onto a 4096^2 map of 25 x 25 Einstein radii, with synthetic
seeded lens positions standing in for GERLUMPH's. A step runs the FP32-
compensated shooter, the normalisation to magnification and the statistics
reduction, with the lens field already resident in HBM.

Printed: one JSON line with ray-lens evaluations per second (the headline),
the FP64-plain rate on the same map and the speed-up, maps/hour and per-map
latency percentiles, the batched 64-map workload's maps/hour, a roofline entry
for the dominant kernel (timed with events on the stream it runs on) and the
oracle's rate on a bounded sample on the host cores.
"""
import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3          # MI355X FP32 vector peak (AMD published)
FP64_PEAK_TFLOPS = 78.6           # MI355X FP64 vector peak (AMD published)
FLOPS_PER_EVAL = 10               # ~10 flops per lens per ray (Section 2.1)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-map batched workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target oracle time for the CPU baseline sample")
    ap.add_argument("--workload", default="gerlumph-30000sq-2624")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-scale", type=float, default=0.25,
                    help="map-size scale of the served requests (1.0 = 1024^2-4096^2 maps)")
    ap.add_argument("--serve-saturate", action="store_true",
                    help="queue every serving request at t = 0 (the server's saturated rate)")
    ap.add_argument("--serve-rate", type=float, default=None,
                    help="Poisson arrival rate in requests/s (default: 70 %% of the saturated "
                         "request rate implied by the measured evaluations/s)")
    ap.add_argument("--serve-log", default=None,
                    help="append one JSON line per finished request (and a running summary "
                         "every 50) to this file as the run goes")
    ap.add_argument("--serve-chunk-evals", type=float, default=2e11,
                    help="ray-lens evaluations per serving launch")
    ap.add_argument("--serve-min-launch-rays", type=float, default=2.5e7,
                    help="rays per serving launch, at least (about 8 ray cells per wave slot)")
    ap.add_argument("--no-tuning-cache", action="store_true")
    ap.add_argument("--no-post", action="store_true", help="skip the MPD and codec legs")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-mass 11560-lens map timed beside the main workload")
    ap.add_argument("--no-sweep", action="store_true", help="skip the lens-count sweep at 1e8 rays")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a known-size "
                         "kernel for scaling hardware traffic counters)")
    return ap.parse_args()


def kernel_source_hash():
    """sha256 over the shoot kernel's sources (shoot.hip, then internal.h)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("shoot.hip", "internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1406_0559_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per launch of the FP32 shoot kernel from the rocprofv3 --pmc
    summary in profiles/ (FETCH_SIZE and WRITE_SIZE, scaled by a known-size
    copy), or None if none exists or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_shoot_fp32c_{workload}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        line = line.strip()
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("shoot kernel sources sha256") != kernel_source_hash():
        return None
    fetch = float(vals["fetch bytes per launch"])
    write = float(vals["write bytes per launch"])
    ex = vals.get("executed FP32 flops per evaluation")
    return {"bytes": fetch + write, "fetch_bytes": fetch, "write_bytes": write,
            "binning_mode": vals.get("binning mode"),
            "executed_flops_per_eval": float(ex) if ex else None,
            "source": os.path.relpath(path, ROOT)}


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the path is a single-GPU "
                          "kernel and no multi-GPU run is part of it", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1406_0559_amd import autotune
    from paper_1406_0559_amd import inputs
    from paper_1406_0559_amd import raylens as rl

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    rl.load()
    spec = inputs.WORKLOADS[args.workload]()
    field = spec.lenses()
    ctx = rl.Context(0)
    tuned = False
    if not args.no_tuning_cache:
        try:    # applies the cached table only if this library build wrote it
            ctx.autotune(autotune.DEFAULT_CACHE, 0)
            tuned = True
        except rl.RaylensError:
            tuned = False
            table = autotune.load(autotune.DEFAULT_CACHE) or {}
            print(f"bench: the tuning cache was made for {table.get('library')!r}, not for "
                  f"{rl.rl_version()!r}: default kernel shapes (run python -m "
                  "paper_1406_0559_amd.autotune on the GPU to retune)", file=sys.stderr, flush=True)
    L = rl.DeviceLenses(field.x1, field.x2, field.m)
    counts, esc = ctx.new_map(spec)
    mu = torch.empty((spec.p2, spec.p1), dtype=torch.float32, device="cuda")
    n_avg = rl.rl_n_avg(rl.grid_of(spec), rl.window_of(spec))
    stream = torch.cuda.current_stream()
    evals = spec.evals
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(prec, ev=None):
        counts.zero_()
        esc.zero_()
        if ev is not None:
            ev[0].record(stream)
        ctx.shoot(L, spec, prec, counts, esc, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        ctx.normalise(counts, spec, n_avg=n_avg, mu=mu, stream=stream)
        return ctx.stats(counts, esc, spec, stream=stream)   # synchronises the stream

    # ---- FP32-compensated: the timed steps -------------------------------------
    for _ in range(args.warmup):
        step("fp32c")
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        st = step("fp32c", events[k])
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in events]
    kern_avg_s = float(np.mean(kern_ms)) / 1e3
    ms_per_step = wall / args.steps * 1e3
    value = evals * args.steps / wall
    assert st["binned"] + st["escaped"] == spec.rays, "ray conservation failed"

    # ---- FP64 plain on the same map ---------------------------------------------
    fp64 = None
    if args.fp64_steps > 0:
        step("fp64")
        ev64 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for _ in range(args.fp64_steps)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(args.fp64_steps):
            st64 = step("fp64", ev64[k])
        torch.cuda.synchronize()
        w64 = time.perf_counter() - t1
        k64 = float(np.mean([a.elapsed_time(b) for a, b in ev64])) / 1e3
        fp64 = {"evals_per_s": evals * args.fp64_steps / w64,
                "kernel_ms": k64 * 1e3,
                "tflops_alg": FLOPS_PER_EVAL * evals / k64 / 1e12,
                "frac_fp64_peak": FLOPS_PER_EVAL * evals / k64 / 1e12 / FP64_PEAK_TFLOPS,
                "mean_mu": st64["mean_mu"],
                "mean_mu_rel_diff_fp32c": abs(st["mean_mu"] - st64["mean_mu"]) / st64["mean_mu"]}

    # ---- post-processing of the map: MPD (Section 3.2.1 / 4) and codec (App. B) ----
    post = None
    if not args.no_post:
        mu_th_abs = abs(st["mu_th"])
        n_pix = spec.p1 * spec.p2
        final = counts.clone()

        def timed(fn, reps=5):
            """Median device time of one call: a GPU sleep of ~0.4 ms is queued
            ahead of the events, so the call's host work (argument checks,
            thresholds, launches) is done while the GPU is still busy and the
            events bracket only its copies and kernels on the stream."""
            fn()
            torch.cuda.synchronize()
            ms = []
            for _ in range(reps):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                with torch.cuda.stream(stream):
                    torch.cuda._sleep(1000000)
                a.record(stream)
                fn()
                b.record(stream)
                b.synchronize()
                ms.append(a.elapsed_time(b))
            return float(np.median(ms))

        hist = torch.zeros(st["max_count"] + 1, dtype=torch.int64, device="cuda")
        bins = torch.zeros(102, dtype=torch.int64, device="cuda")
        t_hist = timed(lambda: ctx.count_histogram(final, spec, hist.numel(), hist=hist,
                                                   stream=stream))
        t_mpd = timed(lambda: ctx.mpd(final, spec, mu_th_abs, -1.5, 1.5, 100, n_avg=n_avg,
                                      bins=bins, stream=stream))
        t_sum = timed(lambda: ctx.probability_sums(final, spec, 1.25 * mu_th_abs, n_avg=n_avg,
                                                   stream=stream))
        values, bits, packed = ctx.encode(final, spec, stream=stream)
        t_enc = timed(lambda: ctx.encode(final, spec, stream=stream), reps=3)
        back = torch.empty_like(final)
        t_dec = timed(lambda: ctx.decode(packed, bits, values, spec, counts=back, stream=stream))
        assert torch.equal(back, final), "codec round trip failed"
        # finite source (Section 2.4, eq. 6): Gaussian disc of 0.2 Einstein radii
        kern = ctx.source_kernel(spec, "gaussian", 0.2, stream=stream)
        conv = torch.empty((spec.p2, spec.p1), dtype=torch.float64, device="cuda")
        t_kern = timed(lambda: ctx.source_kernel(spec, "gaussian", 0.2, kernel=kern, stream=stream))
        # the same disc as a tabulated profile of the stored size (Section 3.2:
        # regular grids of 1000 - 3000 points per axis), 2000 x 2000 FP32
        # samples copied from the host on every call
        ax = np.linspace(-0.2, 0.2, 2000)
        rr = np.hypot(ax[None, :], ax[:, None])
        tb = np.where(rr < 0.2, np.exp(-rr * rr / (2 * (0.2 / 3) ** 2)), 0.0).astype(np.float32)
        ax = ax.astype(np.float32)
        ktab = torch.empty_like(kern)
        t_tab = []
        for _ in range(6):     # wall time: the host's checks and copy are part of the call
            stream.synchronize()
            t0 = time.perf_counter()
            ctx.source_kernel_table(spec, ax, ax, tb, kernel=ktab, stream=stream)
            stream.synchronize()
            t_tab.append((time.perf_counter() - t0) * 1e3)
        t_tab = float(np.median(t_tab[1:]))
        t_conv = timed(lambda: ctx.convolve(final, kern, spec, n_avg=n_avg, out=conv, stream=stream))
        # the MPD of the finite-source map (stored for every convolution)
        mbins = torch.zeros(102, dtype=torch.int64, device="cuda")
        t_mpdv = timed(lambda: ctx.mpd_values(conv, spec, mu_th_abs, -1.5, 1.5, 100, bins=mbins, stream=stream))
        # one map against four source sizes in one call (the map's transforms once)
        kerns4 = [ctx.source_kernel(spec, "gaussian", r, stream=stream) for r in (0.1, 0.2, 0.4, 0.8)]
        outs4 = [torch.empty_like(conv) for _ in kerns4]
        t_batch4 = timed(lambda: ctx.convolve_batch(final, kerns4, spec, n_avg=n_avg, outs=outs4, stream=stream))
        del kerns4, outs4
        # the same call with a kernel that is nonzero on every row (no row pair
        # of zeros whose transform can be skipped)
        gd = torch.Generator(device="cuda").manual_seed(12)
        dense = torch.rand((spec.p2, spec.p1), dtype=torch.float64, device="cuda", generator=gd)
        dense /= dense.sum()
        t_conv_dense = timed(lambda: ctx.convolve(final, dense, spec, n_avg=n_avg, out=conv, stream=stream))
        del dense
        # the high-resolution GERLUMPH side: a seeded synthetic 10000^2 count map
        # (uniform in [0, 90)) and the same source on its 25 x 25 Einstein radii
        spec10 = dataclasses.replace(spec, p1=10000, p2=10000, name="synthetic-10000sq")
        g10 = torch.Generator(device="cuda").manual_seed(11)
        m10 = torch.randint(0, 90, (10000, 10000), dtype=torch.int32, device="cuda", generator=g10)
        k10 = ctx.source_kernel(spec10, "gaussian", 0.2, stream=stream)
        c10 = torch.empty((10000, 10000), dtype=torch.float64, device="cuda")
        t_conv10 = timed(lambda: ctx.convolve(m10, k10, spec10, n_avg=n_avg, out=c10, stream=stream))
        del m10, k10, c10
        gbs = lambda nbytes, ms: nbytes / (ms * 1e-3) / 1e9
        post = {"pixels": n_pix,
                "timing": "median device time per call: copies and kernels on the stream, host work hidden",
                "source_kernel_us": t_kern * 1e3,
                "source_kernel_table_wall_ms": t_tab, "source_table_samples": int(tb.size),
                "convolve_ms": t_conv, "convolve_10000sq_ms": t_conv10,
                "convolve_dense_kernel_ms": t_conv_dense,
                "convolve_batch4_ms_per_kernel": t_batch4 / 4,
                "mpd_of_convolved_map_us": t_mpdv * 1e3,
                "convolve_min_GBps": gbs(20 * n_pix, t_conv),
                "count_histogram_us": t_hist * 1e3, "count_histogram_GBps": gbs(4 * n_pix, t_hist),
                "mpd_100bins_us": t_mpd * 1e3, "mpd_GBps": gbs(4 * n_pix, t_mpd),
                "probability_sums_us": t_sum * 1e3,
                "p_mu_above_1.25_mu_th": ctx.probability_sums(final, spec, 1.25 * mu_th_abs,
                                                              n_avg=n_avg)[1] / n_pix,
                "codec_distinct_values": int(values.numel()), "codec_bits": bits,
                "codec_bytes": int(packed.numel() * 4 + values.numel() * 4),
                "codec_ratio_vs_int32": (packed.numel() * 4 + values.numel() * 4) / (4 * n_pix),
                "encode_ms": t_enc, "decode_us": t_dec * 1e3,
                "decode_GBps": gbs(4 * n_pix + packed.numel() * 4, t_dec),
                "hbm_peak_GBps": 8000.0}

    # ---- 64-map batched persistent launch ---------------------------------------
    batch = None
    if not args.no_batch:
        maps = inputs.config_batch()
        Ls = [rl.DeviceLenses(*(lambda f: (f.x1, f.x2, f.m))(m.lenses())) for m in maps]
        outs = [ctx.new_map(m) for m in maps]
        items = [(Lb, m, c, e) for Lb, m, (c, e) in zip(Ls, maps, outs)]

        def run_batch():
            for c, e in outs:
                c.zero_()
                e.zero_()
            ctx.shoot_batch(items, "fp32c", stream=stream)
            torch.cuda.synchronize()

        run_batch()
        tb = time.perf_counter()
        run_batch()
        wb = time.perf_counter() - tb
        bevals = sum(m.evals for m in maps)
        batch = {"workload": "batch-64x1024sq", "maps": len(maps), "seconds": wb,
                 "maps_per_hour": len(maps) * 3600.0 / wb, "evals_per_s": bevals / wb}

    # ---- second full-size workload: mixed masses, smooth matter, 11560 lenses -------
    mixed = None
    if not args.no_mixed and args.workload != "mixed-20000sq-11560":
        ms_ = inputs.config_mixed()
        fm = ms_.lenses()
        Lm = rl.DeviceLenses(fm.x1, fm.x2, fm.m)
        cm, em = ctx.new_map(ms_)
        evm = []
        for k in range(3):
            cm.zero_()
            em.zero_()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ctx.shoot(Lm, ms_, "fp32c", cm, em, stream=stream)
            b.record(stream)
            b.synchronize()
            if k:
                evm.append(a.elapsed_time(b))
        km = float(np.mean(evm)) / 1e3
        mixed = {"workload": ms_.name, "lenses": ms_.n_lens, "masses": ms_.masses,
                 "kernel_ms": km * 1e3, "evals_per_s": ms_.evals / km,
                 "tflops_alg": FLOPS_PER_EVAL * ms_.evals / km / 1e12,
                 "frac": FLOPS_PER_EVAL * ms_.evals / km / 1e12 / FP32_PEAK_TFLOPS}
        if args.fp64_steps > 0:        # the FP64-plain path on the same map, one launch
            c64, e64 = ctx.new_map(ms_)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ctx.shoot(Lm, ms_, "fp64", c64, e64, stream=stream)
            b.record(stream)
            b.synchronize()
            k64m = a.elapsed_time(b) / 1e3
            st32 = ctx.stats(cm, em, ms_, stream=stream)
            st64m = ctx.stats(c64, e64, ms_, stream=stream)
            mixed.update({"fp64_kernel_ms": k64m * 1e3, "fp64_evals_per_s": ms_.evals / k64m,
                          "speedup_fp32c_over_fp64": k64m / km,
                          "mean_mu_rel_diff_fp32c": abs(st32["mean_mu"] - st64m["mean_mu"]) /
                          abs(st64m["mean_mu"])})
            del c64, e64
        del Lm, cm, em

    # ---- N_* sweep: evaluations/s against the lens count at 1e8 rays --------------
    sweep = None
    if not args.no_sweep:
        base = inputs.config_gerlumph()
        sweep = []
        for n_l in (50, 100, 300, 1000, 3000, 10000, 30000, 100000):
            sp = inputs.scaled(base, ray_factor=(1e8 / base.rays) ** 0.5, name=f"nstar-{n_l}")
            sp = dataclasses.replace(sp, n_lens=n_l,
                                            disc_radius=(n_l / base.kappa_star) ** 0.5, seed=7)
            fs = sp.lenses()
            Ls_ = rl.DeviceLenses(fs.x1, fs.x2, fs.m)
            cs, es = ctx.new_map(sp)
            best = None
            for k in range(6):        # one warm-up, then the best of five
                # device time: the zeroing and a GPU sleep are queued ahead of
                # the events, so the call's host work overlaps them
                with torch.cuda.stream(stream):
                    cs.zero_()
                    es.zero_()
                    torch.cuda._sleep(1000000)
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                ctx.shoot(Ls_, sp, "fp32c", cs, es, stream=stream)
                b.record(stream)
                b.synchronize()
                if k:
                    best = a.elapsed_time(b) if best is None else min(best, a.elapsed_time(b))
            sweep.append({"n_lens": n_l, "rays": sp.rays, "kernel_ms": best,
                          "evals_per_s": sp.evals / (best / 1e3)})
            del Ls_, cs, es

    # ---- realisation batch: 15 lens fields of one macro model -> mean MPD +- sigma --
    reals = None
    if not args.no_batch:
        from paper_1406_0559_amd import realisations
        base = inputs.config_realisation_base()
        rspecs = realisations.realisation_specs(base, 15)
        rL = [rl.DeviceLenses(*(lambda f: (f.x1, f.x2, f.m))(sp.lenses())) for sp in rspecs]
        routs = [ctx.new_map(sp) for sp in rspecs]
        navg_r = rl.rl_n_avg(rl.grid_of(base), rl.window_of(base))
        c0, e0 = routs[0]
        mu_th_r = abs(ctx.stats(c0, e0, base, stream=stream)["mu_th"])   # the library's mu_th
        rbins = torch.zeros((15, 102), dtype=torch.int64, device="cuda")

        def run_reals():
            for c, e in routs:
                c.zero_()
                e.zero_()
            rbins.zero_()
            ctx.shoot_batch([(Lr, sp, c, e) for Lr, sp, (c, e) in zip(rL, rspecs, routs)], "fp32c",
                            stream=stream)
            for r, (sp, (c, _)) in enumerate(zip(rspecs, routs)):
                ctx.mpd(c, sp, mu_th_r, -1.5, 1.5, 100, n_avg=navg_r, bins=rbins[r], stream=stream)
            return ctx.mpd_moments(rbins, base.p1 * base.p2, stream=stream)

        run_reals()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        rmean, rstd = run_reals()
        b.record(stream)
        b.synchronize()
        tr = a.elapsed_time(b) / 1e3
        revals = sum(sp.evals for sp in rspecs)
        reals = {"workload": f"realisations-15x{base.p1}sq-{base.n_lens}", "maps": 15,
                 "lenses": base.n_lens, "seconds": tr, "evals_per_s": revals / tr,
                 "maps_per_hour": 15 * 3600.0 / tr,
                 "mean_mpd_peak_bin": int(torch.argmax(rmean).item()),
                 "max_relative_sigma": float((rstd / rmean.clamp_min(1e-12))[rmean > 1e-3].max().item())}
        del rL, routs

    # ---- serving: Poisson stream of map requests, continuous batching -------------
    serving = None
    if not args.no_serve:
        from paper_1406_0559_amd import serve
        probe = inputs.serve_requests(args.serve_requests, rate=1.0, seed=5,
                                      size_scale=args.serve_scale)
        mean_evals = float(np.mean([r.spec.evals for r in probe]))
        # 70 % of the saturated request rate unless a rate is given
        lam = args.serve_rate if args.serve_rate else 0.7 * value / mean_evals
        reqs = inputs.serve_requests(args.serve_requests, rate=lam, seed=5,
                                     size_scale=args.serve_scale)
        if args.serve_saturate:                 # every request queued at t = 0
            lam = None
        mreqs = [serve.MapRequest(r.rid, r.spec, r.spec.lenses(), 0.0 if args.serve_saturate else r.arrival)
                 for r in reqs]
        by_rid = {r.rid: r for r in reqs}
        be = serve.GpuBackend(ctx=ctx)
        log = open(args.serve_log, "a") if args.serve_log else None
        lat_done = []
        evals_done = [0]
        t_start = [None]

        def progress(res):
            spec = by_rid[res.rid].spec
            if res.state is serve.State.DONE:
                lat_done.append(res.latency)
                evals_done[0] += spec.evals
            if log is not None:
                log.write(json.dumps({"rid": res.rid, "state": res.state.value,
                                      "arrival_s": res.arrival, "admitted_s": res.admitted,
                                      "finished_s": res.finished, "latency_s": res.latency,
                                      "pixels": spec.p1, "lenses": spec.n_lens,
                                      "rays": spec.rays, "evals": spec.evals,
                                      "error": res.error}) + "\n")
                if len(lat_done) % 50 == 0 and res.state is serve.State.DONE:
                    el = time.perf_counter() - t_start[0]
                    log.write(json.dumps({"summary": True, "completed": len(lat_done),
                                          "elapsed_s": el, "p50_s": percentile(lat_done, 50),
                                          "p99_s": percentile(lat_done, 99),
                                          "evals_per_s": evals_done[0] / el}) + "\n")
                log.flush()
            res.counts = None               # delivered; not kept for the whole run
            n = len(lat_done)
            if res.state is serve.State.DONE and n % 25 == 0:
                print(f"serving: {n}/{len(mreqs)} requests finished", file=sys.stderr, flush=True)

        sch = serve.Scheduler(be, budget_bytes=serve.gpu_budget_bytes(0.5), max_active=16,
                              chunk_evals=args.serve_chunk_evals,
                              min_launch_rays=int(args.serve_min_launch_rays), max_inflight=2,
                              work_rate=value, on_finish=progress)
        ts = time.perf_counter()
        t_start[0] = ts
        res = sch.run(mreqs)
        tserve = time.perf_counter() - ts
        if log is not None:
            log.close()
        summ = serve.latency_summary(res)
        sizes = sorted({r.spec.p1 for r in reqs})
        serving = {"workload": f"serve-{args.serve_requests}req-maps{sizes[0]}-{sizes[-1]}"
                               + ("-saturated" if args.serve_saturate else ""),
                   "arrival_rate_per_s": lam, "mean_evals_per_request": mean_evals,
                   "offered_load": (lam * mean_evals / value) if lam else None,
                   "launches": sch.launches, "peak_active": sch.peak_active,
                   "wall_s": tserve, **summ,
                   "p50_ms": summ["p50_s"] * 1e3 if summ["p50_s"] is not None else None,
                   "p99_ms": summ["p99_s"] * 1e3 if summ["p99_s"] is not None else None,
                   "evals_per_s": sum(r.spec.evals for r in reqs) / summ["makespan_s"]
                   if summ["makespan_s"] else None}

    # ---- CPU baseline: the oracle on a bounded row sample of the same map ---------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nthreads = oracle.max_threads()
        r0 = spec.n2 // 2
        probe_rows = max(2, nthreads)
        tp = time.perf_counter()
        oracle.shoot(field.x1, field.x2, field.m, spec.kappa, spec.gamma, spec.s, spec.n1, spec.n2,
                     spec.c1, spec.c2, spec.h1, spec.h2, spec.p1, spec.p2, spec.w1, spec.w2,
                     spec.W1, spec.W2, r0, r0 + probe_rows)
        per_row = (time.perf_counter() - tp) / probe_rows
        rows = int(max(probe_rows, min(spec.n2 - r0, args.cpu_seconds / max(per_row, 1e-9))))
        tc = time.perf_counter()
        oracle.shoot(field.x1, field.x2, field.m, spec.kappa, spec.gamma, spec.s, spec.n1, spec.n2,
                     spec.c1, spec.c2, spec.h1, spec.h2, spec.p1, spec.p2, spec.w1, spec.w2,
                     spec.W1, spec.W2, r0, r0 + rows)
        tcpu = time.perf_counter() - tc
        # one thread on a few rows: the per-core rate
        r1 = max(1, int(2.0 / max(per_row * nthreads, 1e-9)))
        t1 = time.perf_counter()
        oracle.shoot(field.x1, field.x2, field.m, spec.kappa, spec.gamma, spec.s, spec.n1, spec.n2,
                     spec.c1, spec.c2, spec.h1, spec.h2, spec.p1, spec.p2, spec.w1, spec.w2,
                     spec.W1, spec.W2, r0, r0 + r1, nthreads=1)
        per_core = r1 * spec.n1 * spec.n_lens / (time.perf_counter() - t1)
        cpu = {"value": rows * spec.n1 * spec.n_lens / tcpu, "unit": "evals/s", "cores": nthreads,
               "per_core_evals_per_s": per_core, "kind": "oracle",
               "sample": f"ray rows [{r0}, {r0 + rows}) of the {spec.n1}x{spec.n2} grid "
                         f"({rows * spec.n1} rays x {spec.n_lens} lenses, FP64, OpenMP), "
                         f"{tcpu:.1f} s"}
        # accuracy of the GPU positions on two sampled rows against the oracle
        def accuracy(sp, fl, Ld, rb):
            o1, o2, _, rmin = oracle.ray_positions(fl.x1, fl.x2, fl.m, sp.kappa, sp.gamma, sp.s,
                                                   sp.n1, sp.n2, sp.c1, sp.c2, sp.h1, sp.h2, rb, rb + 2)
            lo1, lo2 = sp.w1 - 0.5 * sp.W1 - 1.0, sp.w2 - 0.5 * sp.W2 - 1.0
            inwin = (o1 >= lo1) & (o1 < lo1 + sp.W1 + 2.0) & (o2 >= lo2) & (o2 < lo2 + sp.W2 + 2.0)
            far = inwin & (rmin >= 0.015)
            acc = {"workload": sp.name, "rows": [rb, rb + 2], "rays_in_window": int(inwin.sum()),
                   "near_lens_rays": int((inwin & ~far).sum())}
            for prec in ("fp32c", "fp64"):
                g1, g2 = ctx.ray_positions(Ld, sp, prec, rb, rb + 2)
                g1 = g1.cpu().numpy()
                g2 = g2.cpu().numpy()
                err = np.hypot(g1 - o1, g2 - o2)
                acc[prec] = {"max_abs_dy": float(err[far].max()) if far.any() else None,
                             "rms_dy": float(np.sqrt(np.mean(err[far] ** 2))) if far.any() else None,
                             "bit_identical": bool((g1.view(np.int64) == o1.view(np.int64)).all() and
                                                   (g2.view(np.int64) == o2.view(np.int64)).all())}
            return acc

        cpu["accuracy_vs_oracle"] = accuracy(spec, field, L, r0)
        if mixed is not None:
            ms2 = inputs.config_mixed()
            fm2 = ms2.lenses()
            cpu["accuracy_vs_oracle_mixed"] = accuracy(ms2, fm2, rl.DeviceLenses(fm2.x1, fm2.x2, fm2.m),
                                                       ms2.n2 // 2)

    achieved = FLOPS_PER_EVAL * evals / kern_avg_s / 1e12
    traffic = measured_traffic(spec.name)
    out = {
        "metric": "ray-lens evals/s FP32-comp vs FP64 plain; maps/hour + p50/p99 map latency",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": spec.name, "rays": f"{spec.n1}x{spec.n2}", "lenses": spec.n_lens,
                   "map": f"{spec.p1}x{spec.p2}", "width_RE": spec.W1, "kappa": spec.kappa,
                   "gamma": spec.gamma, "s": spec.s, "evals_per_map": evals},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": traffic["bytes"] if traffic else None,
                     "traffic_detail": traffic,
                     "executed_tflops": (traffic["executed_flops_per_eval"] * evals / kern_avg_s / 1e12
                                         if traffic and traffic.get("executed_flops_per_eval") else None),
                     "kernel": "shoot_kernel (FP32-compensated)",
                     "kernel_ms": kern_avg_s * 1e3,
                     "kernel_ms_min_max": [float(np.min(kern_ms)), float(np.max(kern_ms))],
                     "algorithmic_flops_per_launch": FLOPS_PER_EVAL * evals},
        "cpu_baseline": cpu,
        "fp64_plain": fp64,
        "speedup_fp32c_over_fp64": (value / fp64["evals_per_s"]) if fp64 else None,
        "maps_per_hour": 3600.0 / (ms_per_step / 1e3),
        "map_latency_ms": {"p50": percentile(lat, 50) * 1e3, "p99": percentile(lat, 99) * 1e3},
        "mean_mu": st["mean_mu"],
        "mu_th": st["mu_th"],
        "batch": batch,
        "post_processing": post,
        "mixed_workload": mixed,
        "realisations": reals,
        "nstar_sweep": sweep,
        "serving": serving,
        "tuning": "autotuned cache" if tuned else "defaults",
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Writes tests/golden/full_map_digests.json: the oracle's whole maps of the
full-size workloads, reduced to digests the GPU tests can compare against.

For each map of the GERLUMPH-like workload (30000^2 rays, 2624 lenses), the
mixed-mass workload (20000^2 rays, 11560 lenses) and the 64 maps of the batched
workload, the plain FP64 oracle (Section 2.1, eq. 1 per ray, then the pixel
count of Fig. 1) is run over every ray row. Stored per map:

  * sha256 of the int32 count map (row-major, x1 fastest, little-endian), the
    binned and escaped ray counts and the count sums of 16 bands of pixel rows
    (so a mismatch says where);
  * for a ladder of distances delta, the number of rays whose oracle position
    lies within delta of a pixel edge of the window (either axis, window
    boundary included). A ray whose computed position is off by less than
    delta can only change pixel if it is one of these, so a map computed with
    per-ray errors below delta differs from the oracle's by at most twice
    that number in the sum of |N_ij - N'_ij| (the count bound of the
    FP32-compensated path).

The map is the oracle's binning of the oracle's positions (oracle.ray_positions,
then oracle.bin_positions, the two halves of oracle.shoot); the first and the
last row block of every map are checked against oracle.shoot itself.

Only oracle/ and the seeded input generators are called. Run from the
repository root: `python tests/golden/make_full_map_digests.py [--only NAME]`.
A full run takes about half an hour on 8 cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1406_0559_amd import inputs  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "full_map_digests.json")
DELTAS = (1e-6, 2e-6, 5e-6, 1e-5, 2e-5, 5e-5, 1e-4)
BANDS = 16


def edge_counts(y1, y2, spec):
    """Rays within delta of a pixel edge, for each delta of the ladder. The
    pixel lines sit at lo + k W / P (k = 0..P); a ray counts if it lies within
    delta of one of them on either axis while inside the window grown by delta
    on both axes."""
    lo1 = spec.w1 - 0.5 * spec.W1
    lo2 = spec.w2 - 0.5 * spec.W2
    pix1 = spec.W1 / spec.p1
    pix2 = spec.W2 / spec.p2
    t1 = (y1 - lo1) / pix1
    t2 = (y2 - lo2) / pix2
    ok = np.isfinite(t1) & np.isfinite(t2)
    t1 = np.where(ok, t1, -1e30)
    t2 = np.where(ok, t2, -1e30)
    e1 = np.abs(t1 - np.rint(t1)) * pix1
    e2 = np.abs(t2 - np.rint(t2)) * pix2
    out = []
    for d in DELTAS:
        g1, g2 = d / pix1, d / pix2
        inside = (t1 > -g1) & (t1 < spec.p1 + g1) & (t2 > -g2) & (t2 < spec.p2 + g2)
        out.append(int(np.count_nonzero(inside & ((e1 < d) | (e2 < d)))))
    return np.array(out, np.int64)


def digest_map(spec, block_rows=256, log=print):
    f = spec.lenses()
    counts = np.zeros((spec.p2, spec.p1), np.int32)
    esc = 0
    near = np.zeros(len(DELTAS), np.int64)
    t0 = time.time()
    starts = list(range(0, spec.n2, block_rows))
    for b, r0 in enumerate(starts):
        r1 = min(spec.n2, r0 + block_rows)
        y1, y2, sing, _ = oracle.ray_positions(f.x1, f.x2, f.m, spec.kappa, spec.gamma, spec.s,
                                               spec.n1, spec.n2, spec.c1, spec.c2, spec.h1,
                                               spec.h2, r0, r1)
        _, e = oracle.bin_positions(y1, y2, spec.p1, spec.p2, spec.w1, spec.w2, spec.W1, spec.W2,
                                    singular=sing, counts=counts)
        esc += e
        live = sing.ravel() == 0
        near += edge_counts(y1.ravel()[live], y2.ravel()[live], spec)
        if b == 0 or b == len(starts) - 1:
            part, _ = oracle.bin_positions(y1, y2, spec.p1, spec.p2, spec.w1, spec.w2, spec.W1,
                                           spec.W2, singular=sing)
            ref, _ = oracle.shoot(f.x1, f.x2, f.m, spec.kappa, spec.gamma, spec.s, spec.n1,
                                  spec.n2, spec.c1, spec.c2, spec.h1, spec.h2, spec.p1, spec.p2,
                                  spec.w1, spec.w2, spec.W1, spec.W2, r0, r1)
            assert np.array_equal(part, ref), f"{spec.name}: positions + binning != shoot"
        if (b + 1) % 16 == 0:
            log(f"  {spec.name}: rows {r1}/{spec.n2}, {time.time() - t0:.0f} s")
    binned = int(counts.sum(dtype=np.int64))
    assert binned + esc == spec.rays, f"{spec.name}: ray conservation"
    band = -(-spec.p2 // BANDS)
    return {
        "name": spec.name,
        "rays": spec.rays, "lenses": spec.n_lens, "pixels": [spec.p1, spec.p2],
        "sha256": hashlib.sha256(counts.astype("<i4").tobytes()).hexdigest(),
        "binned": binned, "escaped": int(esc),
        "band_rows": band,
        "band_sums": [int(counts[k:k + band].sum(dtype=np.int64)) for k in range(0, spec.p2, band)],
        "edge_deltas": list(DELTAS),
        "rays_near_edge": [int(v) for v in near],
        "oracle_seconds": round(time.time() - t0, 1),
    }


def workloads():
    yield "gerlumph", inputs.config_gerlumph()
    yield "mixed", inputs.config_mixed()
    for k, spec in enumerate(inputs.config_batch()):
        yield f"batch-{k:02d}", spec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None, help="compute only this key (merged into the file)")
    args = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        data = json.load(open(OUT))
    data.setdefault("source", "written by tests/golden/make_full_map_digests.py from the FP64 "
                    "oracle (oracle/oracle.c) over every ray of each map")
    data.setdefault("maps", {})
    for key, spec in workloads():
        if args.only and key != args.only:
            continue
        print(f"{key}: {spec.name}, {spec.rays} rays x {spec.n_lens} lenses", flush=True)
        data["maps"][key] = digest_map(spec, log=lambda s: print(s, flush=True))
        tmp = OUT + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, OUT)
        print(f"  {key}: done in {data['maps'][key]['oracle_seconds']} s", flush=True)


if __name__ == "__main__":
    main()

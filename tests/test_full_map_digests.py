"""The stored whole-map oracle digests (tests/golden/full_map_digests.json)
on the CPU: every entry is self-consistent, and the cheapest map (a batch map
of 200 lenses) recomputed with the oracle gives the stored entry exactly."""
import importlib.util
import json
import os

import pytest

from paper_1406_0559_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def load_script():
    spec = importlib.util.spec_from_file_location(
        "make_full_map_digests", os.path.join(GOLDEN, "make_full_map_digests.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def digests():
    with open(os.path.join(GOLDEN, "full_map_digests.json")) as fh:
        return json.load(fh)["maps"]


def test_every_workload_map_has_a_consistent_digest():
    d = digests()
    specs = {"gerlumph": inputs.config_gerlumph(), "mixed": inputs.config_mixed()}
    specs.update({f"batch-{k:02d}": s for k, s in enumerate(inputs.config_batch())})
    assert set(d) == set(specs)
    for key, spec in specs.items():
        e = d[key]
        assert e["name"] == spec.name and e["rays"] == spec.rays and e["lenses"] == spec.n_lens
        assert e["binned"] + e["escaped"] == spec.rays, key
        assert sum(e["band_sums"]) == e["binned"], key
        assert len(e["sha256"]) == 64
        near = e["rays_near_edge"]
        # more rays lie within a larger distance of an edge
        assert all(a <= b for a, b in zip(near, near[1:])), key
        assert near[-1] <= e["rays"]


def test_cheapest_map_recomputed_with_the_oracle():
    mod = load_script()
    maps = inputs.config_batch()
    k, spec = min(enumerate(maps), key=lambda ks: ks[1].evals)
    got = mod.digest_map(spec, log=lambda s: None)
    want = digests()[f"batch-{k:02d}"]
    for field in ("sha256", "binned", "escaped", "band_sums", "rays_near_edge", "edge_deltas"):
        assert got[field] == want[field], field

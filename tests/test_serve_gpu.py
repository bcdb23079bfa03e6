"""The map server on the GPU: requests of mixed size, lens count, mass model
and precision arrive while others run, share batched launches, and every map
equals the map of the same request shot alone (bit for bit; FP64 maps also
equal the oracle's)."""
import numpy as np
import pytest

import oracle
from paper_1406_0559_amd import inputs
from paper_1406_0559_amd import raylens as rl
from paper_1406_0559_amd import serve

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def mixed_requests(n=10, seed=5):
    reqs = serve_specs = inputs.serve_requests(n, rate=60.0, seed=seed, sizes=(128, 256, 512),
                                               n_lens_range=(100, 4000), size_scale=0.5)
    out = []
    for k, r in enumerate(serve_specs):
        spec = r.spec
        if k % 3 == 1:
            spec = inputs.dataclasses.replace(spec, masses="salpeter")
        prec = "fp64" if k % 4 == 3 else "fp32c"
        out.append(serve.MapRequest(r.rid, spec, spec.lenses(), r.arrival, prec))
    return out


def test_served_maps_equal_maps_shot_alone():
    assert torch.cuda.is_available()
    reqs = mixed_requests()
    be = serve.GpuBackend()
    sch = serve.Scheduler(be, budget_bytes=serve.gpu_budget_bytes(0.25), max_active=8,
                          chunk_evals=5e8, max_inflight=2)
    res = sch.run(reqs)
    assert all(r.state is serve.State.DONE for r in res.values()), \
        {k: (r.state, r.error) for k, r in res.items()}
    assert sch.launches > len(reqs), "requests were not chunked"
    ctx = be.ctx
    for req in reqs:
        L = rl.DeviceLenses(req.lenses.x1, req.lenses.x2, req.lenses.m)
        c, e = ctx.shoot(L, req.spec, req.precision)
        r = res[req.rid]
        assert (r.counts == c.cpu().numpy()).all(), req.rid
        assert r.escaped == int(e.item()), req.rid
        assert r.stats["binned"] + r.stats["escaped"] == req.spec.rays
        if req.precision == "fp64" and req.spec.evals < 3e9:
            s, f = req.spec, req.lenses
            oc, oe = oracle.shoot(f.x1, f.x2, f.m, s.kappa, s.gamma, s.s, s.n1, s.n2, s.c1, s.c2,
                                  s.h1, s.h2, s.p1, s.p2, s.w1, s.w2, s.W1, s.W2)
            assert (r.counts == oc).all() and r.escaped == oe
    summ = serve.latency_summary(res)
    assert summ["completed"] == len(reqs) and summ["p99_s"] >= summ["p50_s"] > 0
    assert sch.used == 0


def test_checkpoint_resume_and_cancel_on_the_gpu():
    base = mixed_requests(2, seed=8)
    spec = inputs.dataclasses.replace(base[0].spec, n1=600, n2=1100, n_lens=700, masses="salpeter")
    target = serve.MapRequest(50, spec, spec.lenses(), 0.0, "fp32c")
    reqs = [target] + base
    be = serve.GpuBackend()
    # 9 chunks of 128 rows for the target; the first launch is the target's
    # first chunk alone, then the others join; at most two launches before
    # the checkpoint
    sch = serve.Scheduler(be, budget_bytes=serve.gpu_budget_bytes(0.25),
                          chunk_evals=spec.n1 * spec.n_lens * 128, max_inflight=1)
    sch.submit(target)
    sch.step()
    for r in base:
        sch.submit(r)
    sch.step()
    cp = sch.checkpoint(target.rid)
    assert 0 < cp.next_row < spec.n2
    sch.cancel(base[0].rid)
    res = sch.run([serve.MapRequest(target.rid, spec, target.lenses, sch.now(), "fp32c",
                                    resume=cp)])
    L = rl.DeviceLenses(target.lenses.x1, target.lenses.x2, target.lenses.m)
    c, e = be.ctx.shoot(L, spec, "fp32c")
    assert res[target.rid].state is serve.State.DONE
    assert (res[target.rid].counts == c.cpu().numpy()).all()
    assert res[target.rid].escaped == int(e.item())
    assert res[base[0].rid].state in (serve.State.CANCELLED, serve.State.DONE)
    assert sch.used == 0

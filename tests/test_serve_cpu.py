"""Scheduling, admission, faults, cancellation and resume of the map server,
on the CPU: the device is replaced by a backend that shoots each chunk with
the FP64 oracle and reports completion after a simulated duration on a
virtual clock. Every finished map must equal the oracle's map of the same
request shot whole, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1406_0559_amd import inputs
from paper_1406_0559_amd.serve import MapRequest, Scheduler, State, footprint_bytes, latency_summary


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt):
        self.t += max(dt, 1e-6)


class CpuBackend:
    """Chunks run at submission on the CPU; a launch 'finishes' once the
    virtual clock has passed its simulated duration (evals / rate)."""

    def __init__(self, clock, rate=1e9, fail_admit=(), fail_launch=(), fail_finalize=()):
        self.clock = clock
        self.rate = rate
        self.busy_until = 0.0
        self.fail_admit = set(fail_admit)
        self.fail_launch = set(fail_launch)
        self.fail_finalize = set(fail_finalize)
        self.live = 0
        self.launch_log = []

    def admit(self, req):
        if req.rid in self.fail_admit:
            raise MemoryError("injected allocation failure")
        self.live += 1
        return {"rid": req.rid, "spec": req.spec, "f": req.lenses,
                "counts": np.zeros((req.spec.p2, req.spec.p1), np.int32), "esc": 0}

    def launch(self, chunks, precision):
        rids = [h["rid"] for h, _, _, _ in chunks]
        if self.fail_launch & set(rids):
            raise RuntimeError("injected launch failure")
        work = 0
        for h, spec, rb, re in chunks:
            f = h["f"]
            _, e = oracle.shoot(f.x1, f.x2, f.m, spec.kappa, spec.gamma, spec.s, spec.n1, spec.n2,
                                spec.c1, spec.c2, spec.h1, spec.h2, spec.p1, spec.p2, spec.w1,
                                spec.w2, spec.W1, spec.W2, rb, re, counts=h["counts"])
            h["esc"] += e
            work += (re - rb) * spec.n1 * max(1, spec.n_lens)
        start = max(self.busy_until, self.clock())
        self.busy_until = start + work / self.rate
        self.launch_log.append((self.clock(), sorted(rids)))
        return {"end": self.busy_until}

    def done(self, token):
        return self.clock() >= token["end"]

    def wait(self, token, timeout=None):
        if timeout is None or self.clock() + timeout >= token["end"]:
            self.clock.t = max(self.clock.t, token["end"])
            return True
        self.clock.advance(timeout)
        return False

    def read_partial(self, h):
        return h["counts"].copy(), h["esc"]

    def load_partial(self, h, counts, esc):
        h["counts"][...] = counts
        h["esc"] = esc

    def finalize(self, h, keep_mu=False):
        if h["rid"] in self.fail_finalize:
            raise RuntimeError("injected finalisation failure")
        spec = h["spec"]
        navg = oracle.n_avg(spec.n1, spec.n2, spec.h1, spec.h2, spec.p1, spec.p2, spec.W1, spec.W2)
        st = oracle.stats(h["counts"], navg, spec.kappa, spec.gamma)
        return h["counts"].copy(), h["esc"], st, None

    def release(self, h):
        self.live -= 1
        h.clear()


def small_request(rid, n1, n2, n_lens, arrival=0.0, seed=None, p=32):
    spec = inputs.MapSpec(name=f"r{rid}", kappa=0.45, gamma=0.2, s=0.3, n1=n1, n2=n2, h1=6.0,
                          h2=3.0, p1=p, p2=p, W1=4.0, W2=4.0, n_lens=n_lens, disc_radius=8.0,
                          masses="salpeter", seed=100 + rid if seed is None else seed)
    return MapRequest(rid, spec, spec.lenses(), arrival)


def whole(req):
    s, f = req.spec, req.lenses
    return oracle.shoot(f.x1, f.x2, f.m, s.kappa, s.gamma, s.s, s.n1, s.n2, s.c1, s.c2, s.h1,
                        s.h2, s.p1, s.p2, s.w1, s.w2, s.W1, s.W2)


def make(clock, backend, **kw):
    kw.setdefault("budget_bytes", 1 << 30)
    kw.setdefault("chunk_evals", 128 * 300 * 20)
    kw.setdefault("work_rate", backend.rate)
    return Scheduler(backend, clock=clock, sleep=clock.advance, **kw)


def test_every_map_equals_the_whole_shoot_and_small_requests_overtake():
    clock = Clock()
    be = CpuBackend(clock)
    sch = make(clock, be)
    big = small_request(0, 300, 2000, 60, arrival=0.0)
    smalls = [small_request(i, 120, 130, 10, arrival=0.004 * i) for i in range(1, 5)]
    res = sch.run([big] + smalls)
    assert all(r.state is State.DONE for r in res.values())
    for req in [big] + smalls:
        c, e = whole(req)
        assert (res[req.rid].counts == c).all() and res[req.rid].escaped == e
    # continuous batching: the small requests joined launches while the big
    # one was running and finished long before it
    assert all(res[i].finished < res[0].finished for i in range(1, 5))
    mixed = [rids for _, rids in be.launch_log if 0 in rids and len(rids) > 1]
    assert mixed, "no launch carried chunks of several requests"
    assert sch.used == 0 and be.live == 0 and sch.idle()
    summ = latency_summary(res)
    assert summ["completed"] == 5 and summ["p99_s"] >= summ["p50_s"] > 0


def test_admission_respects_the_memory_budget():
    clock = Clock()
    be = CpuBackend(clock)
    reqs = [small_request(i, 128, 256, 15, arrival=0.0, p=64) for i in range(4)]
    fp = footprint_bytes(reqs[0].spec, reqs[0].lenses.n, True)
    sch = make(clock, be, budget_bytes=int(fp * 1.5))
    res = sch.run(reqs)
    assert sch.peak_used <= int(fp * 1.5) and sch.peak_active == 1
    for r in reqs:
        c, e = whole(r)
        assert res[r.rid].state is State.DONE and (res[r.rid].counts == c).all()


def test_request_larger_than_the_budget_fails_cleanly():
    clock = Clock()
    sch = make(clock, CpuBackend(clock), budget_bytes=1000)
    res = sch.run([small_request(0, 64, 64, 5)])
    assert res[0].state is State.FAILED and "budget" in res[0].error


def test_aging_stops_overtaking():
    """A request that does not fit is overtaken by smaller ones only until it
    has waited aging_s; then it blocks the queue until memory frees up."""
    clock = Clock()
    be = CpuBackend(clock, rate=1e6)       # the first request runs ~1.3 s
    first = small_request(0, 128, 512, 20, arrival=0.0, p=64)
    fp_big = footprint_bytes(small_request(1, 128, 128, 20, p=128).spec, 20, True)
    budget = footprint_bytes(first.spec, 20, True) + fp_big - 1     # big does not fit beside first
    big = small_request(1, 128, 128, 20, arrival=0.001, p=128)
    later = [small_request(i, 128, 128, 5, arrival=0.002 + 0.2 * i, p=16) for i in range(2, 30)]
    sch = make(clock, be, budget_bytes=budget, aging_s=0.5)
    res = sch.run([first, big] + later)
    assert all(r.state is State.DONE for r in res.values())
    overtook = [r for r in later if res[r.rid].admitted < res[1].admitted]
    assert overtook, "small requests should backfill while the big one is young"
    # once aged, nothing that arrived after the ageing point was admitted first
    aged_at = big.arrival + 0.5
    assert not any(res[r.rid].admitted < res[1].admitted and r.arrival > aged_at + 1e-9
                   for r in later)


def test_failures_are_isolated():
    clock = Clock()
    be = CpuBackend(clock, fail_admit={1}, fail_finalize={2})
    reqs = [small_request(i, 100, 140, 12, arrival=0.0) for i in range(4)]
    res = make(clock, be).run(reqs)
    assert res[1].state is State.FAILED and "allocation" in res[1].error
    assert res[2].state is State.FAILED and "finalisation" in res[2].error
    for i in (0, 3):
        c, e = whole(reqs[i])
        assert res[i].state is State.DONE and (res[i].counts == c).all()
    assert be.live == 0


def test_failed_launch_fails_only_the_requests_it_carried():
    clock = Clock()
    be = CpuBackend(clock, fail_launch={7})
    first = small_request(0, 100, 300, 12, arrival=0.0)
    doomed = small_request(7, 100, 140, 12, arrival=5.0)     # arrives after request 0 is done
    res = make(clock, be).run([first, doomed])
    assert res[7].state is State.FAILED
    c, e = whole(first)
    assert res[0].state is State.DONE and (res[0].counts == c).all()
    assert be.live == 0


def test_cancel_returns_memory_and_leaves_others_exact():
    clock = Clock()
    be = CpuBackend(clock)
    reqs = [small_request(i, 200, 600, 20, arrival=0.0) for i in range(3)]
    sch = make(clock, be, chunk_evals=128 * 200 * 20)
    for r in reqs:
        sch.submit(r)
    for _ in range(3):
        sch.step()
    assert sch.cancel(1)
    queued = small_request(9, 64, 64, 5, arrival=0.0)
    sch.submit(queued)
    assert sch.cancel(9)
    res = sch.run([])
    assert res[1].state is State.CANCELLED and res[9].state is State.CANCELLED
    for i in (0, 2):
        c, e = whole(reqs[i])
        assert res[i].state is State.DONE and (res[i].counts == c).all()
    assert sch.used == 0 and be.live == 0


def test_checkpoint_and_resume_is_bit_identical():
    clock = Clock()
    be = CpuBackend(clock)
    req = small_request(0, 256, 1000, 25, arrival=0.0)
    sch = make(clock, be, chunk_evals=128 * 256 * 25)
    sch.submit(req)
    for _ in range(4):
        sch.step()
    cp = sch.checkpoint(0)
    assert 0 < cp.next_row < req.spec.n2 and cp.next_row % 128 == 0
    assert sch.results[0].state is State.CANCELLED and be.live == 0
    resumed = MapRequest(0, req.spec, req.lenses, arrival=clock(), resume=cp)
    res = sch.run([resumed])
    c, e = whole(req)
    assert res[0].state is State.DONE and (res[0].counts == c).all() and res[0].escaped == e


def test_duplicate_submission_is_rejected():
    clock = Clock()
    sch = make(clock, CpuBackend(clock))
    r = small_request(0, 64, 64, 5)
    sch.submit(r)
    with pytest.raises(ValueError):
        sch.submit(r)


def test_on_finish_is_called_once_per_request():
    seen = []
    clock = Clock()
    sch = make(clock, CpuBackend(clock), on_finish=lambda r: seen.append((r.rid, r.state)))
    reqs = [small_request(i, 64, 128, 10, arrival=0.001 * i, p=16) for i in range(5)]
    res = sch.run(reqs)
    assert sorted(rid for rid, _ in seen) == sorted(res) == list(range(5))
    assert all(st is State.DONE for _, st in seen)


def tiny_request(rid, n1, n2, arrival):
    """A request whose cost is set by its ray count (10 unit lenses, 16^2 map)."""
    spec = inputs.MapSpec(name=f"t{rid}", kappa=0.45, gamma=0.2, s=0.0, n1=n1, n2=n2, h1=6.0,
                          h2=3.0, p1=16, p2=16, W1=4.0, W2=4.0, n_lens=10, disc_radius=5.0,
                          masses="unit", seed=500 + rid)
    return MapRequest(rid, spec, spec.lenses(), arrival)


def test_small_request_behind_large_ones_finishes_within_two_launches():
    """Smallest remaining work first: a small request that arrives while three
    large ones are active goes into the next launch that starts after it
    arrives and finishes with it (at most max_inflight launches later)."""
    clock = Clock()
    be = CpuBackend(clock, rate=1e6)
    bigs = [tiny_request(i, 200, 1280, 0.0) for i in range(3)]          # 2.56 s of work each
    small = tiny_request(9, 64, 64, 1.0)                                # 0.04 s
    sch = make(clock, be, chunk_evals=128 * 200 * 10, max_inflight=2)  # 0.256 s per launch
    res = sch.run(bigs + [small])
    assert all(r.state is State.DONE for r in res.values())
    for req in bigs + [small]:
        c, e = whole(req)
        assert (res[req.rid].counts == c).all() and res[req.rid].escaped == e
    after = [t for t, _ in be.launch_log if t >= small.arrival]
    first = next(t for t, rids in be.launch_log if 9 in rids)
    assert first == after[0], "the small request missed the first launch after its arrival"
    assert res[9].latency <= 3 * 0.256 + 1e-9
    assert all(res[9].finished < res[i].finished for i in range(3))


def _stream_with_one_large(age_weight):
    clock = Clock()
    be = CpuBackend(clock, rate=1e6)
    big = tiny_request(0, 200, 1000, 0.0)                               # 2 s of work
    smalls = [tiny_request(i, 64, 64, 0.05 * i) for i in range(1, 241)]  # 0.041 s each, load 0.82
    sch = make(clock, be, chunk_evals=0.2e6, age_weight=age_weight)
    res = sch.run([big] + smalls)
    assert all(r.state is State.DONE for r in res.values())
    for req in (big, smalls[0], smalls[-1]):
        c, e = whole(req)
        assert (res[req.rid].counts == c).all() and res[req.rid].escaped == e
    return res, big, smalls


def test_aging_bounds_the_wait_of_a_large_request():
    """Under a steady stream of small requests (82 % load), the large request's
    key (remaining seconds - age_weight * waited) reaches zero after
    remaining / age_weight seconds; from then on no newcomer goes first, so
    it finishes within that time plus its own work plus a launch or two.
    Pure smallest-remaining-first (age_weight = 0) finishes it later."""
    work = 200 * 1000 * 10 / 1e6
    res, big, smalls = _stream_with_one_large(0.25)
    bound = big.arrival + work / 0.25 + work + 2 * 0.2
    assert res[0].finished <= bound, (res[0].finished, bound)
    # while the large request is young the small ones wait for at most the
    # two queued launches (each about one large chunk of 0.256 s) and their own
    young = [res[s.rid].latency for s in smalls if s.arrival < 2.0]
    assert max(young) < 4 * 0.3
    assert np.median([res[s.rid].latency for s in smalls]) < 1.0
    pure, _, _ = _stream_with_one_large(0.0)
    assert pure[0].finished > res[0].finished

"""Continuous-batching server for magnification-map requests.

Requests (a lens field plus kappa, gamma, s, ray grid and map window, as in
the map table of Vernardos & Fluke 2014, Section 3.2.1) arrive over time. The
scheduler:

  * admits a queued request when its device footprint (count map,
    magnification map, lens field and its FP32 copy) fits the free HBM budget
    and an active slot is free; a request that does not fit may be overtaken
    by later ones that do, but only until it has waited `aging_s`;
  * keeps each admitted request's lens field and partial count map resident;
  * cuts requests into chunks of ray rows (multiples of 128 rows) and, at
    every tick, fills one batched persistent launch with about `chunk_evals`
    ray-lens evaluations (and at least `min_launch_rays` rays, so a launch
    holds enough ray cells to fill the device), taking chunks from the active
    requests in order of smallest remaining work first with an aging bound:
    a request's key is its remaining work in seconds minus `age_weight` times
    the time it has waited since arrival. A request that arrives while others
    run joins the very next launch if its key is smallest, and its work
    overlaps with theirs on the device; a request is overtaken by a later
    arrival only while the newcomer's remaining work is smaller than its own
    key, so after waiting remaining / age_weight seconds nothing that arrives
    later goes before it;
  * keeps up to `max_inflight` launches queued on the stream so the device
    never waits for the host, and finalises a request (normalisation and
    statistics) as soon as the launch holding its last chunk has finished;
  * records arrival, admission and completion times for p50/p99 latency and
    maps/hour.

Integer counts over disjoint row ranges add up exactly and no kernel shape or
batching changes a ray's arithmetic, so every map equals the map of the same
request shot alone, bit for bit. A request can be cancelled (its memory is
returned once no launch references it), and checkpointed and resumed from its
partial map and next-row cursor with a bit-identical result.

The device work goes through a backend: `GpuBackend` drives the raylens
C-ABI; tests substitute a CPU backend to exercise the scheduling logic.
"""
from __future__ import annotations

import collections
import dataclasses
import enum
import time
from typing import Callable, Dict, List, Optional

import numpy as np

ROW_ALIGN = 128   # chunk boundaries on multiples of 128 rows (every cell height divides it)


class State(enum.Enum):
    QUEUED = "queued"
    RUNNING = "running"
    DONE = "done"
    FAILED = "failed"
    CANCELLED = "cancelled"


@dataclasses.dataclass
class MapRequest:
    rid: int
    spec: object                  # inputs.MapSpec
    lenses: object                # inputs.LensField (host arrays)
    arrival: float = 0.0          # seconds on the server clock
    precision: str = "fp32c"
    resume: Optional["Checkpoint"] = None


@dataclasses.dataclass
class Checkpoint:
    rid: int
    counts: np.ndarray            # partial int32 map (p2 x p1)
    escaped: int
    next_row: int                 # rows [0, next_row) are in `counts`


@dataclasses.dataclass
class MapResult:
    rid: int
    state: State
    counts: Optional[np.ndarray] = None
    escaped: int = 0
    stats: Optional[dict] = None
    mu: Optional[np.ndarray] = None
    arrival: float = 0.0
    admitted: float = float("nan")
    finished: float = float("nan")
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass
class _Active:
    req: MapRequest
    handle: object
    footprint: int
    next_row: int
    admitted: float
    inflight: int = 0             # launches still holding a chunk of this request
    last_token: object = None
    cancelled: bool = False
    paused: bool = False
    failed: Optional[str] = None


def footprint_bytes(spec, n_lens: int, has_masses: bool) -> int:
    """Device bytes a request holds while active: int32 counts, float32 mu,
    int64 escaped, the FP64 lens field and its FP32 hi/lo copy."""
    pix = spec.p1 * spec.p2
    lens = n_lens * (8 * (3 if has_masses else 2) + 20)
    return 4 * pix + 4 * pix + 8 + lens


class Scheduler:
    def __init__(self, backend, budget_bytes: int, max_active: int = 16,
                 chunk_evals: float = 2.0e11, max_inflight: int = 2, aging_s: float = 5.0,
                 clock: Callable[[], float] = time.perf_counter, keep_mu: bool = False,
                 sleep: Callable[[float], None] = time.sleep,
                 on_finish: Optional[Callable[["MapResult"], None]] = None,
                 min_launch_rays: int = 0, age_weight: float = 0.25,
                 work_rate: float = 8.0e12):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_active = max_active
        self.chunk_evals = chunk_evals           # ray-lens evaluations per launch
        self.min_launch_rays = min_launch_rays   # rays per launch, at least (work permitting)
        self.age_weight = age_weight             # seconds of priority gained per second waited
        self.work_rate = work_rate               # evaluations/s that turn work into seconds
        self.max_inflight = max_inflight
        self.aging_s = aging_s
        self.clock = clock
        self.sleep = sleep
        self.keep_mu = keep_mu
        self.on_finish = on_finish      # called once per request that reaches a final state
        self.t0 = clock()
        self.queue: collections.deque = collections.deque()
        self.active: Dict[int, _Active] = {}
        self.inflight: collections.deque = collections.deque()   # (token, [rids], [last-chunk rids])
        self.results: Dict[int, MapResult] = {}
        self.used = 0
        self.launches = 0
        self.peak_used = 0
        self.peak_active = 0

    # -------------------------------------------------------------- interface
    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: MapRequest) -> None:
        prev = self.results.get(req.rid)
        if req.resume is not None and prev is not None and prev.state is State.CANCELLED:
            del self.results[req.rid]      # resuming a checkpointed request
        if req.rid in self.results or any(r.rid == req.rid for r in self.queue) or req.rid in self.active:
            raise ValueError(f"request {req.rid} already submitted")
        fp = footprint_bytes(req.spec, req.lenses.n, req.lenses.m is not None)
        if fp > self.budget:
            self._record(MapResult(req.rid, State.FAILED, arrival=req.arrival, finished=self.now(),
                                   error=f"footprint {fp} B exceeds the budget {self.budget} B"))
            return
        self.queue.append(req)

    def cancel(self, rid: int) -> bool:
        for r in list(self.queue):
            if r.rid == rid:
                self.queue.remove(r)
                self._record(MapResult(rid, State.CANCELLED, arrival=r.arrival, finished=self.now()))
                return True
        a = self.active.get(rid)
        if a is not None:
            a.cancelled = True
            self._retire_if_idle(a)
            return True
        return False

    def checkpoint(self, rid: int) -> Checkpoint:
        """Stops launching the request, waits for its queued launches, and
        returns its partial map with the next row to shoot; the request ends
        as CANCELLED. If its last chunk was already queued it completes
        instead, and the checkpoint holds the whole map (next_row = n2)."""
        a = self.active[rid]
        a.paused = True
        while a.inflight:
            self._wait_oldest()
        if rid not in self.active:          # it finished while we waited
            r = self.results[rid]
            return Checkpoint(rid, r.counts, r.escaped, a.req.spec.n2)
        counts, esc = self.backend.read_partial(a.handle)
        cp = Checkpoint(rid, counts, esc, a.next_row)
        a.cancelled = True
        self._retire_if_idle(a)
        return cp

    def idle(self) -> bool:
        return not self.queue and not self.active and not self.inflight

    # -------------------------------------------------------------- one tick
    def step(self) -> bool:
        """One scheduling round. Returns True if it did anything."""
        did = self._poll()
        did |= self._admit()
        if len(self.inflight) < self.max_inflight:
            did |= self._launch()
        return did

    def run(self, requests: List[MapRequest], poll_sleep: float = 2e-4) -> Dict[int, MapResult]:
        """Feeds `requests` at their arrival times (server clock) and runs
        until every request has finished."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        while pending or not self.idle():
            now = self.now()
            while pending and pending[0].arrival <= now:
                self.submit(pending.popleft())
            did = self.step()
            if not did:
                if self.inflight:
                    self._wait_oldest(timeout=poll_sleep)
                elif pending:
                    self.sleep(min(poll_sleep * 10, max(1e-6, pending[0].arrival - self.now())))
        return self.results

    # -------------------------------------------------------------- internals
    def _record(self, res: "MapResult") -> None:
        self.results[res.rid] = res
        if self.on_finish is not None:
            self.on_finish(res)

    @staticmethod
    def _evals_per_row(spec) -> int:
        return max(1, spec.n1 * max(spec.n_lens, 1))

    def priority(self, a: "_Active", now: float) -> tuple:
        """Launch order key: remaining work (seconds at work_rate) minus
        age_weight times the time waited since arrival; ties by arrival."""
        remaining = (a.req.spec.n2 - a.next_row) * self._evals_per_row(a.req.spec)
        return (remaining / self.work_rate - self.age_weight * (now - a.req.arrival),
                a.req.arrival, a.req.rid)

    def _admit(self) -> bool:
        did = False
        now = self.now()
        for req in list(self.queue):
            if len(self.active) >= self.max_active:
                break
            fp = footprint_bytes(req.spec, req.lenses.n, req.lenses.m is not None)
            if self.used + fp > self.budget:
                if now - req.arrival > self.aging_s:
                    break       # the head has aged: nobody overtakes it any more
                continue
            self.queue.remove(req)
            try:
                handle = self.backend.admit(req)
            except Exception as exc:   # allocation or upload failure
                self._record(MapResult(req.rid, State.FAILED, arrival=req.arrival,
                                       finished=self.now(), error=repr(exc)))
                continue
            start = 0
            if req.resume is not None:
                self.backend.load_partial(handle, req.resume.counts, req.resume.escaped)
                start = req.resume.next_row
            self.active[req.rid] = _Active(req, handle, fp, start, now)
            self.used += fp
            self.peak_used = max(self.peak_used, self.used)
            self.peak_active = max(self.peak_active, len(self.active))
            did = True
        return did

    def _launch(self) -> bool:
        now = self.now()
        ready = [a for a in self.active.values()
                 if not (a.cancelled or a.failed or a.paused or a.next_row >= a.req.spec.n2)]
        if not ready:
            return False
        ready.sort(key=lambda a: self.priority(a, now))
        # fill one launch per precision: chunks in key order until the launch
        # holds chunk_evals evaluations and min_launch_rays rays
        by_prec: Dict[str, list] = {}
        filled: Dict[str, list] = {}
        for a in ready:
            prec = a.req.precision
            ev, rays = filled.setdefault(prec, [0, 0])
            need_ev = self.chunk_evals - ev
            need_rays = self.min_launch_rays - rays
            if need_ev <= 0 and need_rays <= 0:
                continue
            spec = a.req.spec
            per_row = self._evals_per_row(spec)
            rows = max(-(-int(max(need_ev, 0)) // per_row), -(-int(max(need_rays, 0)) // spec.n1))
            rows = max(ROW_ALIGN, -(-rows // ROW_ALIGN) * ROW_ALIGN)
            rb = a.next_row
            re = min(spec.n2, rb + rows)
            by_prec.setdefault(prec, []).append((a, rb, re))
            filled[prec] = [ev + (re - rb) * per_row, rays + (re - rb) * spec.n1]
        for prec, chunks in by_prec.items():
            try:
                token = self.backend.launch([(a.handle, a.req.spec, rb, re) for a, rb, re in chunks],
                                            prec)
            except Exception as exc:
                # a failing launch fails the requests it carried; nothing of it ran
                for a, _, _ in chunks:
                    a.failed = repr(exc)
                    self._retire_if_idle(a)
                continue
            self.launches += 1
            last = []
            for a, rb, re in chunks:
                a.next_row = re
                a.inflight += 1
                a.last_token = token
                if re >= a.req.spec.n2:
                    last.append(a.req.rid)
            self.inflight.append((token, [a.req.rid for a, _, _ in chunks], last))
        return True

    def _poll(self) -> bool:
        did = False
        while self.inflight and self.backend.done(self.inflight[0][0]):
            self._complete(self.inflight.popleft())
            did = True
        return did

    def _wait_oldest(self, timeout: Optional[float] = None) -> None:
        if not self.inflight:
            return
        if timeout is None:
            self.backend.wait(self.inflight[0][0])
            self._complete(self.inflight.popleft())
        elif self.backend.wait(self.inflight[0][0], timeout=timeout):
            self._complete(self.inflight.popleft())

    def _complete(self, entry) -> None:
        token, rids, last = entry
        for rid in rids:
            a = self.active.get(rid)
            if a is None:
                continue
            a.inflight -= 1
            if a.cancelled or a.failed:
                self._retire_if_idle(a)
            elif rid in last:
                self._finish(a)

    def _finish(self, a: _Active) -> None:
        try:
            counts, esc, stats, mu = self.backend.finalize(a.handle, keep_mu=self.keep_mu)
            res = MapResult(a.req.rid, State.DONE, counts, esc, stats, mu, arrival=a.req.arrival,
                            admitted=a.admitted, finished=self.now())
        except Exception as exc:
            res = MapResult(a.req.rid, State.FAILED, arrival=a.req.arrival, admitted=a.admitted,
                            finished=self.now(), error=repr(exc))
        self._release(a)
        self._record(res)

    def _retire_if_idle(self, a: _Active) -> None:
        if a.inflight or not (a.cancelled or a.failed) or a.req.rid not in self.active:
            return      # still running, memory still referenced by a queued launch, or gone
        state = State.CANCELLED if a.cancelled else State.FAILED
        self._record(MapResult(a.req.rid, state, arrival=a.req.arrival,
                               admitted=a.admitted, finished=self.now(), error=a.failed))
        self._release(a)

    def _release(self, a: _Active) -> None:
        if a.req.rid in self.active:
            del self.active[a.req.rid]
            self.used -= a.footprint
            self.backend.release(a.handle)


def latency_summary(results: Dict[int, MapResult]) -> dict:
    done = [r for r in results.values() if r.state is State.DONE]
    lat = np.array([r.latency for r in done]) if done else np.zeros(0)
    span = (max(r.finished for r in done) - min(r.arrival for r in done)) if done else 0.0
    return {"completed": len(done),
            "failed": sum(r.state is State.FAILED for r in results.values()),
            "cancelled": sum(r.state is State.CANCELLED for r in results.values()),
            "p50_s": float(np.percentile(lat, 50)) if done else None,
            "p99_s": float(np.percentile(lat, 99)) if done else None,
            "mean_s": float(lat.mean()) if done else None,
            "makespan_s": span,
            "maps_per_hour": len(done) * 3600.0 / span if span > 0 else None}


# ---------------------------------------------------------------------------
# GPU backend (raylens C-ABI + torch memory and streams)
# ---------------------------------------------------------------------------

class GpuBackend:
    """Device side of the server, on three streams at the default priority:
    uploads of admitted requests (lens field, zeroed count map), the batched
    launches, and finalisation. The launch stream waits on each upload with
    an event, so an upload never waits for queued launches."""

    def __init__(self, ctx=None, device: int = 0):
        import torch
        from . import raylens as rl

        self.torch = torch
        self.rl = rl
        self.device = device
        self.ctx = ctx if ctx is not None else rl.Context(device)
        self.upload_stream = torch.cuda.Stream(device=device)
        self.launch_stream = torch.cuda.Stream(device=device)
        self.final_stream = torch.cuda.Stream(device=device)

    def admit(self, req):
        torch = self.torch
        with torch.cuda.stream(self.upload_stream):
            L = self.rl.DeviceLenses(req.lenses.x1, req.lenses.x2, req.lenses.m,
                                     device=f"cuda:{self.device}")
            counts, esc = self.ctx.new_map(req.spec)
            ready = torch.cuda.Event()
            ready.record(self.upload_stream)
        self.launch_stream.wait_event(ready)
        return {"L": L, "counts": counts, "esc": esc, "spec": req.spec}

    def load_partial(self, h, counts: np.ndarray, escaped: int) -> None:
        with self.torch.cuda.stream(self.launch_stream):
            h["counts"].copy_(self.torch.from_numpy(np.ascontiguousarray(counts, np.int32)))
            h["esc"].fill_(int(escaped))

    def read_partial(self, h):
        self.launch_stream.synchronize()
        return h["counts"].cpu().numpy(), int(h["esc"].item())

    def launch(self, chunks, precision):
        items = [(h["L"], spec, h["counts"], h["esc"], rb, re) for h, spec, rb, re in chunks]
        self.ctx.shoot_batch(items, precision, stream=self.launch_stream)
        ev = self.torch.cuda.Event()
        ev.record(self.launch_stream)
        return ev

    def done(self, token) -> bool:
        return token.query()

    def wait(self, token, timeout: Optional[float] = None) -> bool:
        if timeout is None:
            token.synchronize()
            return True
        end = time.perf_counter() + timeout
        while time.perf_counter() < end:
            if token.query():
                return True
            time.sleep(timeout / 20)
        return token.query()

    def finalize(self, h, keep_mu: bool = False):
        """Called once the launch holding the request's last chunk has
        completed, so the final stream needs no wait on the launch stream (a
        wait there would also wait for every launch queued after it)."""
        torch = self.torch
        s = self.final_stream
        spec = h["spec"]
        with torch.cuda.stream(s):
            mu = self.ctx.normalise(h["counts"], spec, stream=s) if keep_mu else None
            st = self.ctx.stats(h["counts"], h["esc"], spec, stream=s)   # synchronises s
            counts = h["counts"].cpu().numpy()
            mu_h = mu.cpu().numpy() if mu is not None else None
        return counts, int(st["escaped"]), st, mu_h

    def release(self, h) -> None:
        h.clear()


def gpu_budget_bytes(fraction: float = 0.5, device: int = 0) -> int:
    import torch
    free, total = torch.cuda.mem_get_info(device)
    return int(free * fraction)

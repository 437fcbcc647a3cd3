"""Continuous-batching server for parameter-sweep simulations.

Requests (box size, particles, step count, precision class) arrive over time.
The server keeps every admitted request's state resident on the GPU and
advances all of them together: between chunks of steps it admits new
arrivals as slots and HBM budget free up (admission by ``lb_footprint_bytes``
plus the particle tables), groups the live requests by storage precision,
and advances each group with one batched launch per kernel
(``lb_batch_step``), one group after the other (optionally each group on a
stream of its own).  A request whose steps are done is read back (FP64
totals and particle states) and its memory released at once.

Time-to-result = completion time - arrival time.  Each result is identical
to the same request run alone (the batched step is bitwise equal to the
single-box step).
"""
import faulthandler
import heapq
import math
import time

from . import inputs as I
from . import lb


def request_bytes(spec):
    """HBM footprint of one request: lattice arena plus particle tables."""
    n = lb.footprint_bytes(spec["shape"], spec["precision"])
    cols = spec.get("colloids", [])
    if cols:
        r = max(c["radius"] for c in cols)
        side = 2 * math.ceil(r) + 8
        bb = min(side, spec["shape"][0]) * min(side, spec["shape"][1]) * min(side, spec["shape"][2])
        ro, ri = r + 1.5, max(0.0, r - 0.5)
        lcap = int(10.0 * 4.0 / 3.0 * math.pi * (ro ** 3 - ri ** 3)) + 512
        per = 512 + lcap * 5 + bb * 4 + (bb // 256 + 1) * 68 + (lcap // 512 + 1) * 224
        n += len(cols) * per  # tables sized for exactly the request's particles
    return n


class Server:
    """One GPU; ``budget_bytes`` caps the resident state, ``max_slots`` the
    number of live requests, ``chunk`` the steps taken between admission
    points.  Boxes of precision p live on ``streams[p]`` if given, else on
    ``stream``."""

    def __init__(self, budget_bytes, max_slots=256, chunk=200, stream=None, collect=None,
                 streams=None):
        self.collect = collect  # optional box -> dict, read on retirement
        self.peak_used = 0
        self.peak_live = 0
        self.budget = int(budget_bytes)
        self.max_slots = max_slots
        self.chunk = chunk
        self.stream = stream
        self.streams = dict(streams or {})
        self.used = 0
        self.live = []        # dicts: id, box, spec, remaining, arrival, bytes
        self.queue = []       # (arrival, seq, id, spec) waiting for admission
        self.done = {}        # id -> result dict
        self.seq = 0
        self.lattice_updates = 0

    def submit(self, rid, spec, arrival):
        heapq.heappush(self.queue, (arrival, self.seq, rid, spec))
        self.seq += 1

    def _admit(self, now):
        while self.queue and self.queue[0][0] <= now and len(self.live) < self.max_slots:
            arrival, _, rid, spec = self.queue[0]
            need = request_bytes(spec)
            if need > self.budget:
                heapq.heappop(self.queue)
                self.done[rid] = dict(error="request larger than the HBM budget", arrival=arrival,
                                      finished=now)
                continue
            if self.used + need > self.budget:
                break  # wait for memory to free up (first come, first served)
            heapq.heappop(self.queue)
            box = lb.from_spec(spec, stream=self._stream_of(spec["precision"]),
                               max_colloids=max(1, len(spec.get("colloids", []))))
            self.used += need
            self.peak_used = max(self.peak_used, self.used)
            self.live.append(dict(id=rid, box=box, spec=spec, remaining=int(spec["steps"]),
                                  arrival=arrival, bytes=need, admitted=now))
            self.peak_live = max(self.peak_live, len(self.live))

    def _stream_of(self, precision):
        return self.streams.get(precision, self.stream)

    def _advance(self):
        k = min(self.chunk, min(r["remaining"] for r in self.live))
        groups = {}
        for r in self.live:
            groups.setdefault(r["spec"]["precision"], []).append(r)
        for reqs in groups.values():
            lb.batch_step([r["box"] for r in reqs], k)
        for r in self.live:
            r["remaining"] -= k
            s = r["spec"]["shape"]
            self.lattice_updates += k * s[0] * s[1] * s[2]
        return k

    def _retire(self, now_fn):
        keep = []
        for r in self.live:
            if r["remaining"] > 0:
                keep.append(r)
                continue
            tot, cols = r["box"].observables(check=False)
            t = now_fn()
            self.done[r["id"]] = dict(totals=tot, colloids=cols, arrival=r["arrival"],
                                      admitted=r["admitted"], finished=t,
                                      time_to_result=t - r["arrival"])
            if self.collect:
                self.done[r["id"]].update(self.collect(r["box"]))
            r["box"].close()
            self.used -= r["bytes"]
        self.live = keep

    def run(self, clock=None, idle_sleep=0.001):
        """Serve until the queue and the slots are empty.  ``clock`` returns
        the current time on the arrival timeline (default: wall clock from
        the first call)."""
        t0 = time.perf_counter()
        now_fn = clock or (lambda: time.perf_counter() - t0)
        while self.queue or self.live:
            now = now_fn()
            self._admit(now)
            if not self.live:
                if self.queue:
                    wait = self.queue[0][0] - now_fn()
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                    else:
                        time.sleep(idle_sleep)
                continue
            self._advance()
            self._retire(now_fn)
        return self.done


def replay(trace, budget_bytes, max_slots=256, chunk=200, step_scale=1.0, stream=None,
           limit=None, collect=None, streams=None):
    """Serve a Poisson trace from ``inputs.serving_trace`` on the wall clock.
    step_scale shortens every request (for bounded runs).  Returns
    (results by request id, summary with p50/p99 time-to-result and
    sustained MLUPS)."""
    faulthandler.enable()  # a native crash prints the Python stack
    srv = Server(budget_bytes, max_slots=max_slots, chunk=chunk, stream=stream, collect=collect,
                 streams=streams)
    reqs = trace[:limit] if limit else trace
    specs = []
    for i, r in enumerate(reqs):
        spec = I.serving_request(r)
        spec["steps"] = max(2, int(round(r["steps"] * step_scale)))
        specs.append(spec)
        srv.submit(i, spec, r["t"])
    t0 = time.perf_counter()
    res = srv.run()
    wall = time.perf_counter() - t0
    ttr = sorted(v["time_to_result"] for v in res.values() if "time_to_result" in v)

    def pct(q):
        if not ttr:
            return None
        i = min(len(ttr) - 1, max(0, int(math.ceil(q * len(ttr))) - 1))
        return ttr[i]

    summary = dict(requests=len(reqs), completed=len(ttr), p50_s=pct(0.50), p99_s=pct(0.99),
                   wall_s=wall, mlups=srv.lattice_updates / wall / 1e6,
                   lattice_updates=srv.lattice_updates, peak_bytes=srv.peak_used,
                   peak_live=srv.peak_live, budget_bytes=srv.budget)
    return res, summary, specs

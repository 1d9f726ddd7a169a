"""Continuous-batching solve server on one GPU.

Requests (a problem key and a right-hand side) arrive over time.  Every
problem's hierarchy is built once, sparsified, and kept resident.  Problems
are grouped by size onto a few HIP streams (as many as the runtime has
hardware queues by default), so that work for problems of different sizes
overlaps on the device and the launches of a small problem never wait in a
hardware queue behind the long kernels of a large one.  A problem with waiting requests gets a batch engine (``amg_batch``
in the C ABI): up to ``slots`` right-hand sides are solved together by PCG,
one CG recurrence per slot, and a slot that finishes takes the next waiting
request at the next iteration while the other slots keep iterating.  A
request's result does not depend on which requests it shared the engine
with (every kernel treats each slot with the same operations in the same
order), so it is the same alone and in the mix.

Admission is by device bytes: hierarchies are always resident; an engine is
created only if the bytes allocated by all handles plus the engine's own
(``amg_batch_bytes``) stay within the HBM budget, after destroying idle
engines (least recently used first) if needed; otherwise its requests wait.

This module is scheduling only: every solve step runs in the library's
kernels.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

from . import amg


@dataclass
class Request:
    rid: int
    key: str
    b: object                 # float64 CUDA tensor of n entries
    arrival: float            # seconds after the start of the run
    x: object = None          # float64 CUDA tensor receiving the solution
    admitted: float | None = None
    done: float | None = None
    iters: int = 0
    relres: float | None = None
    status: int | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class ServeStats:
    makespan: float = 0.0
    steps: int = 0
    engines_created: int = 0
    engines_evicted: int = 0
    max_live_engines: int = 0
    peak_bytes: int = 0
    waits_for_budget: int = 0
    latencies: list = field(default_factory=list)
    occupancy: dict = field(default_factory=dict)    # key -> [occupied slot-steps, steps]


class SolveServer:
    def __init__(self, problems: dict, hbm_budget: int, slots: int = 16, precision: int = 32,
                 tol: float = 1e-10, maxit: int = 300, gamma: float = 0.01, step_target_s: float = 1.5e-3,
                 max_iters_per_step: int = 8, graphs: bool = True, stream_groups: int = 4):
        torch = amg._torch()
        self.slots, self.precision, self.tol, self.maxit = int(slots), int(precision), float(tol), int(maxit)
        # iterations per engine step: as many as fit in step_target_s (so that
        # small problems are not bound by host round trips), at most
        # max_iters_per_step (new requests join only at step boundaries)
        self.step_target_s, self.max_iters = float(step_target_s), int(max_iters_per_step)
        self.graphs = bool(graphs)
        self.iter_time: dict = {}
        self.budget = int(hbm_budget)
        self.hier, self.streams = {}, {}
        by_size = sorted(problems, key=lambda k: (problems[k].n, k))
        groups = max(1, min(int(stream_groups), len(by_size)))
        pool = [torch.cuda.Stream() for _ in range(groups)]
        for rank, key in enumerate(by_size):
            s = pool[rank * groups // len(by_size)]
            with torch.cuda.stream(s):
                h = amg.Hierarchy(problems[key])
                if gamma > 0:
                    h.sparsify(gamma, 2)
            self.hier[key], self.streams[key] = h, s
        torch.cuda.synchronize()
        self.engines: dict = {}
        self.last_used: dict = {}
        self.stats = ServeStats()
        need = self.device_bytes() + max(h.batch_bytes(self.slots, self.precision) for h in self.hier.values())
        if need > self.budget:
            raise ValueError(f"HBM budget {self.budget} B cannot hold the hierarchies and the largest engine "
                             f"({need} B)")

    # -- memory ----------------------------------------------------------------
    def device_bytes(self) -> int:
        return sum(h.device_bytes() for h in self.hier.values())

    def _idle(self, key) -> bool:
        return all(s == amg.Batch.FREE for s in self.engines[key].states())

    def _admit(self, key):
        """The engine of `key`, created if the budget allows (evicting idle
        engines, least recently used first); None if it has to wait."""
        if key in self.engines:
            return self.engines[key]
        h = self.hier[key]
        need = h.batch_bytes(self.slots, self.precision)
        victims = sorted((k for k in self.engines if self._idle(k)), key=lambda k: self.last_used[k])
        while self.device_bytes() + need > self.budget and victims:
            self._drop(victims.pop(0))
            self.stats.engines_evicted += 1
        if self.device_bytes() + need > self.budget:
            self.stats.waits_for_budget += 1
            return None
        torch = amg._torch()
        with torch.cuda.stream(self.streams[key]):
            self.engines[key] = h.batch(self.slots, self.precision, self.tol, self.maxit, self.graphs)
        self.last_used[key] = time.perf_counter()
        self.stats.engines_created += 1
        self.stats.max_live_engines = max(self.stats.max_live_engines, len(self.engines))
        self.stats.peak_bytes = max(self.stats.peak_bytes, self.device_bytes())
        return self.engines[key]

    def _drop(self, key):
        self.engines.pop(key).close()
        self.last_used.pop(key, None)

    def close_engines(self):
        for key in list(self.engines):
            self._drop(key)

    def close(self):
        self.close_engines()
        for h in self.hier.values():
            h.close()
        self.hier = {}

    # -- serving -----------------------------------------------------------------
    def _after_caller(self):
        """Orders every engine stream after the work the caller has enqueued so
        far on its current stream (the requests' right-hand sides and solution
        buffers are produced there); the streams' copies read b and write x."""
        caller = amg._torch().cuda.current_stream()
        for s in self.streams.values():
            s.wait_stream(caller)

    def run(self, requests) -> ServeStats:
        """Serves `requests` (their `arrival` times are honoured in real time;
        all zeros = everything queued at once).  Each request's `x` must be
        a preallocated float64 CUDA tensor; on return it holds the solution
        and the request its timing and status."""
        torch = amg._torch()
        self._after_caller()
        self.stats = ServeStats()
        order = sorted(requests, key=lambda r: (r.arrival, r.rid))
        queues = collections.defaultdict(collections.deque)
        owner = {}                       # (key, slot) -> request
        in_flight = {}                   # key -> (launch time, iterations)
        remaining, nxt = len(order), 0
        t0 = time.perf_counter()
        while remaining:
            now = time.perf_counter() - t0
            while nxt < len(order) and order[nxt].arrival <= now:
                queues[order[nxt].key].append(order[nxt])
                nxt += 1
            for key, q in queues.items():
                if not q:
                    continue
                eng = self._admit(key)
                if eng is None:
                    continue
                free = int((eng.states() == amg.Batch.FREE).sum())
                while q and free:
                    r = q.popleft()
                    owner[(key, eng.submit(r.b))] = r
                    r.admitted = now
                    free -= 1
            for key, eng in self.engines.items():
                if key in in_flight:
                    continue
                est = self.iter_time.get(key)
                iters = 1 if est is None else max(1, min(self.max_iters, int(self.step_target_s / est)))
                busy = int(((eng.states() == amg.Batch.SUBMITTED) | (eng.states() == amg.Batch.ITERATING)).sum())
                if eng.step(iters):
                    occ = self.stats.occupancy.setdefault(key, [0, 0])
                    occ[0] += busy * iters
                    occ[1] += iters
                    in_flight[key] = (time.perf_counter(), iters)
                    self.last_used[key] = time.perf_counter()
                    self.stats.steps += 1
            progressed = False
            for key in list(in_flight):
                eng = self.engines[key]
                fin = eng.poll(wait=False)
                if fin is None:
                    continue
                t_launch, iters = in_flight.pop(key)
                per = (time.perf_counter() - t_launch) / iters
                old = self.iter_time.get(key)
                self.iter_time[key] = per if old is None else 0.5 * (old + per)
                progressed = True
                t_done = time.perf_counter() - t0
                for slot in fin:
                    r = owner.pop((key, slot))
                    r.iters, r.relres, r.status = eng.collect(slot, r.x)
                    r.done = t_done
                    remaining -= 1
            if not progressed:
                if not in_flight and nxt < len(order) and not any(queues.values()):
                    wait = order[nxt].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(wait)
                else:
                    time.sleep(0)
        torch.cuda.synchronize()
        self.stats.makespan = time.perf_counter() - t0
        self.stats.latencies = [r.latency for r in requests]
        return self.stats

    def run_sequential(self, requests, method=amg.PCG, precision=64) -> ServeStats:
        """Baseline without batching: one solve at a time in arrival order
        (single right-hand side amg_solve), honouring arrival times."""
        torch = amg._torch()
        self.close_engines()
        self._after_caller()
        self.stats = ServeStats()
        order = sorted(requests, key=lambda r: (r.arrival, r.rid))
        t0 = time.perf_counter()
        for r in order:
            wait = r.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            r.admitted = time.perf_counter() - t0
            h = self.hier[r.key]
            with torch.cuda.stream(self.streams[r.key]):
                r.x.zero_()
                res = h.solve(r.b, r.x, method=method, tol=self.tol, maxit=self.maxit, precision=precision)
            r.iters, r.relres, r.status = res.iters, res.relres, res.status
            r.done = time.perf_counter() - t0
            self.stats.steps += res.iters
        torch.cuda.synchronize()
        self.stats.makespan = time.perf_counter() - t0
        self.stats.latencies = [r.latency for r in requests]
        return self.stats


def percentile(values, q: float) -> float:
    """q-th percentile (0..100) by linear interpolation between order statistics."""
    v = sorted(values)
    if not v:
        return float("nan")
    pos = (len(v) - 1) * q / 100.0
    lo = int(pos)
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (pos - lo)

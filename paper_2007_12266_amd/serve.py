"""Continuous-batching solve server for colour-LBM solves on one GPU.

Requests (a rock sub-volume and its fluid parameters: a steady-state solve with periodic
boundaries and a body force, or a displacement solve driven by pressure or flux faces at z)
arrive over time. The server
  * computes each request's exact device footprint on a CPU worker (host pre-pass) and builds
    its domain there once the footprint fits the HBM budget (requests are taken in arrival
    order; a request that does not fit waits, and so do the ones behind it);
  * admits built domains into one pool at chunk boundaries, so work that arrives while others
    run shares the batched launches of the next chunk;
  * advances the pool in chunks of `chunk` steps and, every `check_every` steps of a member's
    own count, tests the steady-state criterion |Sw(t) - Sw(t - check_every)| < tol (Sw the
    mean of (1 + phi)/2, FP64 reduction), stopping at `max_steps`;
  * retires finished members, frees their memory and reports latency (completion - arrival).

Every member's arithmetic is that of a solo run (pool members are bitwise identical to solo
domains), so a request's result does not depend on what else is being served. The flow control
is the paper's steady-state loop (analysis at an interval, convergence over an interval, step
ceiling) with the saturation change in place of the capillary-number change; a displacement
solve usually runs to its step ceiling (its injection length), or stops early once the
saturation no longer changes.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import time
from typing import Callable, List, Optional

import numpy as np

from . import lbm


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the start of the run
    problem: object                # inputs.Problem
    max_steps: int = 20000
    check_every: int = 1000
    tol: float = 1e-5


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    completed: float
    steps: int
    converged: bool
    n_pore: int
    final: dict
    state: Optional[bytes] = None

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


def _check_due(steps: int, check_every: int) -> bool:
    return steps > 0 and steps % check_every == 0


class Server:
    def __init__(self, hbm_budget: int, precision: int = lbm.FP32_MIXED, chunk: int = 200,
                 graph_chunk: int = 100, max_slots: int = 64, workers: int = 4,
                 keep_state: bool = False, stream=None, group_bytes: int = 256 << 20):
        if chunk % graph_chunk or graph_chunk % 2:
            raise ValueError("chunk must be a multiple of an even graph_chunk")
        self.budget = int(hbm_budget)
        self.precision = precision
        self.chunk = chunk
        self.pool = lbm.Pool(self.budget, precision=precision, max_slots=max_slots,
                             chunk_steps=graph_chunk, stream=stream)
        # Members run in cache groups of about the last-level cache (256 MB Infinity Cache on
        # MI355X) inside each captured chunk; results do not depend on it.
        self.pool.set_group_bytes(group_bytes)
        self.workers = cf.ThreadPoolExecutor(max_workers=workers)
        self.keep_state = keep_state

    def close(self):
        self.pool.close()
        self.workers.shutdown(wait=True)

    def _footprint(self, req: Request) -> int:
        return lbm.footprint(req.problem, self.precision)

    def _build(self, req: Request) -> lbm.Domain:
        return lbm.Domain(req.problem, precision=self.precision, allocator="hip")

    def run(self, requests: List[Request], realtime: bool = True,
            on_result: Optional[Callable[[Result], None]] = None) -> List[Result]:
        """Serve `requests`; with realtime=False every request is taken to have arrived.
        `on_result`, if given, is called with each result as it completes."""
        for r in requests:
            if r.check_every % self.chunk:
                raise ValueError("check_every must be a multiple of the chunk")
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else (lambda: float("inf"))
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        arrived = collections.deque()          # waiting for a footprint / the budget
        sizing = {}                            # rid -> future of footprint
        building = {}                          # rid -> (future of Domain, bytes)
        ready = collections.deque()            # (req, dom, bytes) built, waiting for a slot
        live = {}                              # slot -> [req, dom, bytes, admitted, steps, sw]
        reserved = 0
        results = []
        while pending or arrived or building or ready or live:
            now = clock()
            while pending and pending[0].arrival <= now:
                req = pending.popleft()
                arrived.append(req)
                sizing[req.rid] = self.workers.submit(self._footprint, req)
            # Build in arrival order while the budget allows.
            while arrived and sizing[arrived[0].rid].done():
                req = arrived[0]
                need = sizing[req.rid].result()
                if need > self.budget:
                    raise RuntimeError("request %d needs %d bytes, more than the budget"
                                       % (req.rid, need))
                if reserved + need > self.budget:
                    break
                arrived.popleft()
                del sizing[req.rid]
                reserved += need
                building[req.rid] = (req, self.workers.submit(self._build, req), need)
            for rid in [k for k, (_, fut, _) in building.items() if fut.done()]:
                req, fut, need = building.pop(rid)
                ready.append((req, fut.result(), need))
            # Admit at the chunk boundary (the pool's step count is always even here).
            while ready:
                req, dom, need = ready[0]
                try:
                    slot = self.pool.admit(dom)
                except lbm.LbmError as e:
                    if e.status in (lbm.LBM_ERR_OOM,):
                        break
                    raise
                ready.popleft()
                live[slot] = [req, dom, need, clock() if realtime else 0.0, 0, None]
            if not live:
                if not (pending or arrived or building or ready):
                    break
                time.sleep(0.0005)
                continue
            self.pool.step(self.chunk)
            due = []
            for slot, m in live.items():
                m[4] += self.chunk
                if _check_due(m[4], m[0].check_every) or m[4] >= m[0].max_steps:
                    due.append(slot)
            if not due:
                continue
            reds = self.pool.reduce()
            for slot in due:
                req, dom, need, admitted, steps, last_sw = live[slot]
                r = reds[slot]
                converged = (last_sw is not None and _check_due(steps, req.check_every)
                             and abs(r["sw"] - last_sw) < req.tol)
                if _check_due(steps, req.check_every):
                    live[slot][5] = r["sw"]
                if converged or steps >= req.max_steps or r["unstable"]:
                    self.pool.retire(slot)
                    done = clock() if realtime else 0.0
                    state = dom.save() if self.keep_state else None
                    results.append(Result(req.rid, req.arrival, admitted, done, steps,
                                          bool(converged), dom.n_pore, r, state))
                    if on_result:
                        on_result(results[-1])
                    dom.close()
                    reserved -= need
                    del live[slot]
        return sorted(results, key=lambda x: x.rid)


def solve_alone(req: Request, precision: int, chunk: int = 200) -> Result:
    """The same solve with a single domain stepped on its own (no pool), for comparison."""
    dom = lbm.Domain(req.problem, precision=precision, allocator="hip")
    steps, last_sw = 0, None
    while True:
        dom.step(chunk)
        steps += chunk
        if not (_check_due(steps, req.check_every) or steps >= req.max_steps):
            continue
        r = dom.reduce()
        converged = (last_sw is not None and _check_due(steps, req.check_every)
                     and abs(r["sw"] - last_sw) < req.tol)
        if _check_due(steps, req.check_every):
            last_sw = r["sw"]
        if converged or steps >= req.max_steps or r["unstable"]:
            res = Result(req.rid, req.arrival, 0.0, 0.0, steps, bool(converged), dom.n_pore, r,
                         dom.save())
            dom.close()
            return res


def fifo_baseline(requests: List[Request], precision: int = lbm.FP64, chunk: int = 1000,
                  on_result: Optional[Callable[[Result], None]] = None) -> List[Result]:
    """One request at a time in arrival order on the plain path (no pool), in real time."""
    t0 = time.perf_counter()
    out = []
    for req in sorted(requests, key=lambda r: (r.arrival, r.rid)):
        wait = req.arrival - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        start = time.perf_counter() - t0
        res = solve_alone(req, precision, chunk)
        res.admitted = start
        res.completed = time.perf_counter() - t0
        res.state = None
        out.append(res)
        if on_result:
            on_result(res)
    return out


def poisson_trace(count: int, rate: float, seed: int, make_problem) -> List[Request]:
    """`count` requests with exponential inter-arrival times of mean 1/rate (seeded);
    make_problem(k) builds request k's problem."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    return [Request(k, float(t[k]), make_problem(k)) for k in range(count)]


def latency_stats(results: List[Result]) -> dict:
    lat = np.array([r.latency for r in results])
    first = min(r.arrival for r in results)
    last = max(r.completed for r in results)
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "solves_per_s": len(results) / (last - first),
            "converged": int(sum(r.converged for r in results)), "count": len(results)}

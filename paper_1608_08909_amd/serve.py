"""Serving loop over the layout pool: continuous batching of layout requests.

Requests arrive over time (each with its graph, k and sweep count).  The loop
admits arrived requests while the pool's arena has room (admission by device
memory budget), prepares each newly admitted batch on a second stream while
the already-running graphs sweep on the first, and retires a graph as soon as
its sweep count is reached or its stop test (Algorithm 1's relative
positional change, when the request sets a tolerance) has fired (its stress
and layout are read, its slot freed).
Graphs join and leave between sweep quanta, so the device always sweeps every
graph that is ready, whatever its size or arrival time.

Every step runs in the library's kernels; this module only schedules calls.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np
import torch

from . import ssm


@dataclasses.dataclass
class Request:
    rid: int
    graph: object  # graphs.CSR
    k: int
    arrival: float  # seconds after the start of the stream
    sweeps: int = 200
    first: int = 0
    tol: float = 0.0  # Algorithm 1's stop test (0: run `sweeps` sweeps)
    # filled by the loop
    slot: int = -1
    done: int = 0  # sweeps enqueued
    sweeps_run: int = 0  # sweeps the layout took (fewer than `sweeps` when the stop test fired)
    admitted: float = float("nan")
    finished: float = float("nan")
    stress: float = float("nan")
    layout: torch.Tensor | None = None
    status: str = "pending"


@dataclasses.dataclass
class Report:
    requests: list
    wall_s: float
    rounds: int
    prepares: int
    peak_active: int
    peak_bytes: int
    host_s: dict  # host time of the loop's phases: admission, sweep enqueue, preparation, retirement, waiting

    def completed(self):
        return [r for r in self.requests if r.status == "done"]

    def latencies_ms(self):
        return np.array([(r.finished - r.arrival) * 1e3 for r in self.completed()])


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process with `rate` requests per second."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def serve(requests, pool_bytes: int, quantum: int = 25, warm: int = 1, max_prepare: int = 1024,
          first_prepare: int = 128, prep_quantum: int = 100, keep_layouts: bool = False,
          clock=time.perf_counter) -> Report:
    """Runs the stream to completion and returns the per-request record.
    While nothing is running yet, a preparation batch holds at most
    `first_prepare` requests, so that sweeping starts early; later batches
    (prepared while others sweep) hold up to `max_prepare`.  A round that
    prepares a batch first queues `prep_quantum` sweeps of the running
    graphs (enough to keep the device busy during the preparation), other
    rounds `quantum`."""
    pool = ssm.Pool(pool_bytes)
    s_sweep = torch.cuda.Stream()
    s_prep = torch.cuda.Stream()
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    waiting = collections.deque()
    active: dict[int, Request] = {}
    rounds = prepares = peak_active = peak_bytes = 0
    host = dict.fromkeys(["admit", "sweep", "prepare", "retire", "wait"], 0.0)
    t0 = clock()
    while pending or waiting or active:
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            waiting.append(pending.popleft())
        # admission: as many arrived requests as the arena holds
        ta = clock()
        new = []
        cap_new = max_prepare if active else min(max_prepare, first_prepare)
        while waiting and len(new) < cap_new:
            r = waiting[0]
            try:
                slot = pool.add(r.graph, r.k, r.first, r.sweeps)
            except ssm.SSMError as e:  # a graph the pool cannot take at all
                waiting.popleft()
                r.status, r.finished = f"rejected:{e.status}", clock() - t0
                continue
            if slot is None:
                if not active and not new:  # larger than the whole arena
                    waiting.popleft()
                    r.status, r.finished = "rejected:capacity", clock() - t0
                    continue
                break
            waiting.popleft()
            if r.tol > 0:
                pool.set_tol(slot, r.tol)
            r.slot, r.admitted, r.status = slot, clock() - t0, "admitted"
            new.append(r)
        peak_bytes = max(peak_bytes, pool.usage()[0])
        tb = clock()
        host["admit"] += tb - ta
        # one sweep quantum for the running graphs, overlapped with the
        # preparation of the new ones
        if active:
            q = prep_quantum if new else quantum
            with torch.cuda.stream(s_sweep):
                pool.sweep(list(active), q)
            for r in active.values():
                r.done = min(r.sweeps, r.done + q)
            rounds += 1
        tc = clock()
        host["sweep"] += tc - tb
        if new:
            with torch.cuda.stream(s_prep):
                pool.prepare([r.slot for r in new], warm)
            prepares += 1
            for r in new:
                info = pool.info(r.slot)
                if info["state"] != ssm.POOL_READY:
                    r.status, r.finished = f"failed:{info['fail']}", clock() - t0
                    pool.remove(r.slot)
                    continue
                r.done = min(r.sweeps, warm)
                active[r.slot] = r
        peak_active = max(peak_active, len(active))
        td = clock()
        host["prepare"] += td - tc
        # graphs whose stop test has fired take no more sweeps (the query
        # waits for the sweeps queued so far)
        tol_slots = [s for s, r in active.items() if r.tol > 0 and r.done < r.sweeps]
        if tol_slots:
            with torch.cuda.stream(s_sweep):
                ran = pool.stopped(tol_slots)
            for s, v in zip(tol_slots, ran):
                if v >= 0:
                    active[s].done = active[s].sweeps
                    active[s].sweeps_run = int(v)
        # retire the graphs whose sweep count is reached
        fin = [s for s, r in active.items() if r.done >= r.sweeps]
        if fin:
            with torch.cuda.stream(s_sweep):
                st = pool.stress(fin)
                t_done = clock() - t0
                for s, v in zip(fin, st):
                    r = active[s]
                    if r.sweeps_run == 0:
                        r.sweeps_run = r.sweeps
                    if keep_layouts:
                        r.layout = pool.layout(s, r.graph.n)
                    r.stress, r.finished, r.status = float(v), t_done, "done"
                if keep_layouts:
                    s_sweep.synchronize()  # the copies are done before the slots are reused
                for s in fin:
                    del active[s]
                    pool.remove(s)
        te = clock()
        host["retire"] += te - td
        if not active and not new and not waiting and pending:
            wait = pending[0].arrival - (clock() - t0)
            if wait > 0:
                time.sleep(wait)
            host["wait"] += clock() - te
    torch.cuda.synchronize()
    wall = clock() - t0
    pool.close()
    return Report(list(requests), wall, rounds, prepares, peak_active, peak_bytes, host)

"""Continuous batching of independent DPD replicas.

A stream of requests (arrival time, box, chain, step count, seed) is served by
one replica batch (dpd_batch_*): requests are admitted in arrival order as soon
as their device footprint fits the memory budget, every resident replica
advances by windows of K steps (one captured HIP graph per window), and a
finished replica is retired at the end of its window and freed while the next
one runs.  The systems for newly arrived requests (and their initial forces)
are created while a window runs on the GPU, and admitted before the next one.

`serve_one_at_a_time` replays the same stream with each replica stepped alone
by plain dpd_step, first come first served, as the baseline.

Times are host monotonic seconds from the start of the replay; a request's
latency is its completion time minus its arrival time.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass

import numpy as np

from . import dpd, workloads


@dataclass
class Record:
    rid: int
    arrival: float
    n: int
    steps: int
    admitted: float = float("nan")
    done: float = float("nan")

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def _summary(records, t_end: float, extra: dict) -> dict:
    lat = np.array([r.latency for r in records])
    ps = float(sum(r.n * r.steps for r in records))
    span = t_end
    out = {"requests": len(records), "makespan_s": span,
           "particle_steps": ps,
           "particle_steps_per_s": ps / span if span > 0 else float("nan"),
           "replica_steps_per_s": float(sum(r.steps for r in records)) / span,
           "latency_p50_s": float(np.percentile(lat, 50)),
           "latency_p99_s": float(np.percentile(lat, 99)),
           "latency_max_s": float(lat.max())}
    out.update(extra)
    return out


def serve_batched(requests, budget_bytes: int, window: int = 100, max_replicas: int = 1024,
                  variant: int = -1, cell_capacity: int = 0, make=workloads.replica,
                  stream=None, realtime: bool = True, autotune_at: int = 64,
                  autotune_window: int = 20):
    """Serves `requests` (workloads.Request, ascending arrival) through one batch.

    The first time `autotune_at` replicas are resident the batch's brick shape
    is autotuned (a few short windows of real steps; 0 disables it).  Returns
    (records, summary).  With realtime=False every request is taken as arrived
    at time 0 (a throughput run)."""
    batch = dpd.Batch(budget_bytes, max_replicas, stream=stream, variant=variant)
    queue = deque(requests)
    prepared = deque()          # (record, system, footprint) created, not yet admitted
    slot_of = {}                # slot -> (record, system, footprint)
    records = []
    used = 0                    # bytes of prepared + resident systems
    host = {"prepare": 0.0, "admit": 0.0, "advance": 0.0, "poll": 0.0, "retire": 0.0}
    tuned = {"variant": None, "ms_per_step": None}
    t0 = time.perf_counter()

    def now():
        return time.perf_counter() - t0

    class _clock:
        # Host seconds spent per phase of the loop.
        def __init__(self, key):
            self.key = key

        def __enter__(self):
            self.t = time.perf_counter()

        def __exit__(self, *exc):
            host[self.key] += time.perf_counter() - self.t

    def prepare():
        # Create systems for the arrived head of the queue while they fit.
        nonlocal used
        while queue and (not realtime or queue[0].arrival <= now()):
            req = queue[0]
            w = make(req)
            fp = dpd.footprint_bytes(w.L, w.n, w.nbonds, w.precision, cell_capacity)
            if fp > budget_bytes:
                raise ValueError(f"request {req.rid} needs {fp} bytes, over the whole budget")
            if used + fp > budget_bytes or len(slot_of) + len(prepared) >= max_replicas:
                break
            queue.popleft()
            rec = Record(req.rid, 0.0 if not realtime else req.arrival, w.n, req.steps)
            records.append(rec)
            sysm = dpd.System.from_workload(w, cell_capacity=cell_capacity)
            sysm.step(0)            # initial force, on the system's own stream
            used += fp
            prepared.append((rec, sysm, fp))

    retired = []                # (system, footprint) retired, freed while the next window runs

    def free_retired():
        nonlocal used
        for sysm, fp in retired:
            sysm.close()
            used -= fp
        retired.clear()

    try:
        while queue or prepared or slot_of or retired:
            if not slot_of:
                # Nothing on the GPU: create now.  Otherwise systems are
                # created only while a window runs, never in the gap between
                # windows.
                with _clock("prepare"):
                    prepare()
            with _clock("admit"):
                while prepared:
                    rec, sysm, fp = prepared.popleft()
                    slot = batch.admit(sysm, rec.steps)
                    rec.admitted = now()
                    slot_of[slot] = (rec, sysm, fp)
            if not slot_of:
                with _clock("retire"):
                    free_retired()
                if queue and not prepared:
                    time.sleep(max(0.0, min(queue[0].arrival - now(), 0.01)))
                continue
            with _clock("advance"):
                if autotune_at and tuned["variant"] is None and len(slot_of) >= autotune_at:
                    tuned["variant"], tuned["ms_per_step"] = batch.autotune(autotune_window)
                batch.advance(window)
            with _clock("prepare"):
                prepare()           # overlaps the window on the GPU
            with _clock("retire"):
                free_retired()      # also overlaps it
            with _clock("poll"):
                done = batch.poll()
            t = now()
            with _clock("retire"):
                for slot in done:
                    rec, sysm, fp = slot_of.pop(slot)
                    batch.retire(slot)
                    rec.done = t
                    sysm.sync()     # surfaces a device error of this replica
                    retired.append((sysm, fp))
        info = batch.info()
    finally:
        for _, sysm, _ in list(prepared) + list(slot_of.values()):
            sysm.close()
        for sysm, _ in retired:
            sysm.close()
        batch.close()
    t_end = max(r.done for r in records)
    return records, _summary(records, t_end, {"window": window, "budget_bytes": budget_bytes,
                                              "graph_captures": info["captures"],
                                              "windows": info["windows"],
                                              "variant": info["variant"],
                                              "autotuned": tuned, "host_s": host})


def serve_one_at_a_time(requests, make=workloads.replica, cell_capacity: int = 0,
                        realtime: bool = True):
    """The baseline: each replica alone through dpd_step, in arrival order."""
    records = []
    t0 = time.perf_counter()
    for req in requests:
        if realtime:
            wait = req.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
        w = make(req)
        rec = Record(req.rid, req.arrival if realtime else 0.0, w.n, req.steps)
        with dpd.System.from_workload(w, cell_capacity=cell_capacity) as sysm:
            rec.admitted = time.perf_counter() - t0
            sysm.step(req.steps)
            sysm.sync()
            rec.done = time.perf_counter() - t0
        records.append(rec)
    t_end = max(r.done for r in records)
    return records, _summary(records, t_end, {})

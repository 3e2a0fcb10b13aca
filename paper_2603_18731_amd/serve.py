"""Continuous-batching ground-state service on one GPU.

Requests (an operator bound to a subspace, plus a tolerance) arrive over time.  The server
admits a waiting request as soon as a slot and its HBM footprint (Krylov basis and work
vectors, allocated from the PyTorch caching allocator) are available, and advances every
admitted request one Lanczos iteration per step with one batched SpMV launch (``qsd_batch_*``).
Requests are split by subspace size into lanes, one batch engine and one stream each, so that
small solves iterate at their own pace while large ones occupy the GPU: work of all lanes
overlaps on the device.  Hash tables, operator tables and Lanczos state stay resident until a
request finishes.

The host loop never blocks on a running lane: each lane's steps end with an event, and a lane
is polled (convergence test, retire, admit) only once its event has completed.
"""
import math
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import LanczosBatch, SubspaceHamiltonian


@dataclass
class Request:
    rid: int
    ham: SubspaceHamiltonian
    arrival: float = 0.0  # seconds after the start of the run
    tol: float = 1e-10
    v0: str = "uniform"
    seed: int = 0
    # filled in by the server
    admitted: float = math.nan
    finished: float = math.nan
    energy: float = math.nan
    iterations: int = 0
    status: int = 0  # 2 converged, 3 iteration limit
    footprint: int = 0
    lane: int = -1

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class _Lane:
    batch: LanczosBatch
    stream: object
    active: dict = field(default_factory=dict)  # slot -> Request
    event: Optional[object] = None


class Server:
    """Admission by HBM footprint, continuous batching at Lanczos-iteration granularity.

    ``lane_bounds`` are the subspace-size boundaries between lanes; ``steps_per_poll`` Lanczos
    iterations are enqueued per lane between two convergence checks."""

    def __init__(self, hbm_budget: int, max_iter: int = 300, spmv_dtype: str = "f64",
                 lane_bounds=(1 << 15, 1 << 18), lane_slots=(128, 16, 2), steps_per_poll: int = 4):
        import torch

        self.budget = int(hbm_budget)
        self.max_iter = max_iter
        self.steps_per_poll = steps_per_poll
        self.bounds = tuple(lane_bounds)
        self.lanes = [_Lane(LanczosBatch(n, max_iter, spmv_dtype), torch.cuda.Stream()) for n in lane_slots]
        assert len(self.lanes) == len(self.bounds) + 1
        self.used = 0
        self.peak_used = 0
        self.peak_active = 0

    def lane_of(self, req: Request) -> int:
        for i, b in enumerate(self.bounds):
            if req.ham.N < b:
                return i
        return len(self.bounds)

    def footprint(self, req: Request) -> int:
        return self.lanes[self.lane_of(req)].batch.footprint(req.ham)

    def _admit(self, lane: _Lane, li: int, req: Request, now: float) -> bool:
        import torch

        fp = lane.batch.footprint(req.ham)
        if self.used + fp > self.budget or len(lane.active) >= lane.batch.max_requests:
            return False
        with torch.cuda.stream(lane.stream):
            ws = torch.empty(fp, dtype=torch.uint8, device="cuda")
        slot = lane.batch.add(req.ham, v0=req.v0, seed=req.seed, tol=req.tol, workspace=ws, stream=lane.stream)
        req.admitted, req.footprint, req.lane = now, fp, li
        lane.active[slot] = req
        self.used += fp
        self.peak_used = max(self.peak_used, self.used)
        return True

    def run(self, requests: List[Request], clock=time.perf_counter, progress=None) -> List[Request]:
        """Serves ``requests`` (arrival times relative to the start) to completion in real time;
        ``progress(k)`` is called after the k-th completion."""
        import torch

        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in pending:
            fp = self.footprint(r)
            if fp > self.budget:
                raise ValueError("request %d needs %d bytes, more than the budget" % (r.rid, fp))
        waiting: List[Request] = []
        done: List[Request] = []
        nxt = 0
        t0 = clock()
        while len(done) < len(requests):
            now = clock() - t0
            while nxt < len(pending) and pending[nxt].arrival <= now:
                waiting.append(pending[nxt])
                nxt += 1
            progressed = False
            for li, lane in enumerate(self.lanes):
                if lane.event is not None:
                    if not lane.event.query():
                        continue
                    lane.event = None
                    st, en, it, _ = lane.batch.poll(stream=lane.stream)
                    now = clock() - t0
                    for slot in list(lane.active):
                        if st[slot] in (LanczosBatch.CONVERGED, LanczosBatch.LIMIT):
                            r = lane.active.pop(slot)
                            r.finished, r.energy, r.iterations, r.status = now, float(en[slot]), int(it[slot]), int(st[slot])
                            lane.batch.remove(slot)
                            self.used -= r.footprint
                            done.append(r)
                            progressed = True
                            if progress is not None:
                                progress(len(done))
                # admissions into this lane happen while it is idle, in arrival order
                for r in list(waiting):
                    if self.lane_of(r) == li and self._admit(lane, li, r, now):
                        waiting.remove(r)
                        progressed = True
                self.peak_active = max(self.peak_active, sum(len(l.active) for l in self.lanes))
                if lane.active:
                    lane.batch.step(self.steps_per_poll, stream=lane.stream)
                    lane.event = torch.cuda.Event()
                    lane.event.record(lane.stream)
            if not progressed:
                busy = any(l.event is not None for l in self.lanes)
                if not busy and nxt < len(pending):
                    time.sleep(max(0.0, min(pending[nxt].arrival - (clock() - t0), 0.01)))
                elif busy:
                    time.sleep(2e-5)
        return done


def fifo_latencies(arrivals: np.ndarray, service: np.ndarray) -> np.ndarray:
    """Latencies of a single FIFO server with the given per-request service times, in arrival
    order: start_i = max(a_i, finish_{i-1})."""
    order = np.argsort(arrivals, kind="stable")
    lat = np.empty_like(arrivals, dtype=np.float64)
    t = 0.0
    for i in order:
        t = max(t, arrivals[i]) + service[i]
        lat[i] = t - arrivals[i]
    return lat


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def percentiles(lat) -> dict:
    lat = np.asarray(lat, dtype=np.float64)
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}

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

Optionally (``csr_min_rows``) a request of at least that many rows whose stored-matrix size is
known (``Request.nnz``) is served from its CSR matrix (lower triangle, mirrored), freed when it
finishes: the matrix and the build's transient scratch count against the HBM budget, and its
SpMV then streams the matrix instead of re-evaluating it.  The build runs on a worker thread and
a stream of its own (it synchronizes once, to size the matrix), so the host loop keeps polling
and stepping every lane meanwhile; the request joins its lane's batch once its matrix is built.
"""
import math
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import INDEX_I32, CsrMatrix, LanczosBatch, SubspaceHamiltonian


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
    nnz: int = 0  # stored entries of H on the subspace, when known (enables CSR serving)
    csr: Optional[object] = None
    used_csr: bool = False
    build_s: float = 0.0  # seconds of its CSR build (worker thread)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class _Lane:
    batch: LanczosBatch
    stream: object
    active: dict = field(default_factory=dict)  # slot -> Request
    event: Optional[object] = None
    building: list = field(default_factory=list)  # [(Request, future, reserved bytes)]


class Server:
    """Admission by HBM footprint, continuous batching at Lanczos-iteration granularity.

    ``lane_bounds`` are the subspace-size boundaries between lanes; ``steps_per_poll`` Lanczos
    iterations are enqueued per lane between two convergence checks."""

    # bytes per stored entry while the lower-triangle build runs (int64 column + value pair
    # scratch, plus the int32 column and value of the result)
    BUILD_BYTES_PER_NNZ = 8 + 16 + 4 + 8

    def __init__(self, hbm_budget: int, max_iter: int = 300, spmv_dtype: str = "f64",
                 lane_bounds=(1 << 15, 1 << 18), lane_slots=(128, 16, 2), steps_per_poll: int = 4,
                 csr_min_rows: Optional[int] = None):
        import torch

        self.budget = int(hbm_budget)
        self.spmv_dtype = spmv_dtype
        self.csr_min_rows = csr_min_rows
        self.max_iter = max_iter
        self.steps_per_poll = steps_per_poll
        self.bounds = tuple(lane_bounds)
        self.lanes = [_Lane(LanczosBatch(n, max_iter, spmv_dtype), torch.cuda.Stream()) for n in lane_slots]
        assert len(self.lanes) == len(self.bounds) + 1
        self.used = 0
        self.peak_used = 0
        self.peak_active = 0
        self._builder = ThreadPoolExecutor(max_workers=1) if csr_min_rows is not None else None
        self._build_stream = torch.cuda.Stream() if csr_min_rows is not None else None
        self.steps_during_builds = 0  # lane steps enqueued while some CSR build was running

    def lane_of(self, req: Request) -> int:
        for i, b in enumerate(self.bounds):
            if req.ham.N < b:
                return i
        return len(self.bounds)

    def footprint(self, req: Request) -> int:
        return self.lanes[self.lane_of(req)].batch.footprint(req.ham)

    def _wants_csr(self, req: Request) -> bool:
        return (self.csr_min_rows is not None and req.nnz > 0 and req.ham.N >= self.csr_min_rows
                and not req.ham.is_complex)

    def _build_csr(self, req: Request):
        import torch

        dt = torch.float32 if self.spmv_dtype == "f32" else torch.float64
        t0 = time.perf_counter()
        csr = CsrMatrix(req.ham, INDEX_I32, dtype=dt, lower_mirror=True, stream=self._build_stream)
        self._build_stream.synchronize()
        req.build_s = time.perf_counter() - t0
        return csr

    def _join(self, lane: _Lane, li: int, req: Request, op, fp: int, now: float):
        import torch

        with torch.cuda.stream(lane.stream):
            ws = torch.empty(lane.batch.footprint(req.ham), dtype=torch.uint8, device="cuda")
        slot = lane.batch.add(op, v0=req.v0, seed=req.seed, tol=req.tol, workspace=ws, stream=lane.stream)
        req.admitted, req.footprint, req.lane = now, fp, li
        lane.active[slot] = req

    def _admit(self, lane: _Lane, li: int, req: Request, now: float) -> bool:
        """Admits ``req`` into ``lane`` if a slot and its bytes are free; a CSR request starts its
        build instead and joins the batch when the build is done (``_finish_builds``)."""
        fp = lane.batch.footprint(req.ham)
        if len(lane.active) + len(lane.building) >= lane.batch.max_requests:
            return False
        use_csr = self._wants_csr(req)
        need = fp + (self.BUILD_BYTES_PER_NNZ * req.nnz + 8 * (req.ham.N + 1) if use_csr else 0)
        if self.used + need > self.budget:
            return False
        self.used += need
        self.peak_used = max(self.peak_used, self.used)
        if use_csr:
            lane.building.append((req, self._builder.submit(self._build_csr, req), need))
        else:
            self._join(lane, li, req, req.ham, fp, now)
        return True

    def _finish_builds(self, lane: _Lane, li: int, now: float) -> bool:
        """Joins the requests of ``lane`` whose CSR build has finished (the lane is idle)."""
        joined = False
        for item in list(lane.building):
            req, fut, reserved = item
            if not fut.done():
                continue
            lane.building.remove(item)
            req.csr = fut.result()  # a failed build raises here
            req.used_csr = True
            fp = lane.batch.footprint(req.ham) + req.csr.bytes
            self.used += fp - reserved
            self._join(lane, li, req, req.csr, fp, now)
            joined = True
        return joined

    def run(self, requests: List[Request], clock=time.perf_counter, progress=None) -> List[Request]:
        """Serves ``requests`` (arrival times relative to the start) to completion in real time;
        ``progress(k)`` is called after the k-th completion."""
        import torch

        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in pending:
            fp = self.footprint(r)
            if self._wants_csr(r):
                fp += self.BUILD_BYTES_PER_NNZ * r.nnz + 8 * (r.ham.N + 1)
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
                            r.csr = None  # the stored matrix is released with the request
                            self.used -= r.footprint
                            done.append(r)
                            progressed = True
                            if progress is not None:
                                progress(len(done))
                # admissions into this lane happen while it is idle, in arrival order
                if lane.building and self._finish_builds(lane, li, now):
                    progressed = True
                for r in list(waiting):
                    if self.lane_of(r) == li and self._admit(lane, li, r, now):
                        waiting.remove(r)
                        progressed = True
                self.peak_active = max(self.peak_active, sum(len(l.active) for l in self.lanes))
                if lane.active:
                    lane.batch.step(self.steps_per_poll, stream=lane.stream)
                    lane.event = torch.cuda.Event()
                    lane.event.record(lane.stream)
                    if any(not f.done() for l in self.lanes for _, f, _ in l.building):
                        self.steps_during_builds += 1
            if not progressed:
                busy = any(l.event is not None or l.building for l in self.lanes)
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


def fifo_run(arrivals: np.ndarray, solve, clock=time.perf_counter) -> np.ndarray:
    """Serves the requests for real, one at a time in arrival order: request i waits for its
    arrival time and for the previous request to finish, then ``solve(i)`` runs it to completion
    (it must synchronize).  Returns the latencies in request order."""
    order = np.argsort(arrivals, kind="stable")
    lat = np.empty(len(arrivals), dtype=np.float64)
    t0 = clock()
    for i in order:
        wait = arrivals[i] - (clock() - t0)
        if wait > 0:
            time.sleep(wait)
        solve(int(i))
        lat[i] = clock() - t0 - arrivals[i]
    return lat


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def percentiles(lat) -> dict:
    lat = np.asarray(lat, dtype=np.float64)
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}

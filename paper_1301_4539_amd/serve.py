"""Continuous-batching serving loop for FDTD solves.

Requests (grid size, material layout, step count, storage format) arrive
over time.  The engine admits them in arrival order while a slot is free and
their device footprint fits the HBM budget, keeps their fields resident, and
advances every admitted solve by a chunk of steps per tick through
fdtd_step_batch, so small grids share persistent launches; solves waiting
long get up to a few chunks per tick.  Solves admitted
between ticks join the next tick; finished solves release their slot and
memory.  Latency runs from arrival to the probe records being on the host.

The scheduler is independent of the device: `GpuBackend` drives the HIP
library; tests drive the same scheduler with a virtual-clock fake.
(Co-scheduled solves share one memory system, as jobs sharing a node do in
Sec. 2.4; batching them keeps the GPU full instead of time-slicing it.)
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Record:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    cell_updates: int = 0
    storage: int = 0
    probes: Optional[np.ndarray] = None
    requeues: int = 0

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass
class Report:
    records: List[Record]
    makespan: float
    busy: float                  # device time of the ticks (pipelined), else time inside step + sync
    rejected: List[int]

    def latencies(self) -> np.ndarray:
        return np.array([r.latency for r in self.records if np.isfinite(r.finished)])

    def summary(self) -> dict:
        lat = self.latencies()
        work = sum(r.cell_updates for r in self.records if np.isfinite(r.finished))
        return {"requests": len(lat), "rejected": len(self.rejected),
                "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
                "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
                "mean_s": float(lat.mean()) if len(lat) else None,
                "throughput_G_per_s": work / self.makespan / 1e9 if self.makespan > 0 else None,
                "makespan_s": self.makespan, "busy_frac": self.busy / self.makespan if self.makespan else None,
                "busy_while_pending": (self.busy / self.pending_time
                                       if getattr(self, "pending_time", 0.0) > 0 else None),
                "requeues": sum(r.requeues for r in self.records)}


class AdmissionError(RuntimeError):
    """Raised by a backend when a solve cannot be allocated right now."""


class Engine:
    """Continuous batching.  Every tick advances each admitted solve by
    `chunk` steps, or by a multiple of it for solves that have waited long:
    k = ceil(age / age_step) chunks, at most `max_boost` (age from arrival).
    A 16-bit solve re-encodes its fields at the end of every block, and its
    blocks end at absolute multiples of its T, so a chunk that is a multiple
    of every T the backend runs (`backend.block_lengths()`) keeps each
    solve's blocks, and so its result, where a solo run puts them; the
    default 48 is a multiple of 1, 2, 3 and 4.  The boost bounds the tail
    latency of long solves."""

    def __init__(self, backend, budget_bytes: int = 24 << 30, max_slots: int = 64, chunk: int = 48,
                 age_step: float = 0.5, max_boost: int = 3):
        assert chunk > 0 and max_boost >= 1 and age_step > 0
        lens = backend.block_lengths() if hasattr(backend, "block_lengths") else ()
        bad = [t for t in lens if chunk % t]
        if bad:
            raise ValueError(f"chunk {chunk} is not a multiple of the block lengths {sorted(set(bad))}: "
                             f"16-bit solves would round differently in the mix than alone")
        self.b = backend
        self.budget = budget_bytes
        self.max_slots = max_slots
        self.chunk = chunk
        self.age_step = age_step
        self.max_boost = max_boost

    def steps_for(self, a, now) -> int:
        age = now - a["req"].arrival
        k = min(self.max_boost, max(1, math.ceil(age / self.age_step)))
        return min(a["left"], k * self.chunk)

    def run(self, requests) -> Report:
        """Serve `requests`.  With a backend that can enqueue a tick without
        waiting for it (`submit`/`wait`), ticks are pipelined: tick n+1 is
        enqueued before the engine waits for tick n, so admissions, probe
        read-backs and the next tick's bookkeeping overlap the device's work
        and the device does not idle between ticks."""
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting: collections.deque = collections.deque()
        active: List[dict] = []
        recs: Dict[int, Record] = {r.rid: Record(r.rid, r.arrival, storage=r.storage) for r in requests}
        rejected = []
        used = 0
        busy = 0.0
        pending_time = 0.0                 # time with a solve admitted or waiting
        piped = hasattr(self.b, "submit") and getattr(self.b, "pipelined", True)
        inflight = None                    # (token, [(solve, steps)]) of the tick on the device
        t0 = self.b.now()
        last = 0.0
        while pending or waiting or active:
            now = self.b.now() - t0
            if active or waiting:
                pending_time += now - last
            last = now
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admission: arrival order, while a slot and the memory budget allow
            while waiting and len(active) < self.max_slots:
                req = waiting[0]
                fp = self.b.footprint(req)
                if fp > self.budget:
                    rejected.append(req.rid)
                    waiting.popleft()
                    continue
                if used + fp > self.budget:
                    break
                try:
                    h = self.b.create(req)
                except AdmissionError:
                    recs[req.rid].requeues += 1
                    break                       # retry at the next tick
                waiting.popleft()
                used += fp
                recs[req.rid].admitted = self.b.now() - t0
                active.append({"req": req, "h": h, "left": req.n_steps, "queued": req.n_steps, "fp": fp})
            runnable = [a for a in active if a["queued"] > 0]
            if not runnable and inflight is None:
                if not active:
                    if hasattr(self.b, "idle"):
                        self.b.idle()               # nothing on the device: deferred clean-up
                    if pending:
                        self.b.wait_until(t0 + pending[0].arrival)
                    elif waiting:
                        # nothing fits even on an idle device: the budget forbids it
                        rejected.append(waiting.popleft().rid)
                continue
            tick = None
            if runnable:
                now = self.b.now() - t0
                counts = [min(a["queued"], self.steps_for(a, now)) for a in runnable]
                if piped:
                    token = self.b.submit([a["h"] for a in runnable], counts)
                else:
                    ts = self.b.now()
                    self.b.step([a["h"] for a in runnable], counts)
                    self.b.sync()
                    busy += self.b.now() - ts
                    token = None
                for a, c in zip(runnable, counts):
                    a["queued"] -= c
                tick = (token, list(zip(runnable, counts)))
            # retire the tick before this one (pipelined), or this one (not)
            done, inflight = (inflight, tick) if piped else (tick, None)
            if done is None:
                continue
            if piped:
                busy += self.b.wait(done[0])
            finished = []
            for a, c in done[1]:
                a["left"] -= c
                if a["left"] == 0:
                    r = recs[a["req"].rid]
                    r.probes = self.b.finish(a["h"], a["req"])
                    r.finished = self.b.now() - t0
                    r.cell_updates = a["req"].nx * a["req"].ny * a["req"].nz * a["req"].n_steps
                    used -= a["fp"]
                    finished.append(a)
            if finished:
                active = [a for a in active if all(a is not f for f in finished)]
        if hasattr(self.b, "idle"):
            self.b.idle()
        done_recs = [r for r in recs.values() if np.isfinite(r.finished)]
        makespan = max((r.finished for r in done_recs), default=0.0) - min((r.arrival for r in done_recs), default=0.0)
        rep = Report(sorted(recs.values(), key=lambda r: r.rid), makespan, busy, rejected)
        rep.pending_time = pending_time
        return rep


# Steps per HBM pass used for each storage format (the fastest on MI355X:
# FP32 storage is compute-bound at 4, 16-bit storage at 3).  A solve is
# bit-identical alone and in the mix when every chunk is a multiple of its T.
DEFAULT_T = {0: 4, 1: 3, 2: 3}


class GpuBackend:
    """Drives the HIP library.  `workloads` maps request id to a pre-built
    Workload (the request payload: grid, materials, sources, probes);
    `time_block` is one T for every solve or a map storage -> T.

    Ticks are enqueued on one stream (`submit`) and waited for by their end
    event (`wait`), so the engine can queue the next tick first.  New solvers
    are created on a side stream (their uploads do not wait for the running
    tick) and then moved to the tick stream; finished solvers' probes are read
    without waiting for later ticks, and the solvers are released when the
    device has nothing queued (`idle`).  `pipelined=False` steps and waits
    tick by tick (no submit)."""

    def __init__(self, workloads, time_block=None, pipelined=True):
        import torch
        from . import fdtd
        self.fdtd = fdtd
        self.torch = torch
        self.wl = workloads
        tb = DEFAULT_T if time_block is None else time_block
        self.T = dict(tb) if isinstance(tb, dict) else {k: int(tb) for k in DEFAULT_T}
        self.alone = set()      # solves fdtd_step_batch does not take: stepped one by one
        self.main = torch.cuda.current_stream()
        self.side = torch.cuda.Stream()          # default priority, like every stream here
        self.to_close = []
        self.pipelined = pipelined

    def block_lengths(self):
        """Every block length T a solve may run: the per-storage T of the
        batched solves and 1..4, the automatic T of graded-spacing solves."""
        return sorted(set(self.T.values()) | {1, 2, 3, 4})

    def solver_options(self, wl):
        """(kernel, T, batched) for a request: uniform grids run the fused
        kernel at the storage's T in shared launches; graded sizes take their
        automatic T and CPML layers the plain kernels, each stepped alone."""
        f = self.fdtd
        if wl.cpml:
            return f.KERNEL_AUTO, 0, False
        if wl.spacing is not None:
            return f.KERNEL_FUSED, 0, False
        return f.KERNEL_FUSED, self.T[wl.storage], True

    def now(self) -> float:
        return time.perf_counter()

    def wait_until(self, t: float):
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(d)

    def footprint(self, req) -> int:
        b = self.fdtd.workspace_bytes(req.nx, req.ny, req.nz, req.storage) + 8 * 8 * (req.n_steps + 256)
        layer = getattr(self.wl[req.rid], "cpml", None)
        if layer:      # two copies of the psi state: 4-float groups over three pairs of slabs
            n = int(layer["thickness"])
            b += 2 * 16 * 2 * n * ((req.ny + 1) * (req.nz + 1) + (req.nx + 1) * (req.nz + 1) + (req.nx + 1) * (req.ny + 1))
        return b

    def create(self, req):
        kernel, tb, batched = self.solver_options(self.wl[req.rid])
        try:
            with self.torch.cuda.stream(self.side):
                h = self.fdtd.Solver.from_workload(self.wl[req.rid], kernel=kernel, time_block=tb,
                                                   stream=self.side)
                # its probe rows for the whole solve, so that no tick waits on
                # a row allocation
                h.reserve_steps(req.n_steps)
            h.set_stream(self.main)              # its uploads are done; it now steps with the others
            if h._ws is not None:
                h._ws.record_stream(self.main)
            if not batched:
                self.alone.add(h)
            return h
        except (self.fdtd.FdtdError, self.torch.cuda.OutOfMemoryError) as e:
            if isinstance(e, self.fdtd.FdtdError) and e.code != self.fdtd.ENOMEM:
                raise
            raise AdmissionError(str(e)) from e

    def step(self, handles, counts):
        batch = [(h, n) for h, n in zip(handles, counts) if h not in self.alone]
        if batch:
            self.fdtd.step_batch([h for h, _ in batch], [n for _, n in batch])
        for h, n in zip(handles, counts):
            if h in self.alone:
                h.step(n)

    def sync(self):
        self.torch.cuda.synchronize()

    def submit(self, handles, counts):
        """Enqueue one tick; returns its (start, end) events."""
        ev0 = self.torch.cuda.Event(enable_timing=True)
        ev1 = self.torch.cuda.Event(enable_timing=True)
        ev0.record(self.main)
        self.step(handles, counts)
        ev1.record(self.main)
        return ev0, ev1

    def wait(self, token) -> float:
        """Wait for a submitted tick; returns its device time in seconds."""
        ev0, ev1 = token
        ev1.synchronize()
        return ev0.elapsed_time(ev1) / 1e3

    def finish(self, h, req) -> np.ndarray:
        p = h.read_probes(0, req.n_steps)      # waits for this solve's own steps only
        self.alone.discard(h)
        self.to_close.append(h)
        return p

    def idle(self):
        """Release the finished solvers (nothing is queued on the device)."""
        for h in self.to_close:
            h.close()
        self.to_close = []

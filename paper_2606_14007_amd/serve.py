"""Plot serving with continuous batching on one GPU.

Requests (k, key) arrive over time.  The server admits them in arrival
order as soon as an execution slot is free and the job's device footprint
(Table 1 + Table 2 capacity + offsets + workspace) fits the HBM budget next
to everything resident.  Each admitted job runs on its own stream, so jobs
overlap on the device; finished jobs keep their tables on the device until
their result is consumed, and then their buffers return to a per-k pool
for reuse.  If the oldest waiting job does not fit, later jobs that do fit
may go first ("backfill"), which keeps the GPU busy without letting a large
job starve: a job that has been passed over `max_bypass` times blocks
backfill until it runs.

The scheduler is written against a small executor interface (footprint /
submit / poll / release) so that the same loop drives the GPU executor
below or a simulated one in CPU tests.
"""
from __future__ import annotations

import heapq
import math
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence


@dataclass
class Job:
    jid: int
    k: int
    key: bytes
    arrival: float                  # seconds since the start of the run
    threshold: Optional[int] = None
    admitted: Optional[float] = None
    finished: Optional[float] = None
    bypassed: int = 0
    handle: object = None
    result: object = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Executor:
    """What the scheduler needs from a device."""

    def footprint(self, k: int) -> int:
        raise NotImplementedError

    def submit(self, job: Job, slot: int):
        raise NotImplementedError

    def poll(self, handle) -> bool:
        raise NotImplementedError

    def release(self, job: Job) -> None:
        raise NotImplementedError


@dataclass
class Stats:
    jobs: List[Job]
    makespan: float
    max_resident: int
    max_concurrent: int

    def latencies(self) -> List[float]:
        return sorted(j.latency for j in self.jobs)

    def percentile(self, p: float) -> float:
        lat = self.latencies()
        if not lat:
            return float("nan")
        i = min(len(lat) - 1, max(0, math.ceil(p / 100.0 * len(lat)) - 1))
        return lat[i]

    def plots_per_hour(self) -> float:
        return len(self.jobs) * 3600.0 / self.makespan if self.makespan > 0 else float("nan")


class Server:
    def __init__(self, executor: Executor, budget_bytes: int, slots: int = 4,
                 max_bypass: int = 8, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep,
                 on_done: Optional[Callable[[Job], None]] = None):
        if slots < 1:
            raise ValueError("need at least one slot")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.slots = slots
        self.max_bypass = max_bypass
        self.clock = clock
        self.sleep = sleep
        self.on_done = on_done

    def run(self, jobs: Sequence[Job]) -> Stats:
        """Serve `jobs` (arrival times relative to now) to completion."""
        for j in jobs:
            if self.ex.footprint(j.k) > self.budget:
                raise ValueError(f"job {j.jid} (k={j.k}) can never fit the budget")
        pending = sorted(jobs, key=lambda j: (j.arrival, j.jid))
        waiting: List[Job] = []
        running: Dict[int, Job] = {}          # slot -> job
        free_slots = list(range(self.slots))
        resident = 0
        max_resident = 0
        max_conc = 0
        done: List[Job] = []
        t0 = self.clock()
        nxt = 0
        while len(done) < len(jobs):
            now = self.clock() - t0
            while nxt < len(pending) and pending[nxt].arrival <= now:
                waiting.append(pending[nxt])
                nxt += 1
            # completions
            progressed = False
            for slot, job in list(running.items()):
                if self.ex.poll(job.handle):
                    job.finished = self.clock() - t0
                    del running[slot]
                    free_slots.append(slot)
                    if self.on_done:
                        self.on_done(job)
                    self.ex.release(job)
                    resident -= self.ex.footprint(job.k)
                    done.append(job)
                    progressed = True
            # admissions, in arrival order with bounded backfill
            i = 0
            while free_slots and i < len(waiting):
                job = waiting[i]
                need = self.ex.footprint(job.k)
                if resident + need <= self.budget:
                    slot = free_slots.pop(0)
                    job.admitted = self.clock() - t0
                    job.handle = self.ex.submit(job, slot)
                    running[slot] = job
                    resident += need
                    max_resident = max(max_resident, resident)
                    max_conc = max(max_conc, len(running))
                    waiting.pop(i)
                    progressed = True
                    continue
                # the job does not fit yet: later ones may pass it, up to a limit
                if job.bypassed >= self.max_bypass:
                    break
                for later in waiting[i + 1:]:
                    if resident + self.ex.footprint(later.k) <= self.budget:
                        job.bypassed += 1
                        break
                i += 1
            if not progressed:
                if running or nxt < len(pending):
                    wait = 2e-4
                    if not running and nxt < len(pending):
                        wait = max(0.0, min(0.01, pending[nxt].arrival - (self.clock() - t0)))
                    self.sleep(wait)
        makespan = max(j.finished for j in done) - min(j.arrival for j in done) if done else 0.0
        return Stats(sorted(done, key=lambda j: j.jid), makespan, max_resident, max_conc)


# ---------------------------------------------------------------------------
# GPU executor
# ---------------------------------------------------------------------------

class GpuExecutor(Executor):
    """Runs each job as one vx_plot on the stream of its slot.  Buffers come
    from a per-k pool; idle pooled buffers count against the budget only
    while they exist, and are dropped (largest first) when a new allocation
    would not fit."""

    def __init__(self, slots: int, budget_bytes: int, tuning_for_k=None, device=None):
        import torch
        from . import plotter as P
        self.torch = torch
        self.P = P
        self.device = P._dev(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.budget = budget_bytes
        self.pool: Dict[int, list] = {}
        self.tuning_for_k = tuning_for_k or (lambda k: None)
        self._fp: Dict[int, int] = {}

    def footprint(self, k: int) -> int:
        if k not in self._fp:
            self._fp[k] = self.P.footprint_bytes(k, tuning=self.tuning_for_k(k))
        return self._fp[k]

    def _idle_bytes(self) -> int:
        return sum(self.footprint(k) * len(v) for k, v in self.pool.items())

    def _buffers(self, k: int, in_use: int):
        if self.pool.get(k):
            return self.pool[k].pop()
        # make room among idle pooled buffers if needed
        while in_use + self._idle_bytes() + self.footprint(k) > self.budget:
            ks = [kk for kk, v in self.pool.items() if v]
            if not ks:
                break
            self.pool[max(ks)].pop()
        return self.P.alloc_plot(k, tuning=self.tuning_for_k(k), device=self.device)

    def submit(self, job: Job, slot: int):
        from . import _native as N
        torch = self.torch
        in_use = getattr(self, "_in_use", 0)
        buf = self._buffers(job.k, in_use)
        self._in_use = in_use + self.footprint(job.k)
        s = self.streams[slot]
        params = N.make_params(job.key, job.k, job.threshold)
        N.vx_plot(params, buf.native(), self.tuning_for_k(job.k), s.cuda_stream)
        ev = torch.cuda.Event()
        ev.record(s)
        job.result = buf
        return ev

    def poll(self, handle) -> bool:
        return handle.query()

    def release(self, job: Job) -> None:
        self._in_use -= self.footprint(job.k)
        self.pool.setdefault(job.k, []).append(job.result)
        job.result = None


def jobs_from_arrivals(arrivals) -> List[Job]:
    return [Job(jid=i, k=a.k, key=a.key, arrival=a.t) for i, a in enumerate(arrivals)]


def expected_service_time(k_lo: int, k_hi: int, per_k_seconds: Dict[int, float]) -> float:
    ks = range(k_lo, k_hi + 1)
    return sum(per_k_seconds[k] for k in ks) / len(ks)


def measure_plain_times(ks: Sequence[int], reps: int = 3, tuning_for_k=None) -> Dict[int, float]:
    """Seconds per plot of the plain path (one plot at a time) for each k."""
    import torch
    from . import _native as N
    from . import plotter as P
    out = {}
    tuning_for_k = tuning_for_k or (lambda k: None)
    for k in ks:
        b = P.alloc_plot(k, tuning=tuning_for_k(k))
        p = N.make_params(bytes(32), k)
        sh = torch.cuda.current_stream().cuda_stream
        N.vx_plot(p, b.native(), tuning_for_k(k), sh)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            N.vx_plot(p, b.native(), tuning_for_k(k), sh)
        torch.cuda.synchronize()
        out[k] = (time.perf_counter() - t0) / reps
        del b
    return out

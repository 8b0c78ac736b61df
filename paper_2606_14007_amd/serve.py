"""Plot serving with continuous batching on one GPU.

Requests (k, key) arrive over time.  The server admits them in arrival
order as soon as an execution slot is free and the job's device footprint
(Table 1 + Table 2 capacity + offsets + workspace) fits the HBM budget next
to everything resident.  Each admitted job runs on its own stream, so jobs
overlap on the device; finished jobs keep their tables on the device until
their result is consumed, and then their memory is returned.  On the GPU
all plot buffers are carved from one arena allocated up front, so serving
never allocates or frees device memory (a free would synchronise every
stream).  If the oldest waiting job does not fit, later jobs that do fit may
go first ("backfill"), which keeps the GPU busy without letting a large job
starve: a job that has been passed over `max_bypass` times blocks backfill
until it runs.

Size classes (optional): jobs with k >= `big_k` are "big" and at most
`max_big` of them run at once, in arrival order among themselves; smaller
jobs take the other slots.  Running every job beside every other stretches
the largest jobs the most (the device is shared, and a large plot already
fills it), which raises the tail latency above a one-at-a-time server's;
keeping the big jobs one at a time bounds their stretch to the small jobs'
share of the work, while small jobs still skip the queue of big ones.

The scheduler is written against a small executor interface (footprint /
submit / poll / release) so that the same loop drives the GPU executor
below or a simulated one in CPU tests.
"""
from __future__ import annotations

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
    error: Optional[str] = None     # set when the device reported a problem with this job

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Executor:
    """What the scheduler needs from a device."""

    def footprint(self, job: Job) -> int:
        raise NotImplementedError

    def submit(self, job: Job, slot: int):
        raise NotImplementedError

    def poll(self, job: Job) -> bool:
        """True once the job is done; may set job.error."""
        raise NotImplementedError

    def release(self, job: Job) -> None:
        raise NotImplementedError

    def can_admit(self, job: Job, resident: int, budget: int) -> bool:
        """Whether the job may start now (default: its bytes fit the budget)."""
        return resident + self.footprint(job) <= budget


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

    def by_k(self) -> Dict[int, Dict[str, float]]:
        out: Dict[int, list] = {}
        for j in self.jobs:
            out.setdefault(j.k, []).append(j.latency)
        res = {}
        for k, v in sorted(out.items()):
            v = sorted(v)
            res[k] = {"n": len(v), "p50_ms": v[len(v) // 2] * 1e3,
                      "p99_ms": v[min(len(v) - 1, max(0, math.ceil(0.99 * len(v)) - 1))] * 1e3}
        return res

    def failed(self) -> List[Job]:
        return [j for j in self.jobs if j.error]


class Server:
    def __init__(self, executor: Executor, budget_bytes: int, slots: int = 4,
                 max_bypass: int = 8, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep,
                 on_done: Optional[Callable[[Job], None]] = None,
                 big_k: Optional[int] = None, max_big: int = 1):
        if slots < 1:
            raise ValueError("need at least one slot")
        if big_k is not None and max_big < 1:
            raise ValueError("max_big must be at least 1")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.slots = slots
        self.max_bypass = max_bypass
        self.clock = clock
        self.sleep = sleep
        self.on_done = on_done
        self.big_k = big_k
        self.max_big = max_big

    def _big(self, job: Job) -> bool:
        return self.big_k is not None and job.k >= self.big_k

    def run(self, jobs: Sequence[Job]) -> Stats:
        """Serve `jobs` (arrival times relative to now) to completion."""
        for j in jobs:
            if self.ex.footprint(j) > self.budget:
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
                if self.ex.poll(job):
                    job.finished = self.clock() - t0
                    del running[slot]
                    free_slots.append(slot)
                    if self.on_done:
                        self.on_done(job)
                    self.ex.release(job)
                    resident -= self.ex.footprint(job)
                    done.append(job)
                    progressed = True
            # admissions, in arrival order with bounded backfill
            n_big = sum(1 for j in running.values() if self._big(j))
            i = 0
            while free_slots and i < len(waiting):
                job = waiting[i]
                need = self.ex.footprint(job)
                if self._big(job) and n_big >= self.max_big:
                    i += 1          # its class is full: waits for a big job to finish
                    continue
                if self.ex.can_admit(job, resident, self.budget):
                    slot = free_slots.pop(0)
                    job.admitted = self.clock() - t0
                    job.handle = self.ex.submit(job, slot)
                    running[slot] = job
                    n_big += self._big(job)
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
                    if (not (self._big(later) and n_big >= self.max_big)
                            and self.ex.can_admit(later, resident, self.budget)):
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

class Arena:
    """First-fit sub-allocator over one preallocated device byte range, with
    coalescing of free neighbours.  Host-side bookkeeping only: serving never
    calls the device allocator, so no allocation or free can stall streams."""

    ALIGN = 2 << 20

    def __init__(self, size: int):
        self.size = size // self.ALIGN * self.ALIGN
        self.free = [(0, self.size)]      # sorted (offset, length)

    def alloc(self, nbytes: int) -> Optional[int]:
        n = -(-nbytes // self.ALIGN) * self.ALIGN
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, ln - n)
                return off
        return None

    def can_alloc(self, nbytes: int) -> bool:
        n = -(-nbytes // self.ALIGN) * self.ALIGN
        return any(ln >= n for _, ln in self.free)

    def release(self, off: int, nbytes: int) -> None:
        n = -(-nbytes // self.ALIGN) * self.ALIGN
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged


class GpuExecutor(Executor):
    """Runs each job as one vx_plot on the stream of its slot.  All plot
    buffers are carved from one device arena allocated up front (the HBM
    budget), so admission is "a contiguous block of the job's footprint is
    free", and finished jobs' tables stay in place until released."""

    def __init__(self, slots: int, budget_bytes: int, tuning_for_k=None, device=None):
        import torch
        from . import plotter as P
        from . import _native as N
        self.torch = torch
        self.P = P
        self.N = N
        self.device = P._dev(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.arena = Arena(budget_bytes)
        self.mem = torch.empty(self.arena.size, dtype=torch.uint8, device=self.device)
        self.tuning_for_k = tuning_for_k or (lambda k: None)
        self._layout: Dict[tuple, tuple] = {}

    def _plan(self, k: int, threshold: Optional[int]):
        """Arena layout of one job: keyed by k and the job's threshold, which
        sets its Table-2 capacity."""
        N = self.N
        T = N.vx_default_threshold(k) if threshold is None else int(threshold)
        if (k, T) not in self._layout:
            p = N.make_params(bytes(32), k, T)
            cap = N.vx_t2_capacity_hint(k, T)
            ws = N.vx_workspace_bytes(p, N.VX_CALL_PLOT, self.tuning_for_k(k))
            if ws == 0:
                raise ValueError(f"invalid plot k={k}")
            n = 1 << k
            parts = [("workspace", ws), ("t1_keys", n * 8), ("t1_nonces", n * 4),
                     ("bucket_offsets", (N.VX_NUM_BUCKETS + 1) * 4), ("t2", cap * 16), ("t2_count", 8)]
            offs, at = {}, 0
            for name, nb in parts:
                offs[name] = (at, nb)
                at += -(-nb // 256) * 256
            self._layout[(k, T)] = (offs, at, cap)
        return self._layout[(k, T)]

    def footprint(self, job: Job) -> int:
        return self._plan(job.k, job.threshold)[1]

    def can_admit(self, job: Job, resident: int, budget: int) -> bool:
        return self.arena.can_alloc(self.footprint(job))

    def _view(self, base: int, off_nb, dtype, shape=None):
        off, nb = off_nb
        t = self.mem.narrow(0, base + off, nb).view(dtype)
        return t.view(shape) if shape else t

    def submit(self, job: Job, slot: int):
        torch, N = self.torch, self.N
        offs, total, cap = self._plan(job.k, job.threshold)
        base = self.arena.alloc(total)
        if base is None:
            raise RuntimeError("arena full: admission and allocation disagree")
        buf = self.P.PlotBuffers(
            k=job.k,
            t1_keys=self._view(base, offs["t1_keys"], torch.int64),
            t1_nonces=self._view(base, offs["t1_nonces"], torch.int32),
            bucket_offsets=self._view(base, offs["bucket_offsets"], torch.int32),
            t2=self._view(base, offs["t2"], torch.int64, (cap, 2)),
            t2_count=self._view(base, offs["t2_count"], torch.int64),
            workspace=self._view(base, offs["workspace"], torch.uint8),
        )
        s = self.streams[slot]
        params = N.make_params(job.key, job.k, job.threshold)
        N.vx_plot(params, buf.native(), self.tuning_for_k(job.k), s.cuda_stream)
        ev = torch.cuda.Event()
        ev.record(s)
        job.result = buf
        job._arena = (base, total)
        job._stream = s
        return ev

    def poll(self, job: Job) -> bool:
        """Done once the job's event has passed; then its Table-2 count and
        device status word are read (the stream is idle, so this does not
        wait) and a problem is recorded in job.error."""
        if not job.handle.query():
            return False
        try:
            self.P.check_plot(job.result, job._stream, what=f"job {job.jid} (k={job.k})")
        except self.P.PlotOverflow as e:
            job.error = str(e)
        return True

    def release(self, job: Job) -> None:
        base, total = job._arena
        self.arena.release(base, total)
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

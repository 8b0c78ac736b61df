"""The serving scheduler on the CPU, with a simulated executor and a
virtual clock: admission by footprint, budget, ordering, bounded backfill,
latency statistics.  No GPU."""
import math

import pytest

from paper_2606_14007_amd.serve import Executor, Job, Server, Stats, jobs_from_arrivals
from vx_inputs import serving_arrivals


class Clock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-5)


class FakeExecutor(Executor):
    """Job of size k takes 2^(k-20) ms of device time; running jobs share the
    device (processor sharing) up to `parallel` at full speed each."""

    def __init__(self, clock, parallel=2.0, fp_per_record=48):
        self.clock = clock
        self.parallel = parallel
        self.fp = fp_per_record
        self.running = {}
        self.resident = 0
        self.peak = 0
        self.order = []

    def footprint(self, job):
        return (1 << job.k) * self.fp

    def _advance(self):
        now = self.clock.now()
        dt = now - getattr(self, "_last", now)
        self._last = now
        if self.running:
            rate = min(1.0, self.parallel / len(self.running))
            for h in self.running:
                self.running[h] -= dt * rate

    def submit(self, job, slot):
        self._advance()
        h = object()
        self.running[h] = 2.0 ** (job.k - 20) * 1e-3
        self.resident += self.footprint(job)
        self.peak = max(self.peak, self.resident)
        self.order.append(job.jid)
        return h

    def poll(self, job):
        h = job.handle
        self._advance()
        if self.running[h] <= 0:
            del self.running[h]
            return True
        return False

    def release(self, job):
        self.resident -= self.footprint(job)


def _run(jobs, slots, budget, **kw):
    c = Clock()
    ex = FakeExecutor(c)
    srv = Server(ex, budget, slots=slots, clock=c.now, sleep=c.sleep, **kw)
    return srv.run(jobs), ex


def test_all_jobs_complete_and_respect_arrival_and_budget():
    arr = serving_arrivals(200, rate_per_s=300.0, k_lo=18, k_hi=24)
    jobs = jobs_from_arrivals(arr)
    budget = (1 << 24) * 48 * 3
    st, ex = _run(jobs, slots=4, budget=budget)
    assert len(st.jobs) == 200
    assert all(j.admitted >= j.arrival - 1e-9 and j.finished >= j.admitted for j in st.jobs)
    assert ex.peak <= budget and st.max_resident <= budget
    assert st.max_concurrent <= 4


def test_single_slot_is_fifo():
    jobs = jobs_from_arrivals(serving_arrivals(60, rate_per_s=500.0, k_lo=18, k_hi=22))
    st, ex = _run(jobs, slots=1, budget=1 << 40, max_bypass=0)
    assert ex.order == sorted(ex.order)
    assert st.max_concurrent == 1


def test_continuous_batching_beats_fifo_latency():
    arr = serving_arrivals(300, rate_per_s=400.0, k_lo=18, k_hi=23)
    fifo, _ = _run(jobs_from_arrivals(arr), slots=1, budget=1 << 40, max_bypass=0)
    cb, _ = _run(jobs_from_arrivals(arr), slots=4, budget=1 << 40)
    assert cb.percentile(50) < fifo.percentile(50)
    assert cb.percentile(99) < fifo.percentile(99)
    assert cb.plots_per_hour() >= fifo.plots_per_hour()


def test_backfill_is_bounded_so_big_jobs_do_not_starve():
    big = Job(0, 24, b"\x00" * 32, 0.0)
    small = [Job(i, 18, b"\x01" * 32, 0.0001 * i) for i in range(1, 200)]
    filler = Job(999, 23, b"\x02" * 32, 0.0)
    budget = ((1 << 24) + (1 << 23)) * 48 - 1  # big + filler do not fit together
    st, ex = _run([filler, big] + small, slots=3, budget=budget, max_bypass=5)
    pos = ex.order.index(0)
    assert big.bypassed <= 5
    assert pos <= 2 + 5 + 3  # admitted soon after the filler leaves


def test_job_larger_than_budget_is_rejected():
    with pytest.raises(ValueError):
        _run([Job(0, 25, b"\x00" * 32, 0.0)], slots=1, budget=1000)


def test_percentiles():
    jobs = []
    for i in range(100):
        j = Job(i, 10, b"", 0.0)
        j.finished = (i + 1) / 100.0
        jobs.append(j)
    st = Stats(jobs, makespan=1.0, max_resident=0, max_concurrent=1)
    assert math.isclose(st.percentile(50), 0.50)
    assert math.isclose(st.percentile(99), 0.99)
    assert math.isclose(st.plots_per_hour(), 360000.0)


def test_arena_first_fit_and_coalescing():
    from paper_2606_14007_amd.serve import Arena
    A = Arena.ALIGN
    a = Arena(10 * A)
    x = a.alloc(3 * A)
    y = a.alloc(1)            # rounds up to one unit
    z = a.alloc(4 * A)
    assert (x, y, z) == (0, 3 * A, 4 * A)
    assert not a.can_alloc(3 * A) and a.can_alloc(2 * A)
    a.release(y, 1)
    a.release(x, 3 * A)       # coalesces with y's unit into 4 units at 0
    assert a.free[0] == (0, 4 * A)
    assert a.alloc(4 * A) == 0
    a.release(0, 4 * A)
    a.release(z, 4 * A)
    assert a.free == [(0, 10 * A)]


def test_gpu_executor_sizes_table2_from_each_jobs_threshold():
    """The arena layout of a job depends on its threshold: a wider threshold
    gets the larger Table-2 capacity it needs (host-side planning only)."""
    from paper_2606_14007_amd import _native as N
    from paper_2606_14007_amd.serve import GpuExecutor
    ex = GpuExecutor.__new__(GpuExecutor)   # planning needs no device
    ex.N = N
    ex.tuning_for_k = lambda k: None
    ex._layout = {}
    k = 28                                  # default threshold 2^36
    plain = Job(0, k, bytes(32), 0.0)
    wide = Job(1, k, bytes(32), 0.0, threshold=1 << 38)
    assert ex.footprint(wide) > ex.footprint(plain)
    offs, total, cap = ex._plan(k, 1 << 38)
    assert cap == N.vx_t2_capacity_hint(k, 1 << 38)
    assert offs["t2"][1] == cap * 16 and total == ex.footprint(wide)
    assert ex._plan(k, None)[2] == N.vx_t2_capacity_hint(k, N.vx_default_threshold(k))


def test_failed_jobs_are_reported():
    class Failing(FakeExecutor):
        def poll(self, job):
            done = super().poll(job)
            if done and job.jid % 7 == 3:
                job.error = "device status 0x4"
            return done

    c = Clock()
    ex = Failing(c)
    jobs = jobs_from_arrivals(serving_arrivals(30, rate_per_s=500.0, k_lo=16, k_hi=20))
    st = Server(ex, 1 << 40, slots=2, clock=c.now, sleep=c.sleep).run(jobs)
    assert [j.jid for j in st.failed()] == [j for j in range(30) if j % 7 == 3]


class ClassCounting(FakeExecutor):
    """Records how many jobs with k >= big_k ran at once and their order."""

    def __init__(self, clock, big_k, **kw):
        super().__init__(clock, **kw)
        self.big_k = big_k
        self.big_now = 0
        self.big_peak = 0
        self.big_order = []

    def submit(self, job, slot):
        h = super().submit(job, slot)
        if job.k >= self.big_k:
            self.big_now += 1
            self.big_peak = max(self.big_peak, self.big_now)
            self.big_order.append(job.jid)
        return h

    def release(self, job):
        super().release(job)
        if job.k >= self.big_k:
            self.big_now -= 1


@pytest.mark.parametrize("max_big", [1, 2])
def test_size_classes_cap_big_jobs_and_keep_their_order(max_big):
    c = Clock()
    ex = ClassCounting(c, big_k=20, parallel=1.0)
    jobs = jobs_from_arrivals(serving_arrivals(300, rate_per_s=300.0, k_lo=14, k_hi=22))
    st = Server(ex, 1 << 40, slots=4, clock=c.now, sleep=c.sleep, big_k=20, max_big=max_big).run(jobs)
    assert len(st.jobs) == 300
    assert ex.big_peak == max_big
    assert ex.big_order == sorted(ex.big_order)
    assert st.max_concurrent <= 4


def test_size_classes_beat_fifo_at_both_percentiles():
    """The serving mix in miniature (sizes 2^-6 .. 2^2 ms, a 64x spread as
    k = 22..30 has 256x) at about 80% load on a device shared evenly by
    running jobs: with one big job at a time, small jobs skip the queue of
    big ones (a far lower median) and the tail stays below FIFO's."""
    mean = sum(2.0 ** (k - 20) for k in range(14, 23)) / 9 * 1e-3
    arr = serving_arrivals(1000, rate_per_s=0.8 / mean, k_lo=14, k_hi=22)

    def run(slots, **kw):
        c = Clock()
        return Server(FakeExecutor(c, parallel=1.0), 1 << 40, slots=slots, clock=c.now,
                      sleep=c.sleep, **kw).run(jobs_from_arrivals(arr))

    fifo = run(1, max_bypass=0)
    classes = run(4, big_k=20, max_big=1)
    assert classes.percentile(50) < 0.5 * fifo.percentile(50)
    assert classes.percentile(99) < fifo.percentile(99)
    assert classes.plots_per_hour() >= 0.99 * fifo.plots_per_hour()


def test_size_classes_reject_zero_big_slots():
    with pytest.raises(ValueError):
        Server(FakeExecutor(Clock()), 1 << 40, big_k=20, max_big=0)

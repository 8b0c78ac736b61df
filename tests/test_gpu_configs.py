"""The batched and serving workloads at their own sizes, bit-exact.

  * batched: 32 plots, k drawn from 22..29 with independent keys (SplitMix64
    seed 4), through vx_plot_batch eagerly and as HIP-graph replays; every
    plot's Table 1, offsets and Table 2 equal a solo vx_plot of the same
    plot (torch.equal on the device), and the two smallest plots equal the
    oracle.  At these sizes every plan has two or three partition passes, so
    the fused hash, the claiming scatters and the gathering sort run on
    concurrent lanes.
  * serving: requests with k from 22..30 (SplitMix64 seed 5) through the
    continuous-batching server; at least three jobs run at once, and every
    job's tables equal a solo run of the same plot made with nothing else on
    the device.
"""
import sys

import numpy as np
import pytest

import oracle
from vx_inputs import batched_plan, derive_key, serving_arrivals

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def vx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_14007_amd as m
    m.lib()
    return m


class Solo:
    """Solo plots, one buffer set per k, reused."""

    def __init__(self, vx):
        self.vx = vx
        self.bufs = {}

    def plot(self, key, k, keep=8):
        if k not in self.bufs and len(self.bufs) >= keep:
            self.bufs.clear()
            torch.cuda.empty_cache()
        b = self.bufs.get(k)
        b = self.vx.plot(key, k, buffers=b) if b is not None else self.vx.plot(key, k)
        self.bufs[k] = b
        self.vx.check_plot(b)
        return b


def _same(vx, a, b, what):
    assert torch.equal(a.t1_keys, b.t1_keys), f"{what}: Table-1 keys differ"
    assert torch.equal(a.t1_nonces, b.t1_nonces), f"{what}: Table-1 nonces differ"
    assert torch.equal(a.bucket_offsets, b.bucket_offsets), f"{what}: offsets differ"
    n = vx.t2_count(b)
    assert vx.t2_count(a) == n, f"{what}: |Table 2| differs"
    assert torch.equal(a.t2[:n], b.t2[:n]), f"{what}: Table 2 differs"


def test_batched_config_equals_solo_plots_eager_and_graph(vx):
    from paper_2606_14007_amd import batch as B
    specs = batched_plan(32)
    assert sorted({s.k for s in specs}) == list(range(22, 30))
    bt = B.alloc_batch(specs)
    say(f"batched config: 32 plots, k={sorted(s.k for s in specs)}, "
        f"{bt.footprint_bytes() / 2**30:.1f} GiB")
    passes = {s.k: vx.vx_partition_passes(vx.make_params(s.key, s.k)) for s in specs}
    assert min(passes.values()) >= 2 and max(passes.values()) == 3
    B.plot_batch(bt)
    counts = B.check(bt)
    say("batched config: eager batch done")
    solo = Solo(vx)
    for i, (s, b) in enumerate(zip(specs, bt.plots)):
        _same(vx, b, solo.plot(s.key, s.k), f"eager plot {i} (k={s.k})")
    say("batched config: eager batch equals solo plots")
    small = sorted(range(len(specs)), key=lambda i: specs[i].k)[:2]
    for i in small:
        s, b = specs[i], bt.plots[i]
        ref = oracle.plot(s.key, s.k, threads=8)
        assert np.array_equal(vx.u64(b.t1_keys), ref.t1_keys)
        assert np.array_equal(vx.u32(b.t1_nonces), ref.t1_nonces)
        assert np.array_equal(vx.u32(b.bucket_offsets), ref.offsets)
        assert counts[i] == len(ref.t2)
        assert np.array_equal(vx.t2_records(b.t2, counts[i]), ref.t2)
    say(f"batched config: plots {small} (k={[specs[i].k for i in small]}) equal the oracle")
    B.capture(bt)
    for r in range(2):
        for b in bt.plots:
            b.t1_keys.fill_(-1)
            b.t1_nonces.fill_(-1)
            b.t2[: min(b.t2_capacity, 1 << 20)].fill_(-1)
            b.t2_count.zero_()
        other = vx.plot(derive_key(700 + r), 20)   # eager work between replays
        torch.cuda.synchronize()
        B.replay(bt, check_result=True)
        vx.check_plot(other)
        for i, (s, b) in enumerate(zip(specs, bt.plots)):
            _same(vx, b, solo.plot(s.key, s.k), f"replay {r} plot {i} (k={s.k})")
        say(f"batched config: graph replay {r} equals solo plots")


def test_serving_config_jobs_equal_solo_runs(vx):
    from paper_2606_14007_amd.serve import GpuExecutor, Server, jobs_from_arrivals
    arr = serving_arrivals(12, rate_per_s=5000.0)
    ks = [a.k for a in arr]
    assert max(ks) == 30 and min(ks) == 22
    say(f"serving config: 12 requests, k={ks}")
    solo = Solo(vx)
    seen = []

    def on_done(job):
        # The job was served next to others; its solo run is made with
        # nothing else on the device (every stream drained first).
        torch.cuda.synchronize()
        ref = solo.plot(job.key, job.k, keep=1)
        torch.cuda.synchronize()
        assert job.error is None, job.error
        _same(vx, job.result, ref, f"job {job.jid} (k={job.k})")
        seen.append(job.jid)
        say(f"serving config: job {job.jid} (k={job.k}) equals its solo run")

    budget = 160 << 30
    ex = GpuExecutor(slots=4, budget_bytes=budget)
    st = Server(ex, budget, slots=4, on_done=on_done).run(jobs_from_arrivals(arr))
    assert sorted(seen) == list(range(12))
    assert not st.failed()
    assert st.max_concurrent >= 3
    say(f"serving config: max concurrent jobs {st.max_concurrent}")

"""Continuous-batching server on the GPU: requests of mixed k overlap on the
device, and every job's tables equal its solo plot (and the oracle)."""
import numpy as np
import pytest

import oracle
from vx_inputs import serving_arrivals

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_14007_amd as m
    m.lib()
    return m


def test_served_results_equal_solo_and_oracle(vx):
    from paper_2606_14007_amd.serve import GpuExecutor, Server, jobs_from_arrivals
    arr = serving_arrivals(24, rate_per_s=2000.0, k_lo=12, k_hi=19)
    jobs = jobs_from_arrivals(arr)
    got = {}

    def on_done(job):
        b = job.result
        n = vx.t2_count(b)
        got[job.jid] = (vx.u64(b.t1_keys), vx.u32(b.t1_nonces), vx.u32(b.bucket_offsets),
                        vx.t2_records(b.t2, n), n)

    budget = 8 << 30
    ex = GpuExecutor(slots=4, budget_bytes=budget)
    st = Server(ex, budget, slots=4, on_done=on_done).run(jobs)
    assert len(st.jobs) == len(jobs) and st.max_concurrent > 1
    for j in jobs:
        solo = vx.plot(j.key, j.k)
        torch.cuda.synchronize()
        k1, n1, off, t2, n = got[j.jid]
        assert np.array_equal(k1, vx.u64(solo.t1_keys))
        assert np.array_equal(n1, vx.u32(solo.t1_nonces))
        assert np.array_equal(off, vx.u32(solo.bucket_offsets))
        assert n == vx.t2_count(solo)
        assert np.array_equal(t2, vx.t2_records(solo.t2, n))
    for j in jobs[:4]:
        ref = oracle.plot(j.key, j.k, threads=8)
        k1, n1, off, t2, n = got[j.jid]
        assert np.array_equal(k1, ref.t1_keys) and np.array_equal(t2, ref.t2)

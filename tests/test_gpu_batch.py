"""Batched plots (vx_plot_batch) and their HIP-graph replay, against the
oracle and against solo vx_plot runs -- bit-exact."""
import numpy as np
import pytest

import oracle
from vx_inputs import PlotSpec, batched_plan, derive_key

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_14007_amd as m
    m.lib()
    return m


def _specs():
    # uneven k, independent keys, one threshold widened so Table 2 is busy
    ks = [16, 10, 18, 13, 17, 12, 15, 14]
    out = [PlotSpec(k=k, key=derive_key(100 + i)) for i, k in enumerate(ks)]
    return out


def _check(vx, b, ref):
    assert np.array_equal(vx.u64(b.t1_keys), ref.t1_keys)
    assert np.array_equal(vx.u32(b.t1_nonces), ref.t1_nonces)
    assert np.array_equal(vx.u32(b.bucket_offsets), ref.offsets)
    cnt = vx.t2_count(b)
    assert cnt == len(ref.t2)
    assert np.array_equal(vx.t2_records(b.t2, cnt), ref.t2)


@pytest.fixture(scope="module")
def refs():
    return [oracle.plot(s.key, s.k, threads=8) for s in _specs()]


def test_batch_equals_oracle(vx, refs):
    from paper_2606_14007_amd import batch as B
    bt = B.alloc_batch(_specs())
    assert len(set(w.data_ptr() for w in bt.workspaces)) <= B.LANES
    B.plot_batch(bt)
    torch.cuda.synchronize()
    for b, ref in zip(bt.plots, refs):
        _check(vx, b, ref)


def test_batch_with_tunings_and_two_lanes(vx, refs):
    from paper_2606_14007_amd import batch as B
    specs = _specs()
    tun = [vx.make_tuning(group_cap=128) if i % 2 else vx.make_tuning(match_chunk_bits=7)
           for i in range(len(specs))]
    bt = B.alloc_batch(specs, tunings=tun, lanes=2)
    B.plot_batch(bt)
    torch.cuda.synchronize()
    for b, ref in zip(bt.plots, refs):
        _check(vx, b, ref)


def test_batch_equals_solo_plots(vx):
    from paper_2606_14007_amd import batch as B
    specs = [PlotSpec(k=s.k, key=s.key) for s in batched_plan(6, k_lo=14, k_hi=20)]
    bt = B.alloc_batch(specs)
    B.plot_batch(bt)
    solo = [vx.plot(s.key, s.k) for s in specs]
    torch.cuda.synchronize()
    for a, b in zip(bt.plots, solo):
        assert torch.equal(a.t1_keys, b.t1_keys) and torch.equal(a.t1_nonces, b.t1_nonces)
        assert torch.equal(a.bucket_offsets, b.bucket_offsets)
        n = vx.t2_count(b)
        assert vx.t2_count(a) == n and torch.equal(a.t2[:n], b.t2[:n])


def test_graph_replay_recomputes_every_time(vx, refs):
    """Capture once, then replay three times; before each replay the outputs
    are wiped and unrelated eager work runs, and every replay is checked."""
    from paper_2606_14007_amd import batch as B
    bt = B.capture(B.alloc_batch(_specs()))
    for r in range(3):
        for b in bt.plots:
            b.t1_keys.fill_(-1)
            b.t1_nonces.fill_(-1)
            b.t2.fill_(-1)
            b.t2_count.zero_()
        other = vx.plot(derive_key(900 + r), 12)  # eager work between replays
        torch.cuda.synchronize()
        B.replay(bt)
        torch.cuda.synchronize()
        for b, ref in zip(bt.plots, refs):
            _check(vx, b, ref)
        assert vx.t2_count(other) >= 0


def test_batch_fused_fronts_mixed_plans(vx, refs):
    """Plans whose hash files two passes and that ask for it share fused
    hash launches across plots (a device work list of slices); the others
    run whole on their lanes.  Two lanes, so workspaces are shared and the batch runs in
    several rounds.  Mixed: sliced and one-launch fronts, three passes, a
    pipelined tail, and one-pass plots."""
    from paper_2606_14007_amd import batch as B
    specs = _specs()  # k = 16, 10, 18, 13, 17, 12, 15, 14
    tun = []
    for i, s in enumerate(specs):
        if i % 4 == 0:
            tun.append(vx.make_tuning(group_bits=s.k - 5, hash_slices=3))
        elif i % 4 == 1:
            tun.append(vx.make_tuning(group_bits=max(10, s.k - 2), hash_slices=1, tail_slices=2))
        elif i % 4 == 2:
            tun.append(vx.make_tuning(group_bits=min(s.k + 2, 18), hash_slices=5))
        else:
            tun.append(None)
    tun = [t if t is not None else vx.make_tuning() for t in tun]
    for t in tun:
        t.batch_shared_hash = 1
    fused = [vx.vx_partition_passes(vx.make_params(s.key, s.k), t) >= 2 for s, t in zip(specs, tun)]
    assert 2 <= sum(fused) < len(specs)
    bt = B.alloc_batch(specs, tunings=tun, lanes=2)
    B.plot_batch(bt, check_result=True)
    torch.cuda.synchronize()
    for b, ref in zip(bt.plots, refs):
        _check(vx, b, ref)
    B.capture(bt)
    for r in range(2):
        for b in bt.plots:
            b.t1_keys.fill_(-1)
            b.t2_count.zero_()
        B.replay(bt, check_result=True)
        torch.cuda.synchronize()
        for b, ref in zip(bt.plots, refs):
            _check(vx, b, ref)


def test_batch_three_pass_fronts_and_replay(vx, refs):
    """Plans that file all three partition passes in their sliced hash
    launches (the second pass into per-slice regions, the third into the
    shared ones) mixed with two-pass sliced and one-launch plans, two lanes
    sharing workspaces, eager and then under graph replay."""
    from paper_2606_14007_amd import batch as B
    specs = _specs()  # k = 16, 10, 18, 13, 17, 12, 15, 14
    tun = []
    for i, s in enumerate(specs):
        if i % 3 == 0:
            tun.append(vx.make_tuning(group_bits=18, hash_slices=3 + i % 2))
        elif i % 3 == 1:
            tun.append(vx.make_tuning(group_bits=18, hash_slices=2, front_subtile=4096))
        else:
            tun.append(vx.make_tuning(hash_slices=2, front_passes=2))
    deep = [vx.vx_front_passes(vx.make_params(s.key, s.k), t) == 3 for s, t in zip(specs, tun)]
    assert 2 <= sum(deep) < len(specs)
    bt = B.alloc_batch(specs, tunings=tun, lanes=2)
    B.plot_batch(bt, check_result=True)
    torch.cuda.synchronize()
    for b, ref in zip(bt.plots, refs):
        _check(vx, b, ref)
    B.capture(bt)
    for r in range(2):
        for b in bt.plots:
            b.t1_keys.fill_(-1)
            b.t1_nonces.fill_(-1)
            b.t2_count.zero_()
        other = vx.plot(derive_key(950 + r), 13)
        torch.cuda.synchronize()
        B.replay(bt, check_result=True)
        torch.cuda.synchronize()
        for b, ref in zip(bt.plots, refs):
            _check(vx, b, ref)
        assert vx.t2_count(other) >= 0

"""GPU parity of chunked plots (vx_plot_chunk, and vx_stage_plot +
vx_plot_staged_chunk) against the oracle, bit-exact.

Chunk r of a plot cut by c bits is the plot restricted to the buckets whose
top c bits equal r: Table 1 is the oracle's slice between those buckets'
offsets, the bucket offsets are the oracle's shifted to start at 0 (clamped
to [0, m] outside the range), and Table 2 is the contiguous slice of the
oracle's canonical Table 2 whose first member lies in the range (pairs never
cross buckets).  One set of buffers serves every chunk in turn, so stale
contents of an earlier chunk would show.
"""
import numpy as np
import pytest

import oracle
from vx_inputs import derive_key
from paper_2606_14007_amd import _native as N

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

KEY0 = derive_key(0)


@pytest.fixture(scope="module")
def vx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_14007_amd as m
    m.lib()
    return m


def _expected_chunk(ref, c, r):
    n = len(ref.t1_keys)
    off = ref.offsets.astype(np.int64)
    b0, b1 = r << (24 - c), (r + 1) << (24 - c)
    lo, hi = int(off[b0]), int(off[b1])
    rank = np.empty(n, np.int64)
    rank[ref.t1_nonces] = np.arange(n)
    ra = rank[ref.t2["nonce_a"]]
    p0, p1 = np.searchsorted(ra, lo), np.searchsorted(ra, hi)
    return (ref.t1_keys[lo:hi], ref.t1_nonces[lo:hi], np.clip(off - lo, 0, hi - lo).astype(np.uint32),
            ref.t2[p0:p1])


def _check_chunk(vx, b, ref, c, r):
    torch.cuda.synchronize()
    ek, en, eoff, et2 = _expected_chunk(ref, c, r)
    m = int(b.t1_count.item())
    assert m == len(ek)
    assert vx.device_status(b.workspace) == 0
    assert np.array_equal(vx.u64(b.t1_keys[:m]), ek)
    assert np.array_equal(vx.u32(b.t1_nonces[:m]), en)
    assert np.array_equal(vx.u32(b.bucket_offsets), eoff)
    cnt = vx.t2_count(b)
    assert cnt == len(et2)
    assert np.array_equal(vx.t2_records(b.t2, cnt), et2)
    return m, cnt


CASES = [
    (20, 2, None),
    (18, 1, None),
    (16, 3, 1 << 44),
    (14, 2, (1 << 64) - 1),
    (13, 2, 0),
    (12, 0, None),
    (9, 4, 1 << 50),
    (3, 3, None),
    (1, 1, None),
]


@pytest.mark.parametrize("k,c,T", CASES)
def test_chunks_match_the_oracle(vx, k, c, T):
    ref = oracle.plot(KEY0, k, threshold=T, threads=8)
    b = vx.alloc_chunk(k, c, threshold=T)
    total1 = total2 = 0
    for r in range(1 << c):
        print(f"k={k} c={c} chunk={r}", flush=True)
        vx.plot_chunk(KEY0, k, c, r, b, threshold=T)
        m, cnt = _check_chunk(vx, b, ref, c, r)
        total1 += m
        total2 += cnt
    assert total1 == 1 << k
    assert total2 == len(ref.t2)


@pytest.mark.parametrize("k,c,T", CASES)
def test_staged_chunks_match_the_oracle(vx, k, c, T):
    # Chunks in reverse order: the stage is read, never consumed.
    ref = oracle.plot(KEY0, k, threshold=T, threads=8)
    st = vx.stage_plot(KEY0, k, c)
    b = vx.alloc_staged_chunk(k, c, threshold=T)
    total1 = total2 = 0
    for r in reversed(range(1 << c)):
        print(f"staged k={k} c={c} chunk={r}", flush=True)
        vx.plot_staged_chunk(KEY0, st, r, b, threshold=T)
        m, cnt = _check_chunk(vx, b, ref, c, r)
        total1 += m
        total2 += cnt
    assert vx.device_status(st.data) == 0
    assert total1 == 1 << k
    assert total2 == len(ref.t2)


@pytest.mark.parametrize("tun", [
    dict(group_cap=64),
    dict(group_bits=14, pass1_bits=4, pass2_bits=5),  # three passes
    dict(group_bits=16, match_chunk_bits=6),
    dict(pipeline_slices=4),                          # ignored by staged plots
])
def test_staged_chunk_tunings(vx, tun):
    k, c = 17, 2
    ref = oracle.plot(KEY0, k, threads=8)
    t = vx.make_tuning(**tun)
    st = vx.stage_plot(KEY0, k, c, tuning=t)
    b = vx.alloc_staged_chunk(k, c, tuning=t)
    for r in range(1 << c):
        vx.plot_staged_chunk(KEY0, st, r, b, tuning=t)
        _check_chunk(vx, b, ref, c, r)
    # the same chunk again, after the others
    vx.plot_staged_chunk(KEY0, st, 1, b, tuning=t)
    _check_chunk(vx, b, ref, c, 1)


@pytest.mark.parametrize("k,c,tun,T", [
    (20, 1, dict(hash_slices=4, group_bits=18), None),
    (22, 2, dict(hash_slices=16, group_bits=20), None),
    (18, 2, dict(hash_slices=3, group_bits=17), 1 << 47),
    (21, 1, dict(hash_slices=5, group_bits=17, front_subtile=2048), None),
])
def test_staged_chunks_sliced_front(vx, k, c, tun, T):
    """A stage hashed in slices with all three partition passes in its
    launches (the form a k=32 stage takes): it holds each chunk's third-pass
    regions, and a chunk only gathers, sorts and matches them."""
    t = vx.make_tuning(**tun)
    p = vx.make_params(KEY0, k)
    assert N.vx_stage_bytes(p, c, t) != N.vx_stage_bytes(p, c, vx.make_tuning(**dict(tun, hash_slices=1)))
    ref = oracle.plot(KEY0, k, threshold=T, threads=8)
    st = vx.stage_plot(KEY0, k, c, tuning=t)
    b = vx.alloc_staged_chunk(k, c, threshold=T, tuning=t)
    total1 = total2 = 0
    for r in reversed(range(1 << c)):
        print(f"sliced stage k={k} c={c} chunk={r}", flush=True)
        vx.plot_staged_chunk(KEY0, st, r, b, threshold=T, tuning=t)
        m, cnt = _check_chunk(vx, b, ref, c, r)
        total1 += m
        total2 += cnt
    assert vx.device_status(st.data) == 0
    assert total1 == 1 << k
    assert total2 == len(ref.t2)
    vx.plot_staged_chunk(KEY0, st, 0, b, threshold=T, tuning=t)  # again, after the others
    _check_chunk(vx, b, ref, c, 0)


def test_sliced_stage_region_overflow_is_reported(vx):
    """Regions of a stage hashed in slices shrunk below their contents (a
    test hook) set the overflow bit in the stage's status word."""
    t = vx.make_tuning(hash_slices=4, group_bits=18, region_pct=25)
    st = vx.stage_plot(KEY0, 18, 1, tuning=t)
    torch.cuda.synchronize()
    assert vx.device_status(st.data) & N.VX_DEV_STATUS_REGION_OVERFLOW


def test_staged_chunk_checks_the_stage(vx):
    k, c = 14, 1
    st = vx.stage_plot(derive_key(5), k, c)
    b = vx.alloc_staged_chunk(k, c)
    with pytest.raises(vx.VxError) as e:
        vx.plot_staged_chunk(KEY0, st, 0, b)   # stage made for another key
    assert e.value.status == N.VX_ERR_INVALID_ARG
    with pytest.raises(vx.VxError) as e:
        vx.plot_staged_chunk(derive_key(5), st, 0, b, tuning=vx.make_tuning(group_bits=11))
    assert e.value.status in (N.VX_ERR_INVALID_ARG, N.VX_ERR_WORKSPACE)
    # and works for the right key afterwards
    ref = oracle.plot(derive_key(5), k)
    vx.plot_staged_chunk(derive_key(5), st, 1, b)
    _check_chunk(vx, b, ref, c, 1)


def test_chunks_concatenate_to_the_whole_plot(vx):
    k, c = 17, 2
    whole = vx.plot(KEY0, k)
    torch.cuda.synchronize()
    b = vx.alloc_chunk(k, c)
    keys, nonces, t2, offs = [], [], [], []
    base = 0
    for r in range(1 << c):
        vx.plot_chunk(KEY0, k, c, r, b)
        torch.cuda.synchronize()
        m = int(b.t1_count.item())
        keys.append(vx.u64(b.t1_keys[:m]))
        nonces.append(vx.u32(b.t1_nonces[:m]))
        t2.append(vx.t2_records(b.t2, vx.t2_count(b)))
        o = vx.u32(b.bucket_offsets).astype(np.int64)
        b0, b1 = r << (24 - c), (r + 1) << (24 - c)
        offs.append(o[b0:b1] + base)
        base += m
    assert np.array_equal(np.concatenate(keys), vx.u64(whole.t1_keys))
    assert np.array_equal(np.concatenate(nonces), vx.u32(whole.t1_nonces))
    assert np.array_equal(np.concatenate(offs + [np.array([base])]),
                          vx.u32(whole.bucket_offsets).astype(np.int64))
    assert np.array_equal(np.concatenate(t2), vx.t2_records(whole.t2, vx.t2_count(whole)))


def test_many_mostly_empty_chunks(vx):
    # 256 records over 256 chunks: most chunks hold zero, one or two records.
    k, c = 8, 8
    ref = oracle.plot(KEY0, k, threshold=1 << 60)
    b = vx.alloc_chunk(k, c, threshold=1 << 60)
    empty = 0
    for r in range(1 << c):
        vx.plot_chunk(KEY0, k, c, r, b, threshold=1 << 60)
        m, _ = _check_chunk(vx, b, ref, c, r)
        empty += m == 0
    assert empty > 0


@pytest.mark.parametrize("tun", [
    dict(group_cap=64),                          # oversized groups take the fallback
    dict(group_bits=4, match_chunk_bits=6),      # one pass, tiny match chunks
    dict(group_bits=13, pass1_bits=5, pass2_bits=4),
    dict(h1_tiles=3),
    dict(group_bits=14, pipeline_slices=4),      # the pipelined plan's 2-6-6 digit split
])
def test_chunk_tunings(vx, tun):
    k, c = 16, 2
    ref = oracle.plot(KEY0, k, threads=8)
    t = vx.make_tuning(**tun)
    b = vx.alloc_chunk(k, c, tuning=t)
    for r in range(1 << c):
        vx.plot_chunk(KEY0, k, c, r, b, tuning=t)
        _check_chunk(vx, b, ref, c, r)


def test_chunk_over_capacity_is_reported(vx):
    k, c = 14, 1
    small = vx.alloc_chunk(k, c, t1_capacity=1 << 12)
    with pytest.raises(vx.VxError) as e:
        vx.plot_chunk(KEY0, k, c, 0, small)
    assert e.value.status == N.VX_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert int(small.t1_count.item()) > 1 << 12  # the records the chunk holds
    # the same device afterwards plots a chunk correctly
    ref = oracle.plot(KEY0, k)
    b = vx.alloc_chunk(k, c)
    vx.plot_chunk(KEY0, k, c, 0, b)
    _check_chunk(vx, b, ref, c, 0)


def test_staged_chunks_generator_makes_the_whole_plot(vx):
    k, c = 18, 2
    ref = oracle.plot(KEY0, k, threads=8)
    keys, t2 = [], []
    for r, b in vx.staged_chunks(KEY0, k, c):
        torch.cuda.synchronize()
        m = int(b.t1_count.item())
        keys.append(vx.u64(b.t1_keys[:m]))
        t2.append(vx.t2_records(b.t2, vx.t2_count(b)))
    assert np.array_equal(np.concatenate(keys), ref.t1_keys)
    assert np.array_equal(np.concatenate(t2), ref.t2)

"""GPU parity: the HIP path through the C ABI against the oracle, bit-exact.

Every input is seeded (vx_inputs) and every expected value comes from the
oracle.  Sizes span one to many tiles, groups and match chunks with ragged
tails; tunings that force the oversized-group fallback are included.
"""
import numpy as np
import pytest

import oracle
from vx_inputs import derive_key

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


def _crowded_keys(k, nbuckets, seed, ties=0):
    rng = np.random.default_rng(seed)
    n = 1 << k
    prefixes = rng.choice(1 << 24, size=nbuckets, replace=False).astype(np.uint64)
    low = rng.integers(0, 1 << 40, size=n, dtype=np.uint64)
    keys = (prefixes[rng.integers(0, nbuckets, size=n)] << np.uint64(40)) | low
    if ties:
        keys[rng.integers(0, n, size=ties)] = keys[rng.integers(0, n, size=ties)]
    return keys


def _to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a).view(dtype)).cuda()


def _assert_plot_equal(vx, b, ref):
    torch.cuda.synchronize()
    assert vx.device_status(b.workspace) == 0
    assert np.array_equal(vx.u64(b.t1_keys), ref.t1_keys)
    assert np.array_equal(vx.u32(b.t1_nonces), ref.t1_nonces)
    assert np.array_equal(vx.u32(b.bucket_offsets), ref.offsets)
    cnt = vx.t2_count(b)
    assert cnt == len(ref.t2)
    assert np.array_equal(vx.t2_records(b.t2, cnt), ref.t2)


@pytest.mark.parametrize("k", [1, 2, 5, 8, 12, 13, 14, 16])
def test_hash_table1_small(vx, k):
    out = vx.hash_table1(KEY0, k)
    torch.cuda.synchronize()
    assert np.array_equal(vx.u64(out), oracle.hash_table1(KEY0, k))


def test_hash_table1_k20_several_keys(vx):
    for seed in (0, 1, 77):
        key = derive_key(seed)
        out = vx.hash_table1(key, 20)
        torch.cuda.synchronize()
        assert np.array_equal(vx.u64(out), oracle.hash_table1(key, 20, threads=8))


def test_device_h1_equals_published_keyed_vector(vx):
    """The device's Table-1 hash of nonce 0x03020100 (bytes 00 01 02 03) under
    the key of the BLAKE3 authors' test vectors is their published
    keyed_hash digest, first 8 bytes read big-endian (no oracle involved)."""
    from conftest import golden_lines
    vec = {(int(n), m): bytes.fromhex(h) for n, m, h in golden_lines("blake3_test_vectors.txt")}
    key = b"whats the Elvish word for friend"
    out = vx.hash_table1(key, 26)
    torch.cuda.synchronize()
    assert int(vx.u64(out[0x03020100:0x03020101])[0]) == int.from_bytes(vec[(4, "keyed_hash")][:8], "big")


@pytest.mark.parametrize("k", [1, 3, 9, 12, 13, 15, 17, 20, 21, 22, 24])
def test_plot_default_threshold(vx, k):
    b = vx.plot(KEY0, k)
    _assert_plot_equal(vx, b, oracle.plot(KEY0, k, threads=8))


@pytest.mark.parametrize("k,hq", [(20, 2), (20, 7), (22, 8), (24, 4), (24, 16), (26, 4)])
def test_plot_sliced_hash(vx, k, hq):
    """The plot hashed in nonce slices, each slice's second pass beside the
    next slice's hash, with the default group bits (two passes up to k=25,
    three above)."""
    b = vx.plot(KEY0, k, tuning=vx.make_tuning(hash_slices=hq))
    _assert_plot_equal(vx, b, oracle.plot(KEY0, k, threads=8))


@pytest.mark.parametrize("k,hq,gb", [(20, 2, 18), (21, 3, 17), (22, 16, 20), (24, 16, 0), (24, 7, 18),
                                     (26, 16, 17), (26, 4, 0), (22, 32, 20), (25, 24, 18), (26, 32, 17)])
def test_plot_three_pass_front(vx, k, hq, gb):
    """Three partition passes in the sliced hash launches: launch i hashes
    slice i, files slice i - 1 by the second digit into regions of its own
    and slice i - 2 by the third into the shared regions that the sort
    gathers from (24 and 26 without group bits: 13 and 15 group bits, where
    the plan falls back to two passes)."""
    t = vx.make_tuning(hash_slices=hq, group_bits=gb)
    p = vx.make_params(KEY0, k)
    assert vx.vx_hash_slices(p, t) == hq
    assert vx.vx_front_passes(p, t) == vx.vx_partition_passes(p, t)
    b = vx.plot(KEY0, k, tuning=t)
    _assert_plot_equal(vx, b, oracle.plot(KEY0, k, threads=8))


@pytest.mark.parametrize("k,hq,gb,fp", [(22, 5, 18, 3), (24, 16, 20, 3), (26, 16, 17, 3), (25, 8, 17, 2)])
def test_plot_wide_front_items(vx, k, hq, gb, fp):
    """The sliced hash launches with 512-thread work-groups on 4096-record
    sub-tiles, filing two or three passes."""
    t = vx.make_tuning(hash_slices=hq, group_bits=gb, front_passes=fp, front_subtile=4096)
    assert vx.vx_front_passes(vx.make_params(KEY0, k), t) == fp
    b = vx.plot(KEY0, k, tuning=t)
    _assert_plot_equal(vx, b, oracle.plot(KEY0, k, threads=8))


@pytest.mark.parametrize("k,hq,zt,gb", [(20, 1, 4, 12), (22, 4, 8, 0), (24, 8, 16, 0), (22, 2, 8, 18),
                                        (23, 16, 8, 20)])
def test_plot_pipelined_tail(vx, k, hq, zt, gb):
    """The third pass, the sort and the match pipelined over zt slices (one
    persistent launch per step), after a one-launch or sliced hash; 18 and
    20 group bits give three passes at these sizes."""
    t = vx.make_tuning(hash_slices=hq, tail_slices=zt, group_bits=gb)
    assert vx.vx_tail_slices(vx.make_params(KEY0, k), t) == zt
    b = vx.plot(KEY0, k, tuning=t)
    _assert_plot_equal(vx, b, oracle.plot(KEY0, k, threads=8))


@pytest.mark.parametrize("k,T", [(14, 1 << 44), (16, 1 << 42), (18, 1 << 41), (12, 0),
                                 (16, (1 << 64) - 1)])
def test_plot_thresholds(vx, k, T):
    b = vx.plot(KEY0, k, threshold=T)
    _assert_plot_equal(vx, b, oracle.plot(KEY0, k, threshold=T, threads=8))


TUNINGS = [
    dict(group_bits=4),                       # groups near LDS capacity -> many take the fallback
    dict(group_bits=10, pass1_bits=3),        # two passes with a narrow first digit
    dict(group_bits=12, pass1_bits=11),       # wide first digit, 1-bit second pass
    dict(group_bits=15, pass1_bits=5, pass2_bits=5),  # three passes
    dict(group_bits=18),                      # three default passes, tiny groups
    dict(group_cap=64),                       # almost every group takes the fallback
    dict(group_cap=200, match_chunk_bits=7),  # fallback + small match chunks
    dict(match_chunk_bits=6),                 # smallest match chunks
    dict(match_chunk_bits=9, h1_tiles=7),     # ragged hash tiles
    dict(fused_sort_match=1),                 # one fused sort + match kernel (look-back bases)
    dict(fused_sort_match=1, group_cap=64),   # fused kernel, most groups on its slow path
    dict(fused_sort_match=1, group_bits=3),   # fused kernel, few large groups
    dict(group_bits=20, pass1_bits=10),       # a 10-bit pass (wide-digit scatter)
    dict(group_bits=13, pipeline_slices=2),   # pipelined tail: 1-6-6 passes, two slices
    dict(group_bits=14, pipeline_slices=4),   # four slices, one per first-pass segment
    dict(group_bits=12, pipeline_slices=3),   # pipelined with two passes, uneven slices
    dict(separate_hash=1),                    # hash and first pass as two kernels
    dict(separate_hash=1, group_bits=15, pass1_bits=5, pass2_bits=5),
    dict(group_bits=16, pass1_bits=8),        # fused hash with 256 first-pass regions
    dict(group_bits=9, pass1_bits=1, pass2_bits=4),  # fused hash with two regions, three passes
    dict(group_bits=16, pipeline_slices=16, group_cap=64),   # 16 slices, oversized groups
    dict(group_bits=15, pipeline_slices=5, match_chunk_bits=6),  # many small chunks per slice
    dict(group_bits=9, pipeline_slices=4),    # one pass: nothing to pipeline
    dict(hash_slices=2),                      # sliced hash, both passes in its launches (3-2)
    dict(hash_slices=3, group_bits=12),       # uneven slices, 6-6
    dict(hash_slices=8, group_bits=15),       # 1-7-7: a claiming third pass after the slices
    dict(hash_slices=16, group_bits=14),      # sixteen slices, 7-7
    dict(hash_slices=4, group_bits=13, pass1_bits=3),    # 3-7-3, three passes in the hash launches
    dict(hash_slices=4, group_bits=13, pass1_bits=3, front_passes=2),  # 3-7-3, third pass after
    dict(hash_slices=5, group_bits=18),       # 4-7-7 over five uneven slices, seven launches
    dict(hash_slices=16, group_bits=17, group_cap=64),  # 3-7-7: sixteen slices, oversized groups
    dict(hash_slices=3, group_bits=16, pass1_bits=5, pass2_bits=5, match_chunk_bits=7),  # 5-5-6
    dict(hash_slices=4, group_bits=18, front_subtile=2048),   # 2048-record items, three passes
    dict(hash_slices=2, group_bits=20, front_passes=2, front_subtile=4096),  # 4096, two passes
    dict(hash_slices=6, group_bits=16, front_subtile=4096),   # 4096-record items, 8-8 digits
    dict(hash_slices=5, group_bits=16, fused_sort_match=1),  # sliced hash, fused tail
    dict(hash_slices=2, group_bits=20),       # 6-7-7 (the k=31 split), tiny groups, all three passes
                                              # in the hash launches
    dict(hash_slices=2, group_bits=20, front_passes=2),  # the same with a separate third pass
    dict(hash_slices=4, group_cap=64),        # sliced hash, oversized groups
    dict(hash_slices=6, group_bits=16),       # 8-8: the sliced kernel with 256 counters
    dict(hash_slices=3, group_bits=17, pass1_bits=8, pass2_bits=8),  # 8-8-1
    dict(tail_slices=2, group_bits=10),       # pipelined tail: sort + match over two slices
    dict(tail_slices=4, group_bits=15, pass1_bits=5, pass2_bits=5),  # third pass, sort, match pipelined
    dict(tail_slices=3, hash_slices=4, group_bits=20),  # sliced hash + pipelined tail, 6-7-7
    dict(tail_slices=16, group_bits=14),      # sixteen slices of two-pass groups
    dict(tail_slices=5, hash_slices=3, group_bits=12),  # uneven tail slices after a sliced hash
    dict(tail_slices=4, group_bits=11, match_chunk_bits=6),  # small match chunks spanning slices
    dict(tail_slices=4, group_cap=64, group_bits=14),   # oversized groups: fallback per slice
]


@pytest.mark.parametrize("tun", TUNINGS, ids=[str(t) for t in TUNINGS])
def test_plot_tunings_do_not_change_outputs(vx, tun):
    k, T = 16, 1 << 44
    ref = oracle.plot(KEY0, k, threshold=T, threads=8)
    t = vx.make_tuning(**tun)
    b = vx.plot(KEY0, k, threshold=T, tuning=t)
    _assert_plot_equal(vx, b, ref)


@pytest.mark.parametrize("T", [1 << 40, 1 << 44])
def test_pipelined_plot_at_large_group_count(vx, T):
    """k=22 with 2^18 groups (the group count of a k=29 plot): the pipelined
    plan (6-6-6 passes, eight slices) and the sequential one against the
    oracle."""
    k = 22
    ref = oracle.plot(KEY0, k, threshold=T, threads=8)
    b = vx.plot(KEY0, k, threshold=T, tuning=vx.make_tuning(group_bits=18, pipeline_slices=8))
    _assert_plot_equal(vx, b, ref)
    b2 = vx.plot(KEY0, k, threshold=T, tuning=vx.make_tuning(group_bits=18))
    _assert_plot_equal(vx, b2, ref)


@pytest.mark.parametrize("T", [1 << 39, 1 << 40, (1 << 64) - 1])
def test_pair_counts_at_the_top_of_the_key_space(vx, T):
    """The key of seed 61 puts three records of its k=22 plot in the last
    bucket.  From T = 2^40 (T >= 2^39 for its upper half) the sort's upper
    bound on a partner's key saturates to all ones there -- the value of the
    sentinels after a group's records -- so those records are counted by
    position instead; the plot must still equal the oracle's."""
    key, k = derive_key(61), 22
    ref = oracle.plot(key, k, threshold=T, threads=8)
    assert ref.offsets[-1] - ref.offsets[-2] >= 2  # records in bucket 2^24 - 1
    b = vx.plot(key, k, threshold=T)
    torch.cuda.synchronize()
    assert vx.device_status(b.workspace) == 0
    assert np.array_equal(vx.u64(b.t1_keys), ref.t1_keys)
    cnt = vx.t2_count(b)
    assert cnt == len(ref.t2)
    assert np.array_equal(vx.t2_records(b.t2, cnt), ref.t2)


@pytest.mark.parametrize("T", [0, 1 << 34, 1 << 37, 1 << 40, (1 << 64) - 1])
def test_bucket_sort_and_match_crowded(vx, T):
    """Caller-supplied keys crowded into few buckets: oversized groups, long
    equal-prefix runs, duplicate keys (nonce tie-break), many pairs."""
    k = 14
    keys = _crowded_keys(k, nbuckets=9, seed=5, ties=40)
    ref_t1k, ref_t1n, ref_off = oracle.bucket_sort(k, keys)
    ref_t2, ref_cnt = oracle.match_table2(KEY0, T, ref_t1k, ref_t1n, ref_off, threads=8)
    dkeys = _to_dev(keys, np.int64)
    t1k, t1n, off, ws = vx.bucket_sort(KEY0, k, dkeys)
    torch.cuda.synchronize()
    assert vx.device_status(ws) == 0
    assert np.array_equal(vx.u64(t1k), ref_t1k)
    assert np.array_equal(vx.u32(t1n), ref_t1n)
    assert np.array_equal(vx.u32(off), ref_off)
    t2, cnt = vx.match_table2(KEY0, k, t1k, t1n, off, threshold=T, t2_capacity=ref_cnt + 5)
    torch.cuda.synchronize()
    assert vx.t2_count(cnt) == ref_cnt
    assert np.array_equal(vx.t2_records(t2, ref_cnt), ref_t2)


def test_table2_count_beyond_32_bits(vx):
    """All 2^17 records in one bucket and every pair within the threshold:
    |Table 2| = n (n - 1) / 2 > 2^32, each chunk's count above 2^26, so the
    64-bit scans carry across 32 bits.  Only the first records fit the
    capacity; the count is exact (a closed form, no oracle run)."""
    k = 17
    keys = _crowded_keys(k, nbuckets=1, seed=11)
    n = len(keys)
    expect = n * (n - 1) // 2
    assert expect > 1 << 32
    dkeys = _to_dev(keys, np.int64)
    t1k, t1n, off, ws = vx.bucket_sort(KEY0, k, dkeys)
    torch.cuda.synchronize()
    assert vx.device_status(ws) == 0
    t2, cnt = vx.match_table2(KEY0, k, t1k, t1n, off, threshold=(1 << 64) - 1, t2_capacity=4096)
    torch.cuda.synchronize()
    assert vx.t2_count(cnt) == expect
    # The first records in canonical order: Table-1 record 0 with its
    # partners 1, 2, ..., the hashes of a few checked with the oracle's H2.
    recs = vx.t2_records(t2, 4096)
    nonces = vx.u32(t1n)
    assert np.array_equal(recs["nonce_a"], np.full(4096, nonces[0], dtype=np.uint32))
    assert np.array_equal(recs["nonce_b"], nonces[1:4097])
    for i in (0, 1, 2047, 4095):
        assert int(recs["hash2"][i]) == oracle.h2(KEY0, int(nonces[0]), int(nonces[i + 1]))


@pytest.mark.parametrize("cap", [0, 2600, 3072])
def test_group_sizes_around_the_lds_capacities(vx, cap):
    """Sort groups of exactly 2560 (the default capacity), 2561, 2800 and
    3072 records (the largest capacity): the four-per-CU kernel, the
    3072-record kernel and the fallback share the groups by capacity, with
    the same outputs."""
    k, gb = 14, 3
    sizes = [2561, 3072, 2800, 2560, 2048, 1800, 1000]
    sizes.append((1 << k) - sum(sizes))
    rng = np.random.default_rng(11)
    # 16 buckets per group, so that buckets and sub-bins are crowded
    mid = rng.integers(0, 1 << 21, size=(len(sizes), 16), dtype=np.uint64)
    parts = []
    for g, s in enumerate(sizes):
        a = ((np.uint64(g) << np.uint64(61)) | (mid[g][rng.integers(0, 16, size=s)] << np.uint64(40)) |
             rng.integers(0, 1 << 40, size=s, dtype=np.uint64))
        a[:3] = a[3:6]  # equal keys (the nonce breaks the tie)
        parts.append(a)
    keys = np.concatenate(parts)
    rng.shuffle(keys)
    T = 1 << 36
    ref_t1k, ref_t1n, ref_off = oracle.bucket_sort(k, keys)
    ref_t2, ref_cnt = oracle.match_table2(KEY0, T, ref_t1k, ref_t1n, ref_off, threads=8)
    t = vx.make_tuning(group_bits=gb, group_cap=cap)
    t1k, t1n, off, ws = vx.bucket_sort(KEY0, k, _to_dev(keys, np.int64), tuning=t)
    torch.cuda.synchronize()
    assert vx.device_status(ws) == 0
    assert np.array_equal(vx.u64(t1k), ref_t1k)
    assert np.array_equal(vx.u32(t1n), ref_t1n)
    assert np.array_equal(vx.u32(off), ref_off)
    t2, cnt = vx.match_table2(KEY0, k, t1k, t1n, off, threshold=T, t2_capacity=ref_cnt + 5)
    torch.cuda.synchronize()
    assert vx.t2_count(cnt) == ref_cnt
    assert np.array_equal(vx.t2_records(t2, ref_cnt), ref_t2)


def test_match_from_oracle_table1(vx):
    """vx_match_table2 on an oracle-built Table 1."""
    k = 18
    T = 1 << 43
    ref = oracle.plot(KEY0, k, threshold=T, threads=8)
    t2, cnt = vx.match_table2(KEY0, k, _to_dev(ref.t1_keys, np.int64),
                              _to_dev(ref.t1_nonces, np.int32), _to_dev(ref.offsets, np.int32),
                              threshold=T)
    torch.cuda.synchronize()
    assert vx.t2_count(cnt) == len(ref.t2)
    assert np.array_equal(vx.t2_records(t2, len(ref.t2)), ref.t2)


def test_t2_capacity_overflow_is_reported_not_written(vx):
    k, T = 16, 1 << 44
    ref = oracle.plot(KEY0, k, threshold=T, threads=8)
    cap = len(ref.t2) // 3
    b = vx.alloc_plot(k, T, t2_capacity=cap + 8)
    sentinel = torch.full((8, 2), -1, dtype=torch.int64, device=b.t2.device)
    b.t2[cap:].copy_(sentinel)
    b2 = vx.PlotBuffers(k, b.t1_keys, b.t1_nonces, b.bucket_offsets, b.t2[:cap], b.t2_count,
                        b.workspace)
    vx.plot(KEY0, k, threshold=T, buffers=b2)
    torch.cuda.synchronize()
    assert vx.t2_count(b2) == len(ref.t2)
    assert np.array_equal(vx.t2_records(b2.t2, cap), ref.t2[:cap])
    assert torch.equal(b.t2[cap:], sentinel)


def test_repeat_runs_are_identical(vx):
    k = 20
    a = vx.plot(KEY0, k)
    b = vx.plot(KEY0, k)
    torch.cuda.synchronize()
    assert torch.equal(a.t1_keys, b.t1_keys) and torch.equal(a.t1_nonces, b.t1_nonces)
    n = vx.t2_count(a)
    assert n == vx.t2_count(b) and torch.equal(a.t2[:n], b.t2[:n])


def test_invalid_arguments_raise(vx):
    with pytest.raises(ValueError):
        vx.make_params(bytes(31), 10)
    p = vx.make_params(KEY0, 0)
    with pytest.raises(vx.VxError):
        vx.vx_hash_table1(p, 0)
    p = vx.make_params(KEY0, 10)
    p.bucket_bits = 20
    with pytest.raises(vx.VxError):
        vx.vx_hash_table1(p, 0)
    with pytest.raises(ValueError):
        vx.plot(KEY0, 10, tuning=vx.make_tuning(group_cap=8))
    b = vx.alloc_plot(10)
    with pytest.raises(vx.VxError):
        vx.plot(KEY0, 10, buffers=b, tuning=vx.make_tuning(group_cap=8))


def test_region_overflow_is_reported(vx):
    """Regions shrunk to a quarter of their capacity (a test hook) must
    overflow, report it in the device status and still finish; the same plan
    at full capacity is exact.  T = 0, so that the records the overflow left
    out of Table 1 cannot make the match walk far."""
    from paper_2606_14007_amd import _native as N
    k = 16
    # a 6-bit first digit: 64 stage regions of ~1024 records, which a quarter
    # of their capacity cannot hold
    small = vx.make_tuning(group_bits=12, pass1_bits=6, region_pct=25)
    b = vx.plot(KEY0, k, threshold=0, tuning=small)
    torch.cuda.synchronize()
    assert vx.device_status(b.workspace) & N.VX_DEV_STATUS_REGION_OVERFLOW
    st = vx.stage_plot(KEY0, k, 1, tuning=small)
    torch.cuda.synchronize()
    assert vx.device_status(st.data) & N.VX_DEV_STATUS_REGION_OVERFLOW
    b = vx.plot(KEY0, k, threshold=0, tuning=vx.make_tuning(group_bits=12, pass1_bits=6))
    _assert_plot_equal(vx, b, oracle.plot(KEY0, k, threshold=0))


@pytest.mark.parametrize("tun", [dict(group_bits=12), dict(group_bits=14, pass1_bits=4, pass2_bits=5),
                                 dict(group_bits=12, hash_slices=4), dict(group_bits=18, hash_slices=3),
                                 dict(group_bits=18, hash_slices=3, front_passes=2),
                                 dict(group_bits=17, hash_slices=2),
                                 dict(group_bits=12, tail_slices=4), dict(group_bits=18, hash_slices=2, tail_slices=3)])
@pytest.mark.parametrize("pct", [10, 25])
def test_region_overflow_with_matching_stays_bounded(vx, tun, pct):
    """Overflowing regions with the default threshold, so that the match
    walks the table: a gathered group holds only its own region's records,
    the holes that overflow leaves in Table 1 carry zero pair counts, and
    the plot finishes with the status bit set.  Table 1 is pre-filled with a
    sentinel, so the records the plot placed are known: each is a genuine
    (H1(nonce), nonce) record, no nonce is placed twice, and every Table-2
    record pairs two placed nonces with the right hash."""
    from paper_2606_14007_amd import _native as N
    k = 16
    tuning = vx.make_tuning(region_pct=pct, **tun)
    b = vx.alloc_plot(k, tuning=tuning)
    b.t1_keys.fill_(-1)
    b.t1_nonces.fill_(-1)
    vx.plot(KEY0, k, buffers=b, tuning=tuning)
    torch.cuda.synchronize()
    assert vx.device_status(b.workspace) & N.VX_DEV_STATUS_REGION_OVERFLOW
    keys, nonces = vx.u64(b.t1_keys), vx.u32(b.t1_nonces)
    placed = nonces != 0xFFFFFFFF
    assert 0 < placed.sum() < 1 << k
    pn = nonces[placed]
    assert len(np.unique(pn)) == len(pn) and np.all(pn < (1 << k))
    assert np.array_equal(keys[placed], oracle.h1_many(KEY0, pn))
    offs = vx.u32(b.bucket_offsets)
    assert np.all(np.diff(offs.astype(np.int64)) >= 0) and offs[-1] == 1 << k
    cnt = vx.t2_count(b)
    assert 0 <= cnt <= b.t2_capacity
    t2 = vx.t2_records(b.t2, cnt)
    ok = set(pn.tolist())
    for r in t2[:2000]:
        assert int(r["nonce_a"]) in ok and int(r["nonce_b"]) in ok
        assert int(r["hash2"]) == oracle.h2(KEY0, int(r["nonce_a"]), int(r["nonce_b"]))

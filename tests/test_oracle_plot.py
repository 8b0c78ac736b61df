"""Pins for the oracle's plot stages (CPU only).

  * Table-1 hash: the C oracle's H1/H2 against the independent Python BLAKE3
    with the message bytes spelled out (LE32 nonce; LE32 a || LE32 b).
  * Table 1: equals numpy.lexsort of the nonce-order hashes by (key64,
    nonce) -- a library sort -- and the bucket offsets equal the cumulative
    numpy.bincount of key64 >> 40.
  * Table 2: brute force over all pairs of a small table, for many
    thresholds, with keys crowded into a few buckets so that pairs exist;
    closed forms T = 0 -> empty and T >= 2^40 -> sum over buckets of C(c, 2).
  * Thread-split and sampled-bucket variants equal the plain oracle.
  * Sanity (statistical, not a pin): |T2| near its expectation at k = 20.
"""
import random

import numpy as np
import pytest

import oracle
from oracle import blake3_py
from vx_inputs import derive_key

KEY0 = derive_key(0)


def _py_h1(key, n):
    return int.from_bytes(blake3_py.blake3(n.to_bytes(4, "little"), key)[:8], "big")


def _py_h2(key, a, b):
    return int.from_bytes(blake3_py.blake3(a.to_bytes(4, "little") + b.to_bytes(4, "little"),
                                           key)[:8], "big")


def test_h1_h2_match_independent_blake3():
    rng = random.Random(3)
    for key in (KEY0, derive_key(17), bytes(32)):
        for _ in range(40):
            n = rng.randrange(1 << 32)
            assert oracle.h1(key, n) == _py_h1(key, n)
            a, b = rng.randrange(1 << 32), rng.randrange(1 << 32)
            assert oracle.h2(key, a, b) == _py_h2(key, a, b)


def test_hash_table1_is_h1_in_nonce_order():
    keys = oracle.hash_table1(KEY0, 10)
    assert keys.dtype == np.uint64 and keys.shape == (1024,)
    for n in (0, 1, 2, 511, 1023):
        assert int(keys[n]) == _py_h1(KEY0, n)


def _check_table1(keys, t1k, t1n, off):
    n = len(keys)
    order = np.lexsort((np.arange(n, dtype=np.uint64), keys))
    assert np.array_equal(t1n, order.astype(np.uint32))
    assert np.array_equal(t1k, keys[order])
    counts = np.bincount((keys >> np.uint64(40)).astype(np.int64), minlength=1 << 24)
    expect_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint32)
    assert np.array_equal(off, expect_off)
    assert off[-1] == n


@pytest.mark.parametrize("k", [1, 4, 12, 16])
def test_table1_equals_library_sort(k):
    keys = oracle.hash_table1(KEY0, k)
    t1k, t1n, off = oracle.bucket_sort(k, keys)
    _check_table1(keys, t1k, t1n, off)


def _crowded_keys(k, nbuckets, seed, ties=0):
    """2^k random keys whose 24-bit prefixes come from a few buckets, with
    some exact duplicates so that the nonce tie-break matters."""
    rng = np.random.default_rng(seed)
    n = 1 << k
    prefixes = rng.choice(1 << 24, size=nbuckets, replace=False).astype(np.uint64)
    low = rng.integers(0, 1 << 40, size=n, dtype=np.uint64)
    keys = (prefixes[rng.integers(0, nbuckets, size=n)] << np.uint64(40)) | low
    if ties:
        src = rng.integers(0, n, size=ties)
        dst = rng.integers(0, n, size=ties)
        keys[dst] = keys[src]
    return keys


def _brute_force_t2(key, keys, T, with_hash=True):
    """All pairs by definition: two records in the same bucket whose keys
    differ by less than T, the smaller (key, nonce) first, listed in Table-1
    order of the first, then of the second record."""
    n = len(keys)
    order = np.lexsort((np.arange(n), keys))
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    k64 = keys.astype(object)
    pairs = []
    for a in range(n):
        for b in range(n):
            if rank[a] >= rank[b]:
                continue
            if (int(k64[a]) >> 40) != (int(k64[b]) >> 40):
                continue
            if int(k64[b]) - int(k64[a]) < T:
                pairs.append((rank[a], rank[b], a, b))
    pairs.sort()
    out = np.zeros(len(pairs), oracle.T2_DTYPE)
    for i, (_, _, a, b) in enumerate(pairs):
        out[i]["nonce_a"] = a
        out[i]["nonce_b"] = b
        if with_hash:
            out[i]["hash2"] = _py_h2(key, a, b)
    return out


@pytest.mark.parametrize("T", [0, 1, 1 << 30, 1 << 34, 1 << 36, 1 << 38, (1 << 40) - 1,
                               1 << 40, (1 << 64) - 1])
def test_table2_brute_force_crowded(T):
    k = 7
    keys = _crowded_keys(k, nbuckets=6, seed=T % 1000 + 11, ties=6)
    t1k, t1n, off = oracle.bucket_sort(k, keys)
    _check_table1(keys, t1k, t1n, off)
    t2, total = oracle.match_table2(KEY0, T, t1k, t1n, off)
    expect = _brute_force_t2(KEY0, keys, T)
    assert total == len(expect)
    assert np.array_equal(t2, expect)


def test_table2_brute_force_real_plot_small_k():
    """A real (hashed) plot at k = 9, threshold widened so that every
    same-bucket pair would count, plus a crowded variant."""
    k = 9
    keys = oracle.hash_table1(KEY0, k)
    t1k, t1n, off = oracle.bucket_sort(k, keys)
    t2, total = oracle.match_table2(KEY0, 1 << 63, t1k, t1n, off)
    assert np.array_equal(t2, _brute_force_t2(KEY0, keys, 1 << 63))


@pytest.mark.parametrize("k", [10, 14])
def test_table2_closed_forms(k):
    keys = _crowded_keys(k, nbuckets=32, seed=k)
    t1k, t1n, off = oracle.bucket_sort(k, keys)
    t2, total = oracle.match_table2(KEY0, 0, t1k, t1n, off)
    assert total == 0 and len(t2) == 0
    counts = np.diff(off.astype(np.int64))
    expect = int(np.sum(counts * (counts - 1) // 2))
    for T in (1 << 40, 1 << 50, (1 << 64) - 1):
        _, total = oracle.match_table2(KEY0, T, t1k, t1n, off, capacity=0)
        assert total == expect


def test_table2_records_satisfy_predicate_and_rehash():
    k = 14
    keys = _crowded_keys(k, nbuckets=200, seed=5, ties=20)
    t1k, t1n, off = oracle.bucket_sort(k, keys)
    T = 1 << 35
    t2, total = oracle.match_table2(KEY0, T, t1k, t1n, off)
    assert total > 1000
    a = t2["nonce_a"].astype(np.int64)
    b = t2["nonce_b"].astype(np.int64)
    ka, kb = keys[a], keys[b]
    assert np.all((ka >> np.uint64(40)) == (kb >> np.uint64(40)))
    assert np.all(kb - ka < np.uint64(T))
    assert np.all((ka < kb) | ((ka == kb) & (a < b)))
    for i in range(0, len(t2), max(1, len(t2) // 50)):
        assert int(t2[i]["hash2"]) == _py_h2(KEY0, int(a[i]), int(b[i]))
    # canonical order: by rank of the first record, then of the second
    rank = np.empty(1 << k, np.int64)
    rank[t1n.astype(np.int64)] = np.arange(1 << k)
    ra, rb = rank[a], rank[b]
    assert np.all((ra[1:] > ra[:-1]) | ((ra[1:] == ra[:-1]) & (rb[1:] > rb[:-1])))


def test_capacity_truncates_but_counts_everything():
    k = 10
    keys = _crowded_keys(k, nbuckets=4, seed=9)
    t1k, t1n, off = oracle.bucket_sort(k, keys)
    full, total = oracle.match_table2(KEY0, 1 << 38, t1k, t1n, off)
    part, total2 = oracle.match_table2(KEY0, 1 << 38, t1k, t1n, off, capacity=17)
    assert total2 == total and np.array_equal(part, full[:17])


def test_threaded_variants_equal_plain():
    k = 16
    plain = oracle.plot(KEY0, k, threads=1)
    mt = oracle.plot(KEY0, k, threads=5)
    assert np.array_equal(plain.keys_nonce_order, mt.keys_nonce_order)
    assert np.array_equal(plain.t1_keys, mt.t1_keys)
    assert np.array_equal(plain.t1_nonces, mt.t1_nonces)
    assert np.array_equal(plain.offsets, mt.offsets)
    assert np.array_equal(plain.t2, mt.t2)
    keys = _crowded_keys(12, nbuckets=8, seed=1)
    a = oracle.match_table2(KEY0, 1 << 36, *oracle.bucket_sort(12, keys))
    b = oracle.match_table2(KEY0, 1 << 36, *oracle.bucket_sort(12, keys, threads=3), threads=3)
    assert a[1] == b[1] and np.array_equal(a[0], b[0])


def test_sampled_buckets_equal_slices_of_full_plot():
    k = 18
    T = 1 << 44  # wide enough that the sampled buckets produce pairs
    full = oracle.plot(KEY0, k, threshold=T, threads=4)
    rng = random.Random(2)
    nonempty = np.nonzero(np.diff(full.offsets.astype(np.int64)) >= 2)[0]
    buckets = sorted(set([0, (1 << 24) - 1] + [int(x) for x in rng.sample(list(nonempty), 40)]
                         + [rng.randrange(1 << 24) for _ in range(10)]))
    s = oracle.sample_buckets(KEY0, k, buckets, threshold=T, threads=3)
    assert list(s.buckets) == buckets
    t1k, t1n, t2 = [], [], []
    pair_lo = {}
    # pair index ranges per bucket in the full Table 2
    first_rank = np.empty(1 << k, np.int64)
    first_rank[full.t1_nonces.astype(np.int64)] = np.arange(1 << k)
    pa = first_rank[full.t2["nonce_a"].astype(np.int64)]
    for i, b in enumerate(buckets):
        lo, hi = int(full.offsets[b]), int(full.offsets[b + 1])
        assert s.bucket_counts[i] == hi - lo
        t1k.append(full.t1_keys[lo:hi])
        t1n.append(full.t1_nonces[lo:hi])
        sel = (pa >= lo) & (pa < hi)
        t2.append(full.t2[sel])
        assert s.pair_counts[i] == int(sel.sum())
    assert np.array_equal(s.t1_keys, np.concatenate(t1k))
    assert np.array_equal(s.t1_nonces, np.concatenate(t1n))
    assert np.array_equal(s.t2, np.concatenate(t2))
    assert s.pair_counts.sum() > 0


def test_k20_table2_size_is_near_expectation():
    """Sanity only: with T = 2^44 every same-bucket pair matches at k = 20,
    so E|T2| = 2^24 * C(lambda) with lambda = 1/16, about 2^15."""
    p = oracle.plot(KEY0, 20, threads=4)
    assert 30000 < len(p.t2) < 35600
    _check_table1(p.keys_nonce_order, p.t1_keys, p.t1_nonces, p.offsets)

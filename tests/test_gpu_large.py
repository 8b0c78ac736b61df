"""GPU parity at the full plot sizes: k = 27 and k = 29 bit-exact against the
oracle in full; k = 31 (about 120 GB on the device) and k = 32 in two chunks
(112 or 170 GB) bit-exact on oracle-computed sampled buckets and sampled
records, plus whole-table properties checked on the device with torch:
Table 1 sorted by (key64, nonce) and a permutation of all nonces, bucket
offsets equal to the bucket histogram's prefix sums, every Table-2 record
valid and in canonical order, and |Table 2| equal to an independent pair
count from searchsorted."""
import os
import random

import numpy as np
import pytest

import oracle
from vx_inputs import derive_key, sampled_buckets

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

KEY0 = derive_key(0)
THREADS = max(1, min(16, os.cpu_count() or 1))
SIGN = -(1 << 63)


@pytest.fixture(scope="module")
def vx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_14007_amd as m
    m.lib()
    return m


@pytest.fixture(autouse=True)
def _release_device_memory():
    """Each test here holds up to ~250 GB; hand the cached blocks back
    between tests so the next one finds the whole HBM free."""
    yield
    import gc
    gc.collect()
    if torch.cuda.is_available():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("k", [27, 29])  # two passes (8-8), three passes (4-7-7)
def test_full_bit_exact(vx, k):
    print(f"k={k}: GPU plot", flush=True)
    b = vx.plot(KEY0, k)
    torch.cuda.synchronize()
    assert vx.device_status(b.workspace) == 0
    print(f"k={k}: oracle with {THREADS} threads", flush=True)
    ref = oracle.plot(KEY0, k, threads=THREADS)
    assert np.array_equal(vx.u64(b.t1_keys), ref.t1_keys)
    assert np.array_equal(vx.u32(b.t1_nonces), ref.t1_nonces)
    assert np.array_equal(vx.u32(b.bucket_offsets), ref.offsets)
    cnt = vx.t2_count(b)
    assert cnt == len(ref.t2)
    assert np.array_equal(vx.t2_records(b.t2, cnt), ref.t2)


def _signed_order(keys_i64):
    """int64 view of u64 keys whose signed order is the unsigned order."""
    return keys_i64 ^ SIGN


@pytest.mark.timeout(900)
def test_k31_sampled_and_whole_table_properties(vx):
    k = 31
    n = 1 << k
    T = vx.vx_default_threshold(k)
    print("k=31: GPU plot", flush=True)
    b = vx.plot(KEY0, k)
    torch.cuda.synchronize()
    assert vx.device_status(b.workspace) == 0
    cnt = vx.t2_count(b)
    assert 0 < cnt <= b.t2_capacity
    keys = b.t1_keys
    non = b.t1_nonces
    sk = _signed_order(keys)
    step = 1 << 28

    print("k=31: Table-1 order and permutation", flush=True)
    for lo in range(0, n - 1, step):
        hi = min(lo + step + 1, n)
        a, c = sk[lo:hi - 1], sk[lo + 1:hi]
        na, nc = non[lo:hi - 1], non[lo + 1:hi]
        assert bool(torch.all((a < c) | ((a == c) & (na < nc))))
    seen = torch.zeros(n, dtype=torch.bool, device=keys.device)
    for lo in range(0, n, step):
        seen[non[lo:lo + step].long()] = True
    assert bool(seen.all())
    del seen

    print("k=31: bucket offsets", flush=True)
    counts = torch.zeros(1 << 24, dtype=torch.int64, device=keys.device)
    for lo in range(0, n, step):
        counts += torch.bincount((keys[lo:lo + step] >> 40) & 0xFFFFFF, minlength=1 << 24)
    off = b.bucket_offsets.long() & 0xFFFFFFFF
    assert int(off[0]) == 0 and int(off[-1]) == n
    assert torch.equal(off[1:] - off[:-1], counts)
    bucket_end = off[1:]

    print("k=31: independent |Table 2| count", flush=True)
    total = 0
    for lo in range(0, n, step):
        hi = min(lo + step, n)
        kk = sk[lo:hi]
        bk = (keys[lo:hi] >> 40) & 0xFFFFFF
        end = bucket_end[bk]
        # first index whose key is >= key + T (unsigned), capped by the bucket end;
        # key + T stays inside the bucket's key range or beyond its end.
        over = kk > (((1 << 63) - 1) - T)  # key + T past the top of the key space
        lim = torch.searchsorted(sk, torch.where(over, kk, kk + T), side="left")
        lim = torch.where(over, torch.full_like(lim, n), lim)
        lim = torch.minimum(lim, end)
        idx = torch.arange(lo, hi, device=keys.device)
        total += int((lim - idx - 1).clamp_min(0).sum())
    assert total == cnt

    print("k=31: Table-2 validity and canonical order", flush=True)
    rank = torch.empty(n, dtype=torch.int32, device=keys.device)
    for lo in range(0, n, step):
        rank[non[lo:lo + step].long()] = torch.arange(lo, min(lo + step, n), dtype=torch.int32,
                                                      device=keys.device)
    t2 = b.t2[:cnt]
    prev = None
    for lo in range(0, cnt, step):
        rec = t2[lo:lo + step]
        na = (rec[:, 0] & 0xFFFFFFFF).long()
        nb = ((rec[:, 0] >> 32) & 0xFFFFFFFF).long()
        ra, rb = rank[na].long(), rank[nb].long()
        ka, kb = keys[ra], keys[rb]
        assert bool(torch.all(ra < rb))
        assert bool(torch.all(((ka >> 40) & 0xFFFFFF) == ((kb >> 40) & 0xFFFFFF)))
        d = kb - ka  # same bucket and ordered: 0 <= d < 2^40, no wrap in int64
        assert bool(torch.all((d >= 0) & (d < T)))
        comp = ra * (1 << 32) + rb
        assert bool(torch.all(comp[1:] > comp[:-1]))
        if prev is not None:
            assert int(comp[0]) > prev
        prev = int(comp[-1])

    print("k=31: sampled records against the oracle hashes", flush=True)
    rng = random.Random(31)
    pos = sorted(rng.randrange(n) for _ in range(4096))
    pk = vx.u64(keys[torch.tensor(pos, device=keys.device)])
    pn = vx.u32(non[torch.tensor(pos, device=keys.device)])
    assert np.array_equal(pk, oracle.h1_many(KEY0, pn))
    tp = sorted(rng.randrange(cnt) for _ in range(4096))
    tr = vx.t2_records(t2[torch.tensor(tp, device=keys.device)], len(tp))
    for r in tr:
        assert int(r["hash2"]) == oracle.h2(KEY0, int(r["nonce_a"]), int(r["nonce_b"]))

    print(f"k=31: oracle sampled buckets with {THREADS} threads", flush=True)
    # 4096 SplitMix64-drawn buckets, the first and last, and the fullest one.
    largest = int(torch.argmax(counts))
    s = oracle.sample_buckets(KEY0, k, sampled_buckets(4096) + [largest], threads=THREADS)
    buckets = [int(x) for x in s.buckets]
    assert largest in buckets and len(buckets) >= 4096
    offh = vx.u32(b.bucket_offsets).astype(np.int64)
    bidx = torch.tensor(buckets, device=keys.device)
    lo_t = off[bidx]
    # Table-2 slice of bucket b: records whose first member ranks in [off[b], off[b+1]).
    # int64 throughout: the end offset of the last bucket is 2^31.
    ra_all = rank[(t2[:, 0] & 0xFFFFFFFF).long()].long()
    p_lo = torch.searchsorted(ra_all, lo_t, side="left").cpu().numpy()
    p_hi = torch.searchsorted(ra_all, off[bidx + 1], side="left").cpu().numpy()
    t1_pos = 0
    t2_pos = 0
    for i, bk in enumerate(buckets):
        a, c = int(offh[bk]), int(offh[bk + 1])
        assert c - a == int(s.bucket_counts[i])
        assert np.array_equal(vx.u64(keys[a:c]), s.t1_keys[t1_pos:t1_pos + c - a])
        assert np.array_equal(vx.u32(non[a:c]), s.t1_nonces[t1_pos:t1_pos + c - a])
        t1_pos += c - a
        pc = int(s.pair_counts[i])
        assert int(p_hi[i] - p_lo[i]) == pc
        got = vx.t2_records(t2[int(p_lo[i]):int(p_hi[i])], pc)
        assert np.array_equal(got, s.t2[t2_pos:t2_pos + pc])
        t2_pos += pc
    assert t2_pos == len(s.t2) and t2_pos > 0


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("mode", ["rehash", "staged"])
def test_k32_in_two_chunks_sampled_and_properties(vx, mode):
    """k = 32 (2^32 nonces) as two chunks of 2^23 buckets each, one set of
    buffers (about 112 GB), each chunk hashing every nonce (vx_plot_chunk)
    or both made from one stage (vx_stage_plot + vx_plot_staged_chunk, about
    170 GB).  Per chunk: every key carries the chunk's prefix,
    Table 1 is sorted by (key64, nonce), the offsets are the bucket
    histogram's prefix sums (0 before the range, m after it), |Table 2|
    equals an independent count and every record is valid and canonical;
    over both chunks every nonce appears exactly once.  Sampled buckets of
    both chunks are bit-exact against the oracle."""
    k, c = 32, 1
    T = vx.vx_default_threshold(k)
    dev = torch.device("cuda")
    print("k=32: oracle sampled buckets", flush=True)
    s = oracle.sample_buckets(KEY0, k, sampled_buckets(4096), threads=THREADS)
    print(f"k=32 ({mode}): allocating chunk buffers", flush=True)
    if mode == "staged":
        stage = vx.stage_plot(KEY0, k, c)
        b = vx.alloc_staged_chunk(k, c)
    else:
        b = vx.alloc_chunk(k, c)
    seen = torch.zeros(1 << k, dtype=torch.bool, device=dev)
    # nonce -> position in its chunk, stored as int32 offset by -2^31 (a chunk
    # holds fewer than 2^32 records; the shift keeps the order)
    rank = torch.empty(1 << k, dtype=torch.int32, device=dev)
    OFS = 1 << 31
    step = 1 << 28
    total_m = 0
    t1_pos = t2_pos = 0
    for r in range(1 << c):
        print(f"k=32: chunk {r}: GPU", flush=True)
        if mode == "staged":
            vx.plot_staged_chunk(KEY0, stage, r, b)
        else:
            vx.plot_chunk(KEY0, k, c, r, b)
        torch.cuda.synchronize()
        assert vx.device_status(b.workspace) == 0
        m = int(b.t1_count.item())
        total_m += m
        cnt = vx.t2_count(b)
        assert 0 < cnt <= b.t2_capacity
        keys, non = b.t1_keys[:m], b.t1_nonces[:m]
        sk = _signed_order(keys)

        print(f"k=32: chunk {r}: order, prefix, nonces", flush=True)
        for lo in range(0, m - 1, step):
            hi = min(lo + step + 1, m)
            a, cc = sk[lo:hi - 1], sk[lo + 1:hi]
            na, nc = non[lo:hi - 1], non[lo + 1:hi]
            na = na.long() & 0xFFFFFFFF
            nc = nc.long() & 0xFFFFFFFF
            assert bool(torch.all((a < cc) | ((a == cc) & (na < nc))))
        for lo in range(0, m, step):
            kk = keys[lo:lo + step]
            assert bool(torch.all(((kk >> 63) & 1) == r))
            ni = non[lo:lo + step].long() & 0xFFFFFFFF
            assert not bool(seen[ni].any())
            seen[ni] = True
            rank[ni] = (torch.arange(lo, min(lo + step, m), dtype=torch.int64, device=dev) - OFS).int()

        print(f"k=32: chunk {r}: bucket offsets", flush=True)
        counts = torch.zeros(1 << 24, dtype=torch.int64, device=dev)
        for lo in range(0, m, step):
            counts += torch.bincount((keys[lo:lo + step] >> 40) & 0xFFFFFF, minlength=1 << 24)
        off = b.bucket_offsets.long() & 0xFFFFFFFF
        b0, b1 = r << 23, (r + 1) << 23
        assert bool(torch.all(off[:b0 + 1] == 0)) and bool(torch.all(off[b1:] == m))
        assert torch.equal(off[1:] - off[:-1], counts)
        bucket_end = off[1:]

        print(f"k=32: chunk {r}: independent |Table 2| count", flush=True)
        total = 0
        for lo in range(0, m, step):
            hi = min(lo + step, m)
            kk = sk[lo:hi]
            bk = (keys[lo:hi] >> 40) & 0xFFFFFF
            over = kk > (((1 << 63) - 1) - T)
            lim = torch.searchsorted(sk, torch.where(over, kk, kk + T), side="left")
            lim = torch.where(over, torch.full_like(lim, m), lim)
            lim = torch.minimum(lim, bucket_end[bk])
            idx = torch.arange(lo, hi, device=dev)
            total += int((lim - idx - 1).clamp_min(0).sum())
        assert total == cnt

        print(f"k=32: chunk {r}: Table-2 validity and canonical order", flush=True)
        t2 = b.t2[:cnt]
        prev = None
        ra_all = torch.empty(cnt, dtype=torch.int32, device=dev)  # ra - 2^31 of every record
        for lo in range(0, cnt, step):
            rec = t2[lo:lo + step]
            na = (rec[:, 0] & 0xFFFFFFFF).long()
            nb = ((rec[:, 0] >> 32) & 0xFFFFFFFF).long()
            ra, rb = rank[na].long() + OFS, rank[nb].long() + OFS
            assert bool(seen[na].all()) and bool(seen[nb].all())
            assert bool(torch.all((ra < m) & (rb < m)))
            ka, kb = keys[ra], keys[rb]
            assert bool(torch.all(ra < rb))
            assert bool(torch.all(((ka >> 40) & 0xFFFFFF) == ((kb >> 40) & 0xFFFFFF)))
            d = _signed_order(kb) - _signed_order(ka)  # same bucket, ordered: 0 <= d < 2^40
            assert bool(torch.all((d >= 0) & (d < T)))
            comp = ra * m + rb  # rb < m; ra * 2^32 would overflow past 2^31 records
            assert bool(torch.all(comp[1:] > comp[:-1]))
            if prev is not None:
                assert int(comp[0]) > prev
            prev = int(comp[-1])
            ra_all[lo:lo + step] = (ra - OFS).int()
            del rec, na, nb, ra, rb, ka, kb, d, comp

        print(f"k=32: chunk {r}: sampled buckets against the oracle", flush=True)
        mine = [(i, bk) for i, bk in enumerate(s.buckets) if b0 <= bk < b1]
        assert mine
        offh = vx.u32(b.bucket_offsets).astype(np.int64)
        for i, bk in mine:
            a, e = int(offh[bk]), int(offh[bk + 1])
            nbk = int(s.bucket_counts[i])
            assert e - a == nbk
            assert np.array_equal(vx.u64(keys[a:e]), s.t1_keys[t1_pos:t1_pos + nbk])
            assert np.array_equal(vx.u32(non[a:e]), s.t1_nonces[t1_pos:t1_pos + nbk])
            t1_pos += nbk
            pc = int(s.pair_counts[i])
            p_lo = int(torch.searchsorted(ra_all, torch.tensor([a - OFS], dtype=torch.int32, device=dev),
                                          side="left"))
            p_hi = int(torch.searchsorted(ra_all, torch.tensor([e - OFS], dtype=torch.int32, device=dev),
                                          side="left"))
            assert p_hi - p_lo == pc
            got = vx.t2_records(t2[p_lo:p_hi], pc)
            assert np.array_equal(got, s.t2[t2_pos:t2_pos + pc])
            t2_pos += pc
        del ra_all
    assert total_m == 1 << k
    assert bool(seen.all())
    if mode == "staged":
        assert vx.device_status(stage.data) == 0
    assert t1_pos == len(s.t1_keys) and t2_pos == len(s.t2) and t2_pos > 0

"""VaultX plot oracle -- TEST INFRASTRUCTURE ONLY.

Python access to the plain C oracle (oracle/vx_oracle.c) plus the
independent pure-Python BLAKE3 (oracle/blake3_py.py).  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this package;
the HIP product path never does and shares no code with it.

Every function here follows the C oracle's definitions (BLAKE3
specification; paper sec. II-B, III-A, III-B for the plot stages).  The
wrappers only marshal numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Sequence

import numpy as np

from . import build as _build

T2_DTYPE = np.dtype([("nonce_a", "<u4"), ("nonce_b", "<u4"), ("hash2", "<u8")])
NBUCKETS = 1 << 24

_lib = None


def lib():
    """Load the oracle library, building it with gcc if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        u8p, u32p, u64p = C.POINTER(C.c_uint8), C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)
        L.or_b3_round.argtypes = [u32p, u32p]
        L.or_b3_iv.argtypes = [u32p]
        L.or_b3_compress.argtypes = [u32p, u8p, C.c_uint64, C.c_uint32, C.c_uint32, u32p]
        L.or_b3_hash.argtypes = [C.c_void_p, C.c_char_p, C.c_size_t, u8p, C.c_size_t]
        L.or_b3_derive_key.argtypes = [C.c_char_p, C.c_size_t, C.c_char_p, C.c_size_t, u8p,
                                       C.c_size_t]
        L.or_h1.argtypes = [C.c_char_p, C.c_uint32]
        L.or_h1.restype = C.c_uint64
        L.or_h2.argtypes = [C.c_char_p, C.c_uint32, C.c_uint32]
        L.or_h2.restype = C.c_uint64
        L.or_default_threshold.argtypes = [C.c_uint32]
        L.or_default_threshold.restype = C.c_uint64
        L.or_hash_table1.argtypes = [C.c_char_p, C.c_uint32, u64p]
        L.or_hash_table1_mt.argtypes = [C.c_char_p, C.c_uint32, u64p, C.c_int]
        L.or_bucket_sort.argtypes = [C.c_uint32, u64p, u64p, u32p, u32p]
        L.or_bucket_sort_mt.argtypes = [C.c_uint32, u64p, u64p, u32p, u32p, C.c_int]
        L.or_match_table2.argtypes = [C.c_char_p, C.c_uint64, u64p, u32p, u32p, C.c_void_p,
                                      C.c_uint64]
        L.or_match_table2.restype = C.c_uint64
        L.or_match_table2_mt.argtypes = [C.c_char_p, C.c_uint64, u64p, u32p, u32p, C.c_void_p,
                                         C.c_uint64, C.c_int]
        L.or_match_table2_mt.restype = C.c_uint64
        L.or_plot_timed.argtypes = [C.c_char_p, C.c_uint32, C.c_uint64, u64p, u64p, u32p, u32p,
                                    C.c_void_p, C.c_uint64, C.c_int, C.POINTER(C.c_double)]
        L.or_plot_timed.restype = C.c_uint64
        L.or_sample_buckets.argtypes = [C.c_char_p, C.c_uint32, C.c_uint64, u32p, C.c_uint32,
                                        C.c_int, u64p, u32p, C.c_uint64, u32p, u64p,
                                        C.c_void_p, C.c_uint64, u64p, u64p]
        L.or_sample_buckets.restype = C.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _key(key: bytes) -> bytes:
    if len(key) != 32:
        raise ValueError("plot key must be 32 bytes")
    return bytes(key)


# ---- BLAKE3 -------------------------------------------------------------

def b3_hash(msg: bytes, key: bytes | None = None, out_len: int = 32) -> bytes:
    out = (C.c_uint8 * out_len)()
    kp = None if key is None else C.c_char_p(_key(key))
    lib().or_b3_hash(kp, msg, len(msg), out, out_len)
    return bytes(out)


def b3_derive_key(context: str, material: bytes, out_len: int = 32) -> bytes:
    out = (C.c_uint8 * out_len)()
    c = context.encode()
    lib().or_b3_derive_key(c, len(c), material, len(material), out, out_len)
    return bytes(out)


def b3_iv() -> np.ndarray:
    iv = np.zeros(8, np.uint32)
    lib().or_b3_iv(_p(iv, C.c_uint32))
    return iv


def b3_round(v: np.ndarray, m: np.ndarray) -> np.ndarray:
    """One round (columns then diagonals) of the oracle's G on a copy of v."""
    v = np.ascontiguousarray(v, dtype=np.uint32).copy()
    m = np.ascontiguousarray(m, dtype=np.uint32)
    lib().or_b3_round(_p(v, C.c_uint32), _p(m, C.c_uint32))
    return v


def b3_compress(cv, block: bytes, counter: int, block_len: int, flags: int) -> np.ndarray:
    cv = np.ascontiguousarray(cv, dtype=np.uint32)
    blk = np.frombuffer(block.ljust(64, b"\x00"), np.uint8).copy()
    out = np.zeros(16, np.uint32)
    lib().or_b3_compress(_p(cv, C.c_uint32), _p(blk, C.c_uint8), counter, block_len, flags,
                         _p(out, C.c_uint32))
    return out


# ---- plot stages --------------------------------------------------------

def default_threshold(k: int) -> int:
    return int(lib().or_default_threshold(k))


def h1(key: bytes, nonce: int) -> int:
    return int(lib().or_h1(_key(key), nonce))


def h2(key: bytes, nonce_a: int, nonce_b: int) -> int:
    return int(lib().or_h2(_key(key), nonce_a, nonce_b))


def h1_many(key: bytes, nonces: Sequence[int]) -> np.ndarray:
    key = _key(key)
    f = lib().or_h1
    return np.array([f(key, int(n)) for n in nonces], dtype=np.uint64)


def hash_table1(key: bytes, k: int, threads: int = 1) -> np.ndarray:
    keys = np.empty(1 << k, np.uint64)
    if threads <= 1:
        lib().or_hash_table1(_key(key), k, _p(keys, C.c_uint64))
    else:
        lib().or_hash_table1_mt(_key(key), k, _p(keys, C.c_uint64), threads)
    return keys


def bucket_sort(k: int, keys_nonce_order: np.ndarray, threads: int = 1):
    n = 1 << k
    src = np.ascontiguousarray(keys_nonce_order, dtype=np.uint64)
    if src.shape != (n,):
        raise ValueError("keys_nonce_order must have 2^k entries")
    t1k = np.empty(n, np.uint64)
    t1n = np.empty(n, np.uint32)
    off = np.empty(NBUCKETS + 1, np.uint32)
    if threads <= 1:
        lib().or_bucket_sort(k, _p(src, C.c_uint64), _p(t1k, C.c_uint64), _p(t1n, C.c_uint32),
                             _p(off, C.c_uint32))
    else:
        lib().or_bucket_sort_mt(k, _p(src, C.c_uint64), _p(t1k, C.c_uint64),
                                _p(t1n, C.c_uint32), _p(off, C.c_uint32), threads)
    return t1k, t1n, off


def match_table2(key: bytes, threshold: int, t1_keys, t1_nonces, offsets, threads: int = 1,
                 capacity: int | None = None):
    """Returns (records, total_count); records holds min(total, capacity)."""
    t1k = np.ascontiguousarray(t1_keys, dtype=np.uint64)
    t1n = np.ascontiguousarray(t1_nonces, dtype=np.uint32)
    off = np.ascontiguousarray(offsets, dtype=np.uint32)
    if capacity is None:
        if threads <= 1:
            total = lib().or_match_table2(_key(key), threshold, _p(t1k, C.c_uint64),
                                          _p(t1n, C.c_uint32), _p(off, C.c_uint32), None, 0)
        else:
            total = lib().or_match_table2_mt(_key(key), threshold, _p(t1k, C.c_uint64),
                                             _p(t1n, C.c_uint32), _p(off, C.c_uint32), None,
                                             0, threads)
        capacity = total
    out = np.zeros(capacity, T2_DTYPE)
    if threads <= 1:
        total = lib().or_match_table2(_key(key), threshold, _p(t1k, C.c_uint64),
                                      _p(t1n, C.c_uint32), _p(off, C.c_uint32),
                                      out.ctypes.data, capacity)
    else:
        total = lib().or_match_table2_mt(_key(key), threshold, _p(t1k, C.c_uint64),
                                         _p(t1n, C.c_uint32), _p(off, C.c_uint32),
                                         out.ctypes.data, capacity, threads)
    return out[:min(total, capacity)], int(total)


@dataclass
class Plot:
    k: int
    threshold: int
    keys_nonce_order: np.ndarray
    t1_keys: np.ndarray
    t1_nonces: np.ndarray
    offsets: np.ndarray
    t2: np.ndarray


def plot(key: bytes, k: int, threshold: int | None = None, threads: int = 1) -> Plot:
    T = default_threshold(k) if threshold is None else int(threshold)
    keys = hash_table1(key, k, threads)
    t1k, t1n, off = bucket_sort(k, keys, threads)
    t2, total = match_table2(key, T, t1k, t1n, off, threads)
    assert len(t2) == total
    return Plot(k, T, keys, t1k, t1n, off, t2)


def plot_timed(key: bytes, k: int, threads: int = 1, threshold: int | None = None,
               t2_capacity: int | None = None):
    """Per-stage wall seconds (hash, bucket+sort, match+H2), |T2| and the
    number of Table-2 records written (each of them hashed: H2 is only
    computed for records that have room, so a timing is complete only when
    the two counts agree).  The default capacity, 2^k + 2^16, holds |T2| of
    the default threshold at every k (about 2^k (1 - 2^(23 - k)) pairs for
    k > 24, 2^(2k - 25) below)."""
    n = 1 << k
    T = default_threshold(k) if threshold is None else int(threshold)
    cap = n + (1 << 16) if t2_capacity is None else int(t2_capacity)
    keys = np.empty(n, np.uint64)
    t1k = np.empty(n, np.uint64)
    t1n = np.empty(n, np.uint32)
    off = np.empty(NBUCKETS + 1, np.uint32)
    t2 = np.empty(cap, T2_DTYPE)
    secs = (C.c_double * 3)()
    total = lib().or_plot_timed(_key(key), k, T, _p(keys, C.c_uint64), _p(t1k, C.c_uint64),
                                _p(t1n, C.c_uint32), _p(off, C.c_uint32), t2.ctypes.data_as(C.c_void_p),
                                cap, threads, secs)
    return [secs[0], secs[1], secs[2]], int(total), min(int(total), cap)


@dataclass
class BucketSample:
    buckets: np.ndarray        # sorted bucket ids
    bucket_counts: np.ndarray  # records per listed bucket
    t1_keys: np.ndarray        # Table-1 slice of the listed buckets, in order
    t1_nonces: np.ndarray
    pair_counts: np.ndarray    # Table-2 records per listed bucket
    t2: np.ndarray             # Table-2 slice of the listed buckets, in order


def sample_buckets(key: bytes, k: int, buckets: Sequence[int], threshold: int | None = None,
                   threads: int = 1) -> BucketSample:
    T = default_threshold(k) if threshold is None else int(threshold)
    b = np.array(sorted(set(int(x) for x in buckets)), dtype=np.uint32)
    nb = len(b)
    expect = max(1024, int(((1 << k) * nb / NBUCKETS) * 2 + 4096))
    while True:
        t1k = np.empty(expect, np.uint64)
        t1n = np.empty(expect, np.uint32)
        t2 = np.zeros(expect * 4, T2_DTYPE)
        cnt = np.zeros(nb, np.uint32)
        pc = np.zeros(nb, np.uint64)
        t1_len = C.c_uint64(0)
        t2_len = C.c_uint64(0)
        st = lib().or_sample_buckets(_key(key), k, T, _p(b, C.c_uint32), nb, threads,
                                     _p(t1k, C.c_uint64), _p(t1n, C.c_uint32), expect,
                                     _p(cnt, C.c_uint32), C.byref(t1_len), t2.ctypes.data,
                                     len(t2), _p(pc, C.c_uint64), C.byref(t2_len))
        if st == 0:
            return BucketSample(b, cnt, t1k[:t1_len.value], t1n[:t1_len.value], pc,
                                t2[:t2_len.value])
        expect = max(int(t1_len.value), int(t2_len.value)) + 1024

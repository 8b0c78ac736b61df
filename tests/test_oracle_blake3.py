"""Pins for the oracle's BLAKE3 (CPU only).

What fixes BLAKE3 here, with no BLAKE3 library in the environment:
  * the published digests of "" and "abc" (tests/golden/blake3_kat.txt) --
    they fix the IV, the flag values for a root chunk, the counter/length
    placement, the output rule and the permutation cycle holding word 0;
  * BLAKE2s built from the oracle's own round function and IV must equal
    hashlib.blake2s: BLAKE2s and BLAKE3 share G, its rotations and the
    column/diagonal order, so a wrong rotation, a swapped index or a wrong IV
    word in the oracle fails here;
  * an independently written pure-Python BLAKE3 with a different structure
    (incremental, lazy subtree merging, precomputed schedule) must agree on
    every length, mode and output size -- this catches transcription slips
    in either one.
"""
import hashlib
import os
import random

import numpy as np
import pytest

import oracle
from oracle import blake3_py
from conftest import golden_lines


def _kat():
    out = []
    for msg, digest in golden_lines("blake3_kat.txt"):
        out.append((b"" if msg == "-" else bytes.fromhex(msg), bytes.fromhex(digest)))
    return out


@pytest.mark.parametrize("msg,digest", _kat())
def test_known_digests_c_oracle(msg, digest):
    assert oracle.b3_hash(msg) == digest


@pytest.mark.parametrize("msg,digest", _kat())
def test_known_digests_python_blake3(msg, digest):
    assert blake3_py.blake3(msg) == digest


def _blake2s_from_oracle_round(data: bytes, key: bytes = b"", outlen: int = 32) -> bytes:
    """BLAKE2s (RFC 7693) whose rounds are the oracle's or_b3_round and whose
    IV is the oracle's IV; everything else is RFC 7693's wrapper."""
    sigma = [[int(x) for x in row] for row in golden_lines("blake2s_sigma.txt")]
    iv = oracle.b3_iv().astype(np.uint64)
    h = [int(x) for x in iv]
    h[0] ^= 0x01010000 ^ (len(key) << 8) ^ outlen
    blocks = []
    if key:
        blocks.append(key.ljust(64, b"\x00"))
    for i in range(0, len(data), 64):
        blocks.append(data[i:i + 64])
    if not blocks:
        blocks.append(b"")
    t = 0
    for bi, blk in enumerate(blocks):
        last = bi == len(blocks) - 1
        t += 64 if (key and bi == 0 and not last) else len(blk)
        if key and bi == 0 and last:
            t = 64
        m = [int.from_bytes(blk.ljust(64, b"\x00")[4 * j:4 * j + 4], "little") for j in range(16)]
        v = h + [int(x) for x in iv]
        v[12] ^= t & 0xFFFFFFFF
        v[13] ^= (t >> 32) & 0xFFFFFFFF
        if last:
            v[14] ^= 0xFFFFFFFF
        va = np.array(v, dtype=np.uint32)
        for r in range(10):
            mr = np.array([m[sigma[r][j]] for j in range(16)], dtype=np.uint32)
            va = oracle.b3_round(va, mr)
        v = [int(x) for x in va]
        h = [h[j] ^ v[j] ^ v[j + 8] for j in range(8)]
    return b"".join(x.to_bytes(4, "little") for x in h)[:outlen]


@pytest.mark.parametrize("length", [0, 1, 3, 4, 8, 55, 63, 64, 65, 127, 128, 129, 300])
def test_blake2s_structure_pins_round_function(length):
    rng = random.Random(length)
    data = bytes(rng.randrange(256) for _ in range(length))
    assert _blake2s_from_oracle_round(data) == hashlib.blake2s(data).digest()
    key = bytes(rng.randrange(256) for _ in range(32))
    assert _blake2s_from_oracle_round(data, key) == hashlib.blake2s(data, key=key).digest()


def test_blake2s_structure_detects_a_planted_rotation_slip():
    """The pin above is sensitive: a G with a wrong rotation (planted on the
    CPU, in a Python copy) no longer matches hashlib."""
    def bad_round(v, m):
        v = [int(x) for x in v]

        def rot(x, n):
            return ((x >> n) | (x << (32 - n))) & 0xFFFFFFFF

        def g(a, b, c, d, x, y):
            v[a] = (v[a] + v[b] + x) & 0xFFFFFFFF
            v[d] = rot(v[d] ^ v[a], 16)
            v[c] = (v[c] + v[d]) & 0xFFFFFFFF
            v[b] = rot(v[b] ^ v[c], 12)
            v[a] = (v[a] + v[b] + y) & 0xFFFFFFFF
            v[d] = rot(v[d] ^ v[a], 8)
            v[c] = (v[c] + v[d]) & 0xFFFFFFFF
            v[b] = rot(v[b] ^ v[c], 9)   # planted: BLAKE2s/BLAKE3 use 7
        for q, (a, b, c, d) in enumerate(((0, 4, 8, 12), (1, 5, 9, 13), (2, 6, 10, 14),
                                          (3, 7, 11, 15), (0, 5, 10, 15), (1, 6, 11, 12),
                                          (2, 7, 8, 13), (3, 4, 9, 14))):
            g(a, b, c, d, int(m[2 * q]), int(m[2 * q + 1]))
        return np.array(v, dtype=np.uint32)

    real = oracle.b3_round
    try:
        oracle.b3_round = bad_round
        assert _blake2s_from_oracle_round(b"abc") != hashlib.blake2s(b"abc").digest()
    finally:
        oracle.b3_round = real


LENGTHS = [0, 1, 4, 8, 31, 32, 63, 64, 65, 128, 1023, 1024, 1025, 2047, 2048, 2049,
           3072, 3073, 4096, 4097, 5120, 7169, 8192, 8193, 16385]


@pytest.mark.parametrize("length", LENGTHS)
def test_c_oracle_equals_python_blake3_all_modes(length):
    rng = random.Random(1000 + length)
    data = bytes(rng.randrange(256) for _ in range(length))
    key = bytes(rng.randrange(256) for _ in range(32))
    assert oracle.b3_hash(data) == blake3_py.blake3(data)
    assert oracle.b3_hash(data, key) == blake3_py.blake3(data, key)
    assert oracle.b3_hash(data, key, 131) == blake3_py.blake3(data, key, 131)
    ctx = "vaultx oracle cross-check context"
    assert oracle.b3_derive_key(ctx, data) == blake3_py.Hasher.derive_key(ctx).update(data).digest(32)


def test_extended_output_is_prefix_stable():
    data = b"extendable output"
    key = bytes(range(32))
    long = oracle.b3_hash(data, key, 300)
    for n in (1, 8, 32, 63, 64, 65, 128, 200):
        assert oracle.b3_hash(data, key, n) == long[:n]


def test_python_incremental_equals_one_shot():
    rng = random.Random(7)
    data = os.urandom(5000)
    one = blake3_py.blake3(data)
    for _ in range(10):
        h = blake3_py.Hasher()
        pos = 0
        while pos < len(data):
            step = rng.choice([1, 7, 64, 100, 1024, 1500])
            h.update(data[pos:pos + step])
            pos += step
        assert h.digest() == one


def test_keyed_mode_differs_from_hash_mode_and_from_other_keys():
    data = b"\x01\x00\x00\x00"
    k1 = bytes(32)
    k2 = bytes([1]) + bytes(31)
    assert oracle.b3_hash(data) != oracle.b3_hash(data, k1)
    assert oracle.b3_hash(data, k1) != oracle.b3_hash(data, k2)


def test_single_block_compress_matches_hash_for_short_inputs():
    """For input <= 64 bytes the hash is one compression of the zero-padded
    block with CHUNK_START|CHUNK_END|ROOT (|KEYED_HASH), counter 0."""
    key = bytes(range(1, 33))
    kw = np.frombuffer(key, "<u4")
    for n in (0, 4, 8, 64):
        msg = bytes((3 * i + 1) & 0xFF for i in range(n))
        out = oracle.b3_compress(kw, msg, 0, n, 1 | 2 | 8 | 16)
        assert out[:8].astype("<u4").tobytes() == oracle.b3_hash(msg, key)

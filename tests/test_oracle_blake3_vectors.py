"""Keyed BLAKE3 pinned to the BLAKE3 authors' published test vectors (CPU only).

tests/golden/blake3_test_vectors.txt holds the published extended outputs of
the hash and keyed_hash modes for inputs of 0..8 bytes (the pattern
0, 1, 2, ... and the key "whats the Elvish word for friend").  They fix what
no other pin here does: the KEYED_HASH flag value, the little-endian load of
the key words into the chaining value, and the second cycle of the message
permutation (the words m1, m6, m4, m7, m13, m14, m15, m8), which message word
m1 -- the second nonce of a Table-2 hash -- travels through.  Lengths 4 and 8
are exactly the one-block shapes of the plotter's Table-1 and Table-2 hashes
(paper sec. I-A, III-B: keyed Blake3 of the nonce, and of a nonce pair), so
the oracle's h1 / h2 are checked against them directly.

Each planted-mistake test changes one of those three things in a copy, on
the CPU, and shows that the published values then fail.
"""
import numpy as np
import pytest

import oracle
from oracle import blake3_py
from conftest import golden_lines

KEY = b"whats the Elvish word for friend"


def _vectors():
    out = {}
    for n, mode, hx in golden_lines("blake3_test_vectors.txt"):
        out[(int(n), mode)] = bytes.fromhex(hx)
    return out


VEC = _vectors()
LENS = sorted({n for n, _ in VEC})


def _msg(n: int) -> bytes:
    return bytes(i % 251 for i in range(n))


def test_fixture_covers_both_modes_for_lengths_0_to_8():
    assert LENS == list(range(9))
    assert all((n, m) in VEC for n in LENS for m in ("hash", "keyed_hash"))
    assert all(130 <= len(v) <= 131 for v in VEC.values())


@pytest.mark.parametrize("n", range(9))
@pytest.mark.parametrize("mode", ["hash", "keyed_hash"])
def test_c_oracle_matches_published_vectors(n, mode):
    key = KEY if mode == "keyed_hash" else None
    want = VEC[(n, mode)]
    assert oracle.b3_hash(_msg(n), key, len(want)) == want
    assert oracle.b3_hash(_msg(n), key) == want[:32]


@pytest.mark.parametrize("n", range(9))
@pytest.mark.parametrize("mode", ["hash", "keyed_hash"])
def test_python_blake3_matches_published_vectors(n, mode):
    key = KEY if mode == "keyed_hash" else None
    want = VEC[(n, mode)]
    assert blake3_py.blake3(_msg(n), key, len(want)) == want


def test_oracle_h1_is_the_published_keyed_hash_of_four_bytes():
    """H1 of nonce 0x03020100 hashes the four bytes 00 01 02 03 (LE32), and
    key64 is the first 8 output bytes read big-endian."""
    want = int.from_bytes(VEC[(4, "keyed_hash")][:8], "big")
    assert oracle.h1(KEY, 0x03020100) == want


def test_oracle_h2_is_the_published_keyed_hash_of_eight_bytes():
    """H2 of the pair (0x03020100, 0x07060504) hashes 00 01 .. 07."""
    want = int.from_bytes(VEC[(8, "keyed_hash")][:8], "big")
    assert oracle.h2(KEY, 0x03020100, 0x07060504) == want


def _single_block(words_key, msg: bytes, flags: int) -> bytes:
    out = oracle.b3_compress(words_key, msg, 0, len(msg), flags)
    return out[:8].astype("<u4").tobytes()


def test_single_block_compression_reproduces_keyed_vectors():
    kw = np.frombuffer(KEY, "<u4")
    for n in LENS:
        assert _single_block(kw, _msg(n), 1 | 2 | 8 | 16) == VEC[(n, "keyed_hash")][:32]


@pytest.mark.parametrize("wrong_flag", [0, 32, 64])
def test_planted_keyed_flag_value_fails_the_vectors(wrong_flag):
    kw = np.frombuffer(KEY, "<u4")
    for n in (0, 4, 8):
        assert _single_block(kw, _msg(n), 1 | 2 | 8 | wrong_flag) != VEC[(n, "keyed_hash")][:32]


def test_planted_big_endian_key_words_fail_the_vectors():
    kw_be = np.frombuffer(KEY, ">u4").astype(np.uint32)
    for n in (0, 4, 8):
        assert _single_block(kw_be, _msg(n), 1 | 2 | 8 | 16) != VEC[(n, "keyed_hash")][:32]


def test_planted_second_permutation_cycle_fails_the_vectors_with_m1():
    """A permutation whose second cycle is altered (entries 4 and 6 swapped:
    m1's path through the rounds changes) still reproduces inputs of at most
    4 bytes, where m1 = 0 -- and fails every published value with m1 != 0."""
    perm = list(blake3_py.MSG_PERMUTATION)
    perm[4], perm[6] = perm[6], perm[4]
    rows = [list(range(16))]
    for _ in range(6):
        rows.append([rows[-1][perm[i]] for i in range(16)])
    real = blake3_py.SCHED
    try:
        blake3_py.SCHED = rows
        for n in range(0, 5):
            assert blake3_py.blake3(_msg(n), KEY) == VEC[(n, "keyed_hash")][:32]
        for n in range(5, 9):
            assert blake3_py.blake3(_msg(n), KEY) != VEC[(n, "keyed_hash")][:32]
    finally:
        blake3_py.SCHED = real
    assert blake3_py.blake3(_msg(8), KEY) == VEC[(8, "keyed_hash")][:32]

"""Independent pure-Python BLAKE3 -- TEST INFRASTRUCTURE ONLY.

A second BLAKE3, written from the specification (O'Connor, Aumasson, Neves,
Wilcox-O'Hearn, "BLAKE3: one function, fast everywhere", 2020) with a
structure different from the C oracle's: an incremental hasher that keeps a
stack of subtree chaining values and merges them as chunks complete (spec
sec. 5.1.2, the "lazy merging" form of the tree of sec. 2.5), and a message
schedule precomputed per round instead of permuting words between rounds.
It exists to catch transcription mistakes in the C oracle; it is slow and
only used on small inputs.
"""
from __future__ import annotations

from typing import List

_M32 = 0xFFFFFFFF

# Spec sec. 2.2: IV (the SHA-256 initial value) and the message permutation.
IV = (0x6A09E667, 0xBB67AE85, 0x3C6EF372, 0xA54FF53A,
      0x510E527F, 0x9B05688C, 0x1F83D9AB, 0x5BE0CD19)
MSG_PERMUTATION = (2, 6, 3, 10, 7, 0, 4, 13, 1, 11, 12, 5, 9, 14, 15, 8)

# Spec sec. 2.3 flags.
CHUNK_START = 1
CHUNK_END = 2
PARENT = 4
ROOT = 8
KEYED_HASH = 16
DERIVE_KEY_CONTEXT = 32
DERIVE_KEY_MATERIAL = 64

BLOCK_LEN = 64
CHUNK_LEN = 1024


def _schedule() -> List[List[int]]:
    """Per-round message index: round r uses word SCHED[r][i] at slot i."""
    rows = [list(range(16))]
    for _ in range(6):
        prev = rows[-1]
        rows.append([prev[MSG_PERMUTATION[i]] for i in range(16)])
    return rows


SCHED = _schedule()

# (a, b, c, d) index quadruples: four columns then four diagonals.
_QUADS = ((0, 4, 8, 12), (1, 5, 9, 13), (2, 6, 10, 14), (3, 7, 11, 15),
          (0, 5, 10, 15), (1, 6, 11, 12), (2, 7, 8, 13), (3, 4, 9, 14))


def _rot(x: int, n: int) -> int:
    return ((x >> n) | (x << (32 - n))) & _M32


def compress(cv, block_words, counter: int, block_len: int, flags: int) -> List[int]:
    """Spec sec. 2.2; returns the 16 output words."""
    s = list(cv) + list(IV[:4]) + [counter & _M32, (counter >> 32) & _M32, block_len, flags]
    for r in range(7):
        sched = SCHED[r]
        for q, (a, b, c, d) in enumerate(_QUADS):
            x = block_words[sched[2 * q]]
            y = block_words[sched[2 * q + 1]]
            s[a] = (s[a] + s[b] + x) & _M32
            s[d] = _rot(s[d] ^ s[a], 16)
            s[c] = (s[c] + s[d]) & _M32
            s[b] = _rot(s[b] ^ s[c], 12)
            s[a] = (s[a] + s[b] + y) & _M32
            s[d] = _rot(s[d] ^ s[a], 8)
            s[c] = (s[c] + s[d]) & _M32
            s[b] = _rot(s[b] ^ s[c], 7)
    return [s[i] ^ s[i + 8] for i in range(8)] + [s[i + 8] ^ cv[i] for i in range(8)]


def _words(block: bytes) -> List[int]:
    block = block + b"\x00" * (BLOCK_LEN - len(block))
    return [int.from_bytes(block[4 * i:4 * i + 4], "little") for i in range(16)]


class _Output:
    def __init__(self, cv, words, counter, block_len, flags):
        self.cv, self.words, self.counter = list(cv), words, counter
        self.block_len, self.flags = block_len, flags

    def chaining_value(self) -> List[int]:
        return compress(self.cv, self.words, self.counter, self.block_len, self.flags)[:8]

    def root_bytes(self, n: int) -> bytes:
        out = bytearray()
        t = 0
        while len(out) < n:
            w = compress(self.cv, self.words, t, self.block_len, self.flags | ROOT)
            out += b"".join(x.to_bytes(4, "little") for x in w)
            t += 1
        return bytes(out[:n])


class _ChunkState:
    def __init__(self, key_words, chunk_counter: int, flags: int):
        self.cv = list(key_words)
        self.counter = chunk_counter
        self.flags = flags
        self.buf = b""
        self.blocks_done = 0

    def length(self) -> int:
        return BLOCK_LEN * self.blocks_done + len(self.buf)

    def _start_flag(self) -> int:
        return CHUNK_START if self.blocks_done == 0 else 0

    def update(self, data: bytes) -> None:
        while data:
            if len(self.buf) == BLOCK_LEN:
                self.cv = compress(self.cv, _words(self.buf), self.counter, BLOCK_LEN,
                                   self.flags | self._start_flag())[:8]
                self.blocks_done += 1
                self.buf = b""
            take = min(BLOCK_LEN - len(self.buf), len(data))
            self.buf += data[:take]
            data = data[take:]

    def output(self) -> _Output:
        return _Output(self.cv, _words(self.buf), self.counter, len(self.buf),
                       self.flags | self._start_flag() | CHUNK_END)


class Hasher:
    """Incremental BLAKE3 (hash, keyed_hash or derive_key material mode)."""

    def __init__(self, key: bytes | None = None, _key_words=None, _flags: int = 0):
        if _key_words is not None:
            self.key_words, self.flags = list(_key_words), _flags
        elif key is not None:
            if len(key) != 32:
                raise ValueError("key must be 32 bytes")
            self.key_words = [int.from_bytes(key[4 * i:4 * i + 4], "little") for i in range(8)]
            self.flags = KEYED_HASH
        else:
            self.key_words, self.flags = list(IV), 0
        self.chunk = _ChunkState(self.key_words, 0, self.flags)
        self.stack: List[List[int]] = []

    @classmethod
    def derive_key(cls, context: str) -> "Hasher":
        ctx = cls(_key_words=IV, _flags=DERIVE_KEY_CONTEXT)
        ctx.update(context.encode())
        ck = ctx.digest(32)
        words = [int.from_bytes(ck[4 * i:4 * i + 4], "little") for i in range(8)]
        return cls(_key_words=words, _flags=DERIVE_KEY_MATERIAL)

    def _parent_cv(self, left, right) -> List[int]:
        return _Output(self.key_words, left + right, 0, BLOCK_LEN,
                       self.flags | PARENT).chaining_value()

    def _push_chunk_cv(self, cv, total_chunks: int) -> None:
        # Merge completed subtrees: one merge per trailing zero bit of the
        # number of chunks finished so far (spec sec. 5.1.2).
        while total_chunks & 1 == 0:
            cv = self._parent_cv(self.stack.pop(), cv)
            total_chunks >>= 1
        self.stack.append(cv)

    def update(self, data: bytes) -> "Hasher":
        data = bytes(data)
        while data:
            if self.chunk.length() == CHUNK_LEN:
                cv = self.chunk.output().chaining_value()
                total = self.chunk.counter + 1
                self._push_chunk_cv(cv, total)
                self.chunk = _ChunkState(self.key_words, total, self.flags)
            take = min(CHUNK_LEN - self.chunk.length(), len(data))
            self.chunk.update(data[:take])
            data = data[take:]
        return self

    def digest(self, n: int = 32) -> bytes:
        out = self.chunk.output()
        for cv in reversed(self.stack):
            out = _Output(self.key_words, cv + out.chaining_value(), 0, BLOCK_LEN,
                          self.flags | PARENT)
        return out.root_bytes(n)


def blake3(data: bytes, key: bytes | None = None, out_len: int = 32) -> bytes:
    return Hasher(key).update(data).digest(out_len)

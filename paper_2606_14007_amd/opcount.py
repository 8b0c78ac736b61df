"""Algorithmic VALU work of one single-block keyed BLAKE3 compression.

Used to put the hashing kernels on an ALU roofline.  The count traces the
compression (BLAKE3 specification sec. 2.2) as a dataflow graph and counts
the 32-bit vector instructions a one-message-per-lane implementation cannot
avoid on CDNA hardware:

  * a + b + m is one instruction (v_add3_u32) when m is a live message word
    and one plain add when m is a literal zero;
  * each xor and each rotate is one instruction (rotate = v_alignbit_b32 or
    a byte permute);
  * values that depend only on the key and constants are uniform across the
    lanes and run on the scalar unit, so they cost no vector instructions;
  * only the digest words that form the kept 8 bytes (out0 = v0 ^ v8,
    out1 = v1 ^ v9) and their byte swaps to big-endian are live; anything
    that does not reach them is dead and not counted.

`ops_per_h1()` / `ops_per_h2()` give the algorithmic form of the same
count (every 32-bit add, xor and rotate is one op, so a + b + m with a live
message word is two), and `textbook_ops()` the plain count (7 rounds x 8 G x
14 scalar ops + 2 output xors) for comparison.
"""
from __future__ import annotations

from functools import lru_cache

_PERM = (2, 6, 3, 10, 7, 0, 4, 13, 1, 11, 12, 5, 9, 14, 15, 8)
_QUADS = ((0, 4, 8, 12), (1, 5, 9, 13), (2, 6, 10, 14), (3, 7, 11, 15),
          (0, 5, 10, 15), (1, 6, 11, 12), (2, 7, 8, 13), (3, 4, 9, 14))


class _Node:
    __slots__ = ("varying", "inputs", "live", "weight")

    def __init__(self, varying, inputs):
        self.varying = varying
        self.inputs = inputs
        self.live = False
        self.weight = 1


def _count(n_message_words: int, algorithmic: bool = False) -> int:
    """Live, lane-varying operations of one compression with message words
    m0 .. m(n-1) non-zero.  Instruction form (algorithmic=False): a + b + m
    is one v_add3_u32 and each output word costs an xor and a byte swap.
    Algorithmic form: every 32-bit add, xor and rotate is one op (a + b + m
    is two adds when m is a live message word, one when m is zero), and the
    output costs its two xors (the byte order of the kept bytes is
    representation, not work)."""
    nodes = []

    def leaf(varying):
        n = _Node(varying, ())
        return n

    def op(*ins, weight=1):
        n = _Node(any(i.varying for i in ins), ins)
        n.weight = weight
        nodes.append(n)
        return n

    zero = None  # literal zero message word
    v = [leaf(False) for _ in range(16)]          # key words, IV, counter, length, flags
    m = [leaf(True) if i < n_message_words else zero for i in range(16)]

    def add3(a, b, x):
        if x is None:
            return op(a, b)
        return op(a, b, x, weight=2 if algorithmic else 1)

    for _ in range(7):
        for q, (a, b, c, d) in enumerate(_QUADS):
            x, y = m[2 * q], m[2 * q + 1]
            v[a] = add3(v[a], v[b], x)
            v[d] = op(op(v[d], v[a]))            # xor, rotate 16
            v[c] = op(v[c], v[d])
            v[b] = op(op(v[b], v[c]))            # xor, rotate 12
            v[a] = add3(v[a], v[b], y)
            v[d] = op(op(v[d], v[a]))            # xor, rotate 8
            v[c] = op(v[c], v[d])
            v[b] = op(op(v[b], v[c]))            # xor, rotate 7
        m = [m[_PERM[i]] for i in range(16)]
    if algorithmic:
        outs = [op(v[0], v[8]), op(v[1], v[9])]                    # xor
    else:
        outs = [op(op(v[0], v[8])), op(op(v[1], v[9]))]            # xor, byte swap
    stack = list(outs)
    while stack:
        n = stack.pop()
        if n.live:
            continue
        n.live = True
        stack.extend(i for i in n.inputs if isinstance(i, _Node) and i.inputs)
    return sum(n.weight for n in nodes if n.live and n.varying)


@lru_cache(maxsize=None)
def valu_per_h1() -> int:
    """Vector instructions per Table-1 hash (4-byte message: word m0)."""
    return _count(1)


@lru_cache(maxsize=None)
def valu_per_h2() -> int:
    """Vector instructions per Table-2 hash (8-byte message: words m0, m1)."""
    return _count(2)


@lru_cache(maxsize=None)
def ops_per_h1() -> int:
    """Algorithmic 32-bit ops per Table-1 hash (add, xor, rotate = 1 op)."""
    return _count(1, algorithmic=True)


@lru_cache(maxsize=None)
def ops_per_h2() -> int:
    """Algorithmic 32-bit ops per Table-2 hash (m1 != 0 adds one add per round)."""
    return _count(2, algorithmic=True)


def textbook_ops() -> int:
    return 7 * 8 * 14 + 2


# MI355X VALU: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz (one 32-bit lane-op
# per lane per clock).
MI355X_VALU_LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9
MI355X_HBM_BYTES_PER_S = 8.0e12


if __name__ == "__main__":
    print("valu per H1 hash:", valu_per_h1())
    print("valu per H2 hash:", valu_per_h2())
    print("algorithmic ops per H1:", ops_per_h1())
    print("algorithmic ops per H2:", ops_per_h2())
    print("textbook ops:", textbook_ops())

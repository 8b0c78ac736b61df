"""Seeded input generators: SplitMix64 against its published outputs, and
the shapes of the key / batch / arrival recipes."""
import math

from conftest import golden_lines
from vx_inputs import (SplitMix64, batched_plan, derive_key, sampled_buckets,
                       serving_arrivals)


def test_splitmix64_published_outputs():
    for row in golden_lines("splitmix64.txt"):
        g = SplitMix64(int(row[0]))
        assert [g.next() for _ in range(3)] == [int(x, 16) for x in row[1:]]


def test_key_is_four_le_outputs():
    g = SplitMix64(0)
    expect = b"".join(g.next().to_bytes(8, "little") for _ in range(4))
    assert derive_key(0) == expect and len(expect) == 32
    assert derive_key(1) != derive_key(0)


def test_batched_plan_range_and_determinism():
    a = batched_plan(32)
    assert a == batched_plan(32)
    assert len(a) == 32 and all(22 <= p.k <= 29 for p in a)
    assert len({p.key for p in a}) == 32


def test_serving_arrivals_monotone_and_rate():
    arr = serving_arrivals(4000, rate_per_s=50.0)
    ts = [a.t for a in arr]
    assert all(b > a for a, b in zip(ts, ts[1:]))
    assert all(22 <= a.k <= 30 for a in arr)
    mean_gap = ts[-1] / len(ts)
    assert math.isclose(mean_gap, 1 / 50.0, rel_tol=0.08)


def test_sampled_buckets_includes_edges():
    b = sampled_buckets(100)
    assert b[0] == 0 and b[-1] == (1 << 24) - 1 and len(b) == 102
    assert b == sorted(set(b))

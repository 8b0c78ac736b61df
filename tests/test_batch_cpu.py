"""Host logic of batching (lane assignment) and the autotuner's candidate set."""
from paper_2606_14007_amd import autotune
from paper_2606_14007_amd.batch import _assign_lanes


def test_lanes_balance_largest_first():
    work = [1 << k for k in (29, 22, 28, 23, 27, 27, 24, 25)]
    lanes = _assign_lanes(work, 4)
    assert sorted(set(lanes)) == [0, 1, 2, 3]
    load = [0] * 4
    for w, l in zip(work, lanes):
        load[l] += w
    assert max(load) == 1 << 29          # the largest plot alone bounds the makespan
    assert lanes[0] != lanes[2]           # the two biggest plots run side by side


def test_lanes_single_lane():
    assert _assign_lanes([5, 3, 9], 1) == [0, 0, 0]


def test_autotune_searches_the_named_tunables():
    """The search covers the hash's slices, the first digit, the group bits
    (bucket-partition granularity), the sort group capacity and the match
    chunk; its single-axis variants map onto vx_tuning fields, and those
    the plan rejects are filtered out before any timing."""
    for k in (22, 27, 29, 31):
        names = [a for a, _ in autotune.axes(k)]
        assert names == ["hash_slices", "group_bits", "pass1_bits", "group_cap", "match_chunk_bits"]
        cands = autotune.candidates(k)
        assert cands[0] == {} and len(cands) >= 10
        for d in cands[1:]:
            (f, v), = d.items()
            assert getattr(autotune.to_native(d), f) == v
        ok = [d for d in cands if autotune.valid(k, d)]
        assert {} in ok and len(ok) >= 8
    assert not autotune.valid(22, {"pass1_bits": 12})

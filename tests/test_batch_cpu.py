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


def test_autotune_candidates_valid():
    for k in (12, 22, 27, 31):
        c = autotune.candidates(k)
        assert c and all(1 <= d["group_bits"] <= 20 for d in c)
        assert all(d["match_chunk_bits"] in (10, 11) for d in c)
        t = autotune.to_native(c[0])
        assert t.group_bits == c[0]["group_bits"]

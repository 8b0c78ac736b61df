"""Chunked plots on the CPU: capacity hints, workspace sizes and the argument
checks of vx_plot_chunk, which all return before any device work."""
import math

import pytest

import paper_2606_14007_amd as vx
from paper_2606_14007_amd import _native as N


def test_chunk_capacity_hint_bounds_the_chunk():
    # A chunk of a 2^k plot cut by c bits holds Binomial(2^k, 2^-c) records.
    for k, c in ((12, 0), (20, 2), (27, 3), (31, 1), (32, 1), (32, 8)):
        cap1, cap2 = vx.vx_chunk_capacity_hint(k, c, 1 << (64 - k))
        mean = 2.0 ** (k - c)
        assert cap1 >= mean + 8 * math.sqrt(mean), (k, c)
        assert cap1 <= mean + 8 * math.sqrt(mean) + 4097, (k, c)
        # Table 2: the whole plot's expectation over 2^c chunks, plus margin
        lam = 2.0 ** (k - 24)
        t = min(1 << (64 - k), 1 << 40) / float(1 << 40)
        expect = mean * lam * t * (1 - t / 2)
        assert cap2 >= expect * 1.04 + 4096, (k, c)


@pytest.mark.parametrize("k,c", [(0, 0), (33, 1), (32, 0), (12, 9), (3, 4)])
def test_chunk_capacity_hint_rejects(k, c):
    assert vx.vx_chunk_capacity_hint(k, c, 1) == (0, 0)


def test_chunk_workspace_sizes():
    p = vx.make_params(bytes(32), 20)
    a = vx.vx_chunk_workspace_bytes(p, 2, 1 << 18)
    b = vx.vx_chunk_workspace_bytes(p, 2, 1 << 19)
    # keys, nonces, scratch and pair counts: at least 25 bytes per record
    assert a >= 25 << 18 and b >= a + (25 << 18)
    assert vx.vx_chunk_workspace_bytes(p, 2, 0) == 0
    assert vx.vx_chunk_workspace_bytes(p, 9, 1 << 18) == 0
    assert vx.vx_chunk_workspace_bytes(p, 2, 1 << 18, vx.make_tuning(fused_sort_match=1)) == 0
    p32 = vx.make_params(bytes(32), 32)
    assert p32.match_threshold == 1 << 32
    assert vx.vx_chunk_workspace_bytes(p32, 1, (1 << 32) - 1) > 0
    assert vx.vx_chunk_workspace_bytes(p32, 1, 1 << 32) == 0
    # whole plots stay at k <= 31
    assert vx.vx_workspace_bytes(p32, vx.VX_CALL_PLOT) == 0


def _buffers(k=20, cap2=1024):
    b = N.VxPlotBuffers()
    b.t1_keys, b.t1_nonces, b.bucket_offsets = 1 << 20, 2 << 20, 3 << 20
    b.t2, b.t2_capacity, b.t2_count = 4 << 20, cap2, 5 << 20
    b.workspace, b.workspace_bytes = 6 << 20, 0
    return b


@pytest.mark.parametrize("case,status", [
    ("chunk_too_big", N.VX_ERR_INVALID_ARG),
    ("chunk_bits_9", N.VX_ERR_INVALID_ARG),
    ("k33", N.VX_ERR_INVALID_ARG),
    ("cap0", N.VX_ERR_INVALID_ARG),
    ("cap_2_32", N.VX_ERR_INVALID_ARG),
    ("fused", N.VX_ERR_UNSUPPORTED),
    ("null_keys", N.VX_ERR_INVALID_ARG),
    ("null_count", N.VX_ERR_INVALID_ARG),
    ("misaligned", N.VX_ERR_INVALID_ARG),
    ("workspace", N.VX_ERR_WORKSPACE),
])
def test_plot_chunk_argument_checks(case, status):
    # Fake aligned device addresses: every case is rejected before any
    # device call.
    p = vx.make_params(bytes(32), 20)
    b = _buffers()
    c, r, cap, cnt, tun = 2, 1, 1 << 18, 7 << 20, None
    if case == "chunk_too_big":
        r = 4
    elif case == "chunk_bits_9":
        c, r = 9, 0
    elif case == "k33":
        p.k = 33
    elif case == "cap0":
        cap = 0
    elif case == "cap_2_32":
        cap = 1 << 32
    elif case == "fused":
        tun = vx.make_tuning(fused_sort_match=1)
    elif case == "null_keys":
        b.t1_keys = None
    elif case == "null_count":
        cnt = 0
    elif case == "misaligned":
        b.t1_keys += 4
    with pytest.raises(vx.VxError) as e:
        vx.vx_plot_chunk(p, c, r, b, cap, cnt, tun)
    assert e.value.status == status
    assert vx.vx_last_error()


def test_stage_sizes_and_limits():
    p32 = vx.make_params(bytes(32), 32)
    st = vx.vx_stage_bytes(p32, 1)
    # Hashed in slices with all three passes (up to 4 chunks): the third
    # pass's regions (21 % slack over 12 bytes per record) and two slices'
    # first- and second-pass regions
    assert (12 << 32) * 1.2 < st < (12 << 32) * 1.5
    assert vx.vx_stage_bytes(p32, 2) == st          # the stage does not depend on the chunk count
    # in one launch: the first pass's regions, 12 bytes per record plus slack and the header
    one = vx.vx_stage_bytes(p32, 1, vx.make_tuning(hash_slices=1))
    assert 12 << 32 < one < (12 << 32) * 1.01
    assert vx.vx_stage_bytes(p32, 1, vx.make_tuning(front_passes=2)) == one
    assert vx.vx_stage_bytes(p32, 3) == one         # 8 chunks: one launch
    assert vx.vx_stage_bytes(p32, 7) == 0           # wider than the first digit (6 bits)
    assert vx.vx_stage_bytes(p32, 0) == 0           # one chunk of 2^32 records
    assert vx.vx_stage_bytes(p32, 1, vx.make_tuning(fused_sort_match=1)) == 0
    assert vx.vx_stage_bytes(p32, 1, vx.make_tuning(separate_hash=1)) == 0
    p12 = vx.make_params(bytes(32), 12)
    assert vx.vx_stage_bytes(p12, 1) > 0            # small plots take smaller groups
    cap = vx.vx_chunk_capacity_hint(32, 1, 1 << 32)[0]
    assert vx.vx_staged_chunk_workspace_bytes(p32, 1, cap) > 0
    assert vx.vx_staged_chunk_workspace_bytes(p32, 1, 0) == 0


@pytest.mark.parametrize("case,status", [
    ("chunk_too_big", N.VX_ERR_INVALID_ARG),
    ("null_stage", N.VX_ERR_INVALID_ARG),
    ("small_stage", N.VX_ERR_INVALID_ARG),
    ("fused", N.VX_ERR_UNSUPPORTED),
    ("workspace", N.VX_ERR_WORKSPACE),
])
def test_plot_staged_chunk_argument_checks(case, status):
    p = vx.make_params(bytes(32), 20)
    c, r, cap = 2, 1, 1 << 18
    need = vx.vx_staged_chunk_workspace_bytes(p, c, cap)
    b = _buffers()
    b.workspace_bytes = need
    stage, stage_bytes, tun = 8 << 20, vx.vx_stage_bytes(p, c), None
    if case == "chunk_too_big":
        r = 4
    elif case == "null_stage":
        stage = 0
    elif case == "small_stage":
        stage_bytes -= 1
    elif case == "fused":
        tun = vx.make_tuning(fused_sort_match=1)
    elif case == "workspace":
        b.workspace_bytes = need - 1
    with pytest.raises(vx.VxError) as e:
        vx.vx_plot_staged_chunk(p, c, r, stage, stage_bytes, b, cap, 7 << 20, tun)
    assert e.value.status == status


def test_stage_plot_argument_checks():
    p = vx.make_params(bytes(32), 20)
    with pytest.raises(vx.VxError) as e:
        vx.vx_stage_plot(p, 2, 8 << 20, vx.vx_stage_bytes(p, 2) - 1)
    assert e.value.status == N.VX_ERR_WORKSPACE
    with pytest.raises(vx.VxError) as e:
        vx.vx_stage_plot(p, 9, 8 << 20, 1 << 30)
    assert e.value.status == N.VX_ERR_INVALID_ARG

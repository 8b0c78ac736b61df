"""Plot-file format and egress argument checks on the CPU (no device)."""
import os
import struct

import numpy as np
import pytest

import paper_2606_14007_amd as vx
from paper_2606_14007_amd import egress as E


def _hand_header(k, T, cnt, nrec, key, chunk_bits=0, chunk=0):
    # The layout include/vx.h documents, written out field by field.
    h = bytearray(128)
    h[0:8] = b"VXPLOT01"
    h[8:12] = (128).to_bytes(4, "little")
    h[12:16] = (16).to_bytes(4, "little")
    h[16:20] = k.to_bytes(4, "little")
    h[20:24] = (24).to_bytes(4, "little")
    h[24:32] = T.to_bytes(8, "little")
    h[32:40] = cnt.to_bytes(8, "little")
    h[40:48] = nrec.to_bytes(8, "little")
    h[48:80] = key
    h[80:84] = chunk_bits.to_bytes(4, "little")
    h[84:88] = chunk.to_bytes(4, "little")
    return bytes(h)


def test_header_layout_matches_the_documented_offsets():
    key = bytes(range(32))
    h = E.PlotFileHeader(k=27, bucket_bits=24, threshold=1 << 37, t2_count=125_000_123, records=99, key=key)
    assert E.pack_header(h) == _hand_header(27, 1 << 37, 125_000_123, 99, key)
    assert E.parse_header(_hand_header(27, 1 << 37, 125_000_123, 99, key)) == h
    hc = E.PlotFileHeader(k=32, bucket_bits=24, threshold=1 << 32, t2_count=7, records=7, key=key,
                          chunk_bits=2, chunk=3)
    assert E.pack_header(hc) == _hand_header(32, 1 << 32, 7, 7, key, 2, 3)
    assert E.parse_header(E.pack_header(hc)) == hc


def test_read_back_concatenated_plot_files(tmp_path):
    rng = np.random.default_rng(3)
    path = tmp_path / "plots.bin"
    expect = []
    with open(path, "wb") as f:
        for k, n in ((12, 5), (13, 0), (14, 17)):
            rec = np.zeros(n, dtype=E.T2_RECORD)
            rec["nonce_a"] = rng.integers(0, 1 << k, n)
            rec["nonce_b"] = rng.integers(0, 1 << k, n)
            rec["hash2"] = rng.integers(0, 1 << 63, n, dtype=np.uint64)
            key = bytes(rng.integers(0, 256, 32, dtype=np.uint8))
            f.write(_hand_header(k, 1 << (64 - k), n + 3, n, key))
            f.write(rec.tobytes())
            expect.append((k, n, key, rec))
    got = E.read_plot_files(str(path))
    assert len(got) == 3
    for (k, n, key, rec), (h, r) in zip(expect, got):
        assert (h.k, h.records, h.t2_count, h.key, h.threshold) == (k, n, n + 3, key, 1 << (64 - k))
        assert np.array_equal(r, rec)


def test_truncated_or_foreign_files_are_rejected(tmp_path):
    p = tmp_path / "bad.bin"
    p.write_bytes(_hand_header(10, 1, 4, 4, bytes(32)) + bytes(16 * 3))
    with pytest.raises(ValueError):
        E.read_plot_files(str(p))
    p.write_bytes(b"NOTAPLOT" + bytes(120))
    with pytest.raises(ValueError):
        E.read_plot_files(str(p))


@pytest.mark.parametrize("slot_bytes,slots", [(1 << 19, 4), ((1 << 20) + 8, 4), (1 << 20, 1), (1 << 20, 65),
                                              ((1 << 30) + 16, 2)])
def test_egress_arguments_checked_before_any_allocation(slot_bytes, slots):
    with pytest.raises(vx.VxError) as ei:
        vx.vx_egress_create(-1, slot_bytes, slots)
    assert ei.value.status == 1


def test_egress_calls_reject_a_null_handle():
    p = vx.make_params(bytes(32), 10)
    with pytest.raises(vx.VxError):
        vx.vx_egress_submit(0, p, 0, 0, 0)
    with pytest.raises(vx.VxError):
        vx.vx_egress_wait(0)
    assert vx.vx_egress_bytes(0) == 0
    vx.vx_egress_destroy(0)

"""Table-2 egress on the GPU: the plot files it writes hold exactly the
oracle's Table 2, also when plots are queued back to back, when the device
table overflowed, and when the next plot already runs on the stream."""
import os

import numpy as np
import pytest
import torch

import oracle
from vx_inputs import derive_key

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_14007_amd as m
    m.lib()
    return m


def _check_file(E, path, cases):
    got = E.read_plot_files(path)
    assert len(got) == len(cases)
    for (key, k, ref, cap), (h, rec) in zip(cases, got):
        n = len(ref.t2) if cap is None else min(cap, len(ref.t2))
        assert (h.k, h.bucket_bits, h.key) == (k, 24, key)
        assert h.threshold == 1 << (64 - k)
        assert h.t2_count == len(ref.t2) and h.records == n
        assert np.array_equal(rec, ref.t2[:n])


def test_one_plot_file_equals_the_oracle(vx, tmp_path):
    from paper_2606_14007_amd import egress as E
    key, k = derive_key(7), 18
    ref = oracle.plot(key, k, threads=8)
    b = vx.plot(key, k)
    path = str(tmp_path / "p.bin")
    fd = E.open_for_append(path)
    try:
        with E.Egress(fd, slot_bytes=1 << 20, slots=3) as eg:   # several pieces per plot
            eg.submit(key, k, b)
            eg.wait()
            assert eg.bytes == 128 + 16 * len(ref.t2)
    finally:
        os.close(fd)
    _check_file(E, path, [(key, k, ref, None)])


def test_back_to_back_plots_overlap_the_next_plot(vx, tmp_path):
    """Each plot's egress is queued before the next plot is enqueued on the
    same stream (into other buffers); the files come out whole and in order."""
    from paper_2606_14007_amd import egress as E
    specs = [(derive_key(20 + i), k) for i, k in enumerate((16, 19, 17))]
    refs = [oracle.plot(key, k, threads=8) for key, k in specs]
    path = str(tmp_path / "three.bin")
    fd = E.open_for_append(path)
    try:
        with E.Egress(fd, slot_bytes=1 << 20, slots=2) as eg:
            bufs = []
            for key, k in specs:
                b = vx.plot(key, k)
                bufs.append(b)
                eg.submit(key, k, b)
            eg.wait()
    finally:
        os.close(fd)
    _check_file(E, path, [(key, k, ref, None) for (key, k), ref in zip(specs, refs)])


def test_overflowed_table_writes_the_records_it_holds(vx, tmp_path):
    from paper_2606_14007_amd import egress as E
    key, k = derive_key(9), 16
    ref = oracle.plot(key, k, threads=8)
    cap = len(ref.t2) // 3
    b = vx.alloc_plot(k, t2_capacity=cap)
    vx.plot(key, k, buffers=b)
    path = str(tmp_path / "o.bin")
    fd = E.open_for_append(path)
    try:
        with E.Egress(fd) as eg:
            eg.submit(key, k, b)
    finally:
        os.close(fd)
    _check_file(E, path, [(key, k, ref, cap)])


def test_discarding_egress_counts_the_bytes(vx):
    from paper_2606_14007_amd import egress as E
    key, k = derive_key(11), 17
    b = vx.plot(key, k)
    torch.cuda.synchronize()
    n = vx.t2_count(b)
    with E.Egress(-1, slot_bytes=4 << 20, slots=4) as eg:
        j1 = eg.submit(key, k, b)
        j2 = eg.submit(key, k, b)
        eg.wait(j1)
        eg.wait(j2)
        assert eg.bytes == 2 * (128 + 16 * n)


def test_chunk_files_concatenate_to_the_plot(vx, tmp_path):
    """The chunks of a staged plot egressed one by one (two buffer sets, each
    reused once its file is out): every file is marked with its chunk, and
    the records concatenate to the oracle's Table 2."""
    from paper_2606_14007_amd import egress as E
    key, k, c = derive_key(9), 18, 2
    ref = oracle.plot(key, k, threads=8)
    st = vx.stage_plot(key, k, c)
    sets = [vx.alloc_staged_chunk(k, c) for _ in range(2)]
    path = str(tmp_path / "chunks.bin")
    fd = E.open_for_append(path)
    try:
        with E.Egress(fd, slot_bytes=1 << 20, slots=2) as eg:
            jobs = []
            for r in range(1 << c):
                if r >= 2:
                    eg.wait(jobs[r - 2])
                b = sets[r % 2]
                vx.plot_staged_chunk(key, st, r, b)
                jobs.append(eg.submit(key, k, b, chunk_bits=c, chunk=r))
            eg.wait()
    finally:
        os.close(fd)
    got = E.read_plot_files(path)
    assert [(h.chunk_bits, h.chunk, h.k) for h, _ in got] == [(c, r, k) for r in range(1 << c)]
    assert sum(h.t2_count for h, _ in got) == len(ref.t2)
    assert np.array_equal(np.concatenate([rec for _, rec in got]), ref.t2)

"""Table-2 egress: stream finished Tables 2 off the device into flat plot
files (vx_egress_* in include/vx.h), and read such files back.

A plot file is a 128-byte little-endian header followed by the Table-2
records in canonical order (16 bytes each: nonce_a u32, nonce_b u32,
hash2 u64).  Header fields: magic "VXPLOT01", header bytes (128), record
bytes (16), k, bucket bits (24), threshold T, |Table 2| as counted on the
device, records that follow (min(|Table 2|, capacity)), the 32-byte key,
chunk_bits and chunk (0 and 0 for a whole plot; a chunk's file holds the
plot's Table 2 restricted to the chunk's buckets).
"""
from __future__ import annotations

import os
import struct
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import _native as N

HEADER_BYTES = 128
RECORD_BYTES = 16
MAGIC = b"VXPLOT01"
_HEADER = struct.Struct("<8sIIIIQQQ32sII40x")
assert _HEADER.size == HEADER_BYTES
T2_RECORD = np.dtype([("nonce_a", "<u4"), ("nonce_b", "<u4"), ("hash2", "<u8")])  # vx_t2_record


@dataclass
class PlotFileHeader:
    k: int
    bucket_bits: int
    threshold: int
    t2_count: int
    records: int
    key: bytes
    chunk_bits: int = 0
    chunk: int = 0


def pack_header(h: PlotFileHeader) -> bytes:
    return _HEADER.pack(MAGIC, HEADER_BYTES, RECORD_BYTES, h.k, h.bucket_bits, h.threshold,
                        h.t2_count, h.records, h.key, h.chunk_bits, h.chunk)


def parse_header(raw: bytes) -> PlotFileHeader:
    if len(raw) < HEADER_BYTES:
        raise ValueError("truncated plot file header")
    magic, hb, rb, k, bb, T, cnt, nrec, key, cbits, chunk = _HEADER.unpack(raw[:HEADER_BYTES])
    if magic != MAGIC or hb != HEADER_BYTES or rb != RECORD_BYTES:
        raise ValueError("not a plot file (magic or sizes differ)")
    return PlotFileHeader(k, bb, T, cnt, nrec, key, cbits, chunk)


def read_plot_files(path: str):
    """All plot files in `path` (one egress may append several): a list of
    (header, records) with records a structured numpy array (T2_RECORD)."""
    out = []
    with open(path, "rb") as f:
        data = f.read()
    off = 0
    while off < len(data):
        h = parse_header(data[off:off + HEADER_BYTES])
        off += HEADER_BYTES
        nbytes = h.records * RECORD_BYTES
        if off + nbytes > len(data):
            raise ValueError("truncated plot file records")
        out.append((h, np.frombuffer(data, dtype=T2_RECORD, count=h.records, offset=off)))
        off += nbytes
    return out


class Egress:
    """Owns a vx_egress.  `fd` is kept open by the caller (-1: discard)."""

    def __init__(self, fd: int = -1, slot_bytes: int = 64 << 20, slots: int = 4):
        self.handle = N.vx_egress_create(fd, slot_bytes, slots)

    def submit(self, key: bytes, k: int, buffers, threshold: Optional[int] = None, stream=None,
               chunk_bits: int = 0, chunk: int = 0) -> int:
        """Queue the plot file of `buffers` (a PlotBuffers whose plot, or a
        ChunkBuffers whose chunk `chunk` of 2^chunk_bits, is enqueued on
        `stream`); returns the job number."""
        from .plotter import _stream
        p = N.make_params(key, k, threshold)
        return N.vx_egress_submit_chunk(self.handle, p, chunk_bits, chunk, buffers.t2.data_ptr(),
                                        buffers.t2.shape[0], buffers.t2_count.data_ptr(), _stream(stream))

    def wait(self, job: int = 0) -> None:
        N.vx_egress_wait(self.handle, job)

    @property
    def bytes(self) -> int:
        return N.vx_egress_bytes(self.handle)

    def close(self) -> None:
        if self.handle:
            h, self.handle = self.handle, 0
            N.vx_egress_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def open_for_append(path: str) -> int:
    return os.open(path, os.O_WRONLY | os.O_CREAT | os.O_TRUNC, 0o644)

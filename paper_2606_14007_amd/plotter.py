"""Device buffers for plots (torch tensors as HIP memory) and one-call helpers
around the C ABI.  Every computation runs in libvx's kernels; this module only
allocates memory, passes pointers and copies results back for inspection."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N

T2_DTYPE = np.dtype([("nonce_a", "<u4"), ("nonce_b", "<u4"), ("hash2", "<u8")])


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev(device):
    return torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)


def _need_cuda(t: torch.Tensor, name: str, nbytes: int) -> int:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{name} holds fewer than {nbytes} bytes")
    return t.data_ptr()


@dataclass
class PlotBuffers:
    """All device memory of one plot at size k (caller-owned, reusable)."""
    k: int
    t1_keys: torch.Tensor        # int64[2^k], read as u64
    t1_nonces: torch.Tensor      # int32[2^k], read as u32
    bucket_offsets: torch.Tensor  # int32[2^24 + 1], read as u32
    t2: torch.Tensor             # int64[cap, 2] = 16-byte records
    t2_count: torch.Tensor       # int64[1], read as u64
    workspace: torch.Tensor      # uint8[workspace_bytes]

    @property
    def t2_capacity(self) -> int:
        return self.t2.shape[0]

    def native(self) -> N.VxPlotBuffers:
        b = N.VxPlotBuffers()
        b.t1_keys = self.t1_keys.data_ptr()
        b.t1_nonces = self.t1_nonces.data_ptr()
        b.bucket_offsets = self.bucket_offsets.data_ptr()
        b.t2 = self.t2.data_ptr() if self.t2_capacity else None
        b.t2_capacity = self.t2_capacity
        b.t2_count = self.t2_count.data_ptr()
        b.workspace = self.workspace.data_ptr()
        b.workspace_bytes = self.workspace.numel()
        return b

    def nbytes(self) -> int:
        return sum(t.numel() * t.element_size() for t in
                   (self.t1_keys, self.t1_nonces, self.bucket_offsets, self.t2, self.t2_count,
                    self.workspace))


def footprint_bytes(k: int, threshold: int | None = None, t2_capacity: int | None = None,
                    tuning: N.VxTuning | None = None) -> int:
    """Device bytes alloc_plot(k) takes: Table 1, offsets, Table 2, workspace."""
    p = N.make_params(bytes(32), k, threshold)
    cap = N.vx_t2_capacity_hint(k, p.match_threshold) if t2_capacity is None else t2_capacity
    n = 1 << k
    return (n * 12 + (N.VX_NUM_BUCKETS + 1) * 4 + cap * 16 + 8 +
            N.vx_workspace_bytes(p, N.VX_CALL_PLOT, tuning))


def alloc_plot(k: int, threshold: int | None = None, t2_capacity: int | None = None,
               tuning: N.VxTuning | None = None, device=None) -> PlotBuffers:
    dev = _dev(device)
    p = N.make_params(bytes(32), k, threshold)
    cap = N.vx_t2_capacity_hint(k, p.match_threshold) if t2_capacity is None else int(t2_capacity)
    ws = N.vx_workspace_bytes(p, N.VX_CALL_PLOT, tuning)
    if ws == 0:
        raise ValueError("invalid plot parameters or tuning")
    n = 1 << k
    return PlotBuffers(
        k=k,
        t1_keys=torch.empty(n, dtype=torch.int64, device=dev),
        t1_nonces=torch.empty(n, dtype=torch.int32, device=dev),
        bucket_offsets=torch.empty(N.VX_NUM_BUCKETS + 1, dtype=torch.int32, device=dev),
        t2=torch.empty((cap, 2), dtype=torch.int64, device=dev),
        t2_count=torch.zeros(1, dtype=torch.int64, device=dev),
        workspace=torch.empty(ws, dtype=torch.uint8, device=dev),
    )


class PlotOverflow(RuntimeError):
    """A plot's Table 2 held more records than its capacity, or the device
    status word reported a condition (a region overflow, a group the sort
    could not place): the tables are incomplete."""


def check_plot(buffers: PlotBuffers, stream=None, what: str = "plot") -> int:
    """Synchronises `stream` (default: the current stream) and raises
    PlotOverflow if |Table 2| exceeds the capacity or the workspace's device
    status word is non-zero; returns |Table 2|."""
    status = N.vx_read_status(buffers.workspace.data_ptr(), _stream(stream))
    cnt = t2_count(buffers)
    if cnt > buffers.t2_capacity:
        raise PlotOverflow(f"{what}: Table 2 holds {cnt} records, capacity {buffers.t2_capacity}")
    if status:
        raise PlotOverflow(f"{what}: device status {status:#x}")
    return cnt


def plot(key: bytes, k: int, threshold: int | None = None, buffers: PlotBuffers | None = None,
         tuning: N.VxTuning | None = None, stream=None, check: bool = False) -> PlotBuffers:
    """Enqueue one whole plot (vx_plot); returns the buffers holding it.
    check=True waits for it and raises PlotOverflow on a Table-2 overflow or
    a device status (check_plot)."""
    p = N.make_params(key, k, threshold)
    if buffers is None:
        buffers = alloc_plot(k, p.match_threshold, tuning=tuning)
    if buffers.k != k:
        raise ValueError("buffers were allocated for another k")
    N.vx_plot(p, buffers.native(), tuning, _stream(stream))
    if check:
        check_plot(buffers, stream)
    return buffers


@dataclass
class ChunkBuffers(PlotBuffers):
    """Device memory of one chunk of a chunked plot (vx_plot_chunk): Table 1
    holds up to t1_capacity records, t1_count receives how many it got."""
    chunk_bits: int = 0
    t1_count: torch.Tensor | None = None  # int64[1], read as u64

    @property
    def t1_capacity(self) -> int:
        return self.t1_keys.shape[0]


def alloc_chunk(k: int, chunk_bits: int, threshold: int | None = None, t1_capacity: int | None = None,
                t2_capacity: int | None = None, tuning: N.VxTuning | None = None, device=None,
                workspace: bool = True) -> ChunkBuffers:
    """Buffers for the chunks of a plot cut into 2^chunk_bits bucket ranges
    (one set serves every chunk in turn)."""
    dev = _dev(device)
    p = N.make_params(bytes(32), k, threshold)
    cap1, cap2 = N.vx_chunk_capacity_hint(k, chunk_bits, p.match_threshold)
    if cap1 == 0:
        raise ValueError("invalid k / chunk_bits (a chunk must hold fewer than 2^32 records)")
    cap1 = cap1 if t1_capacity is None else int(t1_capacity)
    cap2 = cap2 if t2_capacity is None else int(t2_capacity)
    ws = N.vx_chunk_workspace_bytes(p, chunk_bits, cap1, tuning) if workspace else 0
    if workspace and ws == 0:
        raise ValueError("invalid chunk parameters or tuning")
    return ChunkBuffers(
        k=k,
        t1_keys=torch.empty(cap1, dtype=torch.int64, device=dev),
        t1_nonces=torch.empty(cap1, dtype=torch.int32, device=dev),
        bucket_offsets=torch.empty(N.VX_NUM_BUCKETS + 1, dtype=torch.int32, device=dev),
        t2=torch.empty((cap2, 2), dtype=torch.int64, device=dev),
        t2_count=torch.zeros(1, dtype=torch.int64, device=dev),
        workspace=torch.empty(ws, dtype=torch.uint8, device=dev),
        chunk_bits=chunk_bits,
        t1_count=torch.zeros(1, dtype=torch.int64, device=dev),
    )


def plot_chunk(key: bytes, k: int, chunk_bits: int, chunk: int, buffers: ChunkBuffers,
               threshold: int | None = None, tuning: N.VxTuning | None = None, stream=None) -> ChunkBuffers:
    """Chunk `chunk` of a plot (vx_plot_chunk): Table 1 and Table 2 of the
    buckets whose top chunk_bits bits equal `chunk`.  Synchronises `stream`
    once (the record count plans the sort)."""
    if buffers.k != k or buffers.chunk_bits != chunk_bits:
        raise ValueError("buffers were allocated for another k or chunk_bits")
    p = N.make_params(key, k, threshold)
    N.vx_plot_chunk(p, chunk_bits, chunk, buffers.native(), buffers.t1_capacity, buffers.t1_count.data_ptr(),
                    tuning, _stream(stream))
    return buffers


@dataclass
class Stage:
    """A staged plot (vx_stage_plot): every record hashed once and filed by
    its first digit, from which the chunks are made."""
    k: int
    chunk_bits: int
    data: torch.Tensor  # uint8[vx_stage_bytes]


def alloc_stage(k: int, chunk_bits: int, tuning: N.VxTuning | None = None, device=None) -> Stage:
    n = N.vx_stage_bytes(N.make_params(bytes(32), k), chunk_bits, tuning)
    if n == 0:
        raise ValueError("these parameters do not allow a staged plot")
    return Stage(k, chunk_bits, torch.empty(n, dtype=torch.uint8, device=_dev(device)))


def stage_plot(key: bytes, k: int, chunk_bits: int, stage: Stage | None = None, tuning: N.VxTuning | None = None,
               stream=None) -> Stage:
    """Enqueue the one hash of a staged plot into `stage`."""
    if stage is None:
        stage = alloc_stage(k, chunk_bits, tuning)
    if stage.k != k or stage.chunk_bits != chunk_bits:
        raise ValueError("stage was allocated for another k or chunk_bits")
    N.vx_stage_plot(N.make_params(key, k), chunk_bits, stage.data.data_ptr(), stage.data.numel(), tuning,
                    _stream(stream))
    return stage


def alloc_staged_chunk(k: int, chunk_bits: int, threshold: int | None = None, t1_capacity: int | None = None,
                       t2_capacity: int | None = None, tuning: N.VxTuning | None = None,
                       device=None) -> ChunkBuffers:
    """Buffers for the chunks of a staged plot (one set serves every chunk)."""
    b = alloc_chunk(k, chunk_bits, threshold, t1_capacity, t2_capacity, device=device, workspace=False)
    p = N.make_params(bytes(32), k, threshold)
    ws = N.vx_staged_chunk_workspace_bytes(p, chunk_bits, b.t1_capacity, tuning)
    if ws == 0:
        raise ValueError("invalid staged chunk parameters or tuning")
    b.workspace = torch.empty(ws, dtype=torch.uint8, device=b.t1_keys.device)
    return b


def plot_staged_chunk(key: bytes, stage: Stage, chunk: int, buffers: ChunkBuffers, threshold: int | None = None,
                      tuning: N.VxTuning | None = None, stream=None) -> ChunkBuffers:
    """Chunk `chunk` of the staged plot (vx_plot_staged_chunk)."""
    if buffers.k != stage.k or buffers.chunk_bits != stage.chunk_bits:
        raise ValueError("buffers were allocated for another k or chunk_bits")
    p = N.make_params(key, stage.k, threshold)
    N.vx_plot_staged_chunk(p, stage.chunk_bits, chunk, stage.data.data_ptr(), stage.data.numel(), buffers.native(),
                           buffers.t1_capacity, buffers.t1_count.data_ptr(), tuning, _stream(stream))
    return buffers


def staged_chunks(key: bytes, k: int, chunk_bits: int, threshold: int | None = None,
                  tuning: N.VxTuning | None = None, stream=None):
    """Make a whole plot chunk by chunk from one stage (k up to 32): yields
    (chunk, buffers) after each chunk is enqueued; the buffers are reused by
    the next chunk, so copy out what is needed before continuing."""
    stage = stage_plot(key, k, chunk_bits, tuning=tuning, stream=stream)
    buffers = alloc_staged_chunk(k, chunk_bits, threshold=threshold, tuning=tuning)
    for r in range(1 << chunk_bits):
        plot_staged_chunk(key, stage, r, buffers, threshold=threshold, tuning=tuning, stream=stream)
        yield r, buffers


def hash_table1(key: bytes, k: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    p = N.make_params(key, k)
    n = 1 << k
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=_dev(None))
    N.vx_hash_table1(p, _need_cuda(out, "out", n * 8), _stream(stream))
    return out


def bucket_sort(key: bytes, k: int, keys: torch.Tensor, tuning: N.VxTuning | None = None,
                stream=None):
    """Returns (t1_keys, t1_nonces, offsets, workspace) device tensors."""
    p = N.make_params(key, k)
    n = 1 << k
    dev = keys.device
    t1k = torch.empty(n, dtype=torch.int64, device=dev)
    t1n = torch.empty(n, dtype=torch.int32, device=dev)
    off = torch.empty(N.VX_NUM_BUCKETS + 1, dtype=torch.int32, device=dev)
    wsb = N.vx_workspace_bytes(p, N.VX_CALL_BUCKET_SORT, tuning)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    N.vx_bucket_sort(p, _need_cuda(keys, "keys", n * 8), t1k.data_ptr(), t1n.data_ptr(),
                     off.data_ptr(), ws.data_ptr(), wsb, tuning, _stream(stream))
    return t1k, t1n, off, ws


def match_table2(key: bytes, k: int, t1_keys, t1_nonces, offsets, threshold: int | None = None,
                 t2_capacity: int | None = None, tuning: N.VxTuning | None = None, stream=None):
    """Returns (t2 int64[cap, 2], t2_count int64[1]) device tensors."""
    p = N.make_params(key, k, threshold)
    dev = t1_keys.device
    cap = N.vx_t2_capacity_hint(k, p.match_threshold) if t2_capacity is None else int(t2_capacity)
    t2 = torch.empty((max(cap, 1), 2), dtype=torch.int64, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    wsb = N.vx_workspace_bytes(p, N.VX_CALL_MATCH, tuning)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    n = 1 << k
    N.vx_match_table2(p, _need_cuda(t1_keys, "t1_keys", n * 8),
                      _need_cuda(t1_nonces, "t1_nonces", n * 4),
                      _need_cuda(offsets, "offsets", (N.VX_NUM_BUCKETS + 1) * 4),
                      t2.data_ptr(), cap, cnt.data_ptr(), ws.data_ptr(), wsb, tuning,
                      _stream(stream))
    return t2, cnt


# ---- host views (for checks and export) -----------------------------------

def u64(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def u32(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def t2_records(t2: torch.Tensor, count: int) -> np.ndarray:
    """The first `count` Table-2 records as a structured array.  Raises
    PlotOverflow if count exceeds the buffer (the device counted records it
    had no room to write)."""
    n = int(count)
    if n > t2.shape[0]:
        raise PlotOverflow(f"Table 2 holds {n} records, capacity {t2.shape[0]}")
    return t2[:n].detach().cpu().numpy().view(T2_DTYPE).reshape(-1)


def t2_count(buffers_or_tensor) -> int:
    t = buffers_or_tensor.t2_count if isinstance(buffers_or_tensor, PlotBuffers) else buffers_or_tensor
    return int(t.item())


def device_status(workspace: torch.Tensor, stream=None) -> int:
    return N.vx_read_status(workspace.data_ptr(), _stream(stream))

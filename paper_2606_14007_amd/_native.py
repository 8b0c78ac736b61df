"""ctypes view of libvx (include/vx.h): same names, argument marshalling only.

Every step of the plot runs in the HIP kernels of libvx.so.  Loading fails
loudly if the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libvx.so")

VX_OK = 0
VX_ERR_INVALID_ARG = 1
VX_ERR_WORKSPACE = 2
VX_ERR_DEVICE = 3
VX_ERR_OUT_OF_MEMORY = 4
VX_ERR_UNSUPPORTED = 5
STATUS_NAMES = {0: "VX_OK", 1: "VX_ERR_INVALID_ARG", 2: "VX_ERR_WORKSPACE", 3: "VX_ERR_DEVICE",
                4: "VX_ERR_OUT_OF_MEMORY", 5: "VX_ERR_UNSUPPORTED", 6: "VX_ERR_IO"}

VX_DEV_STATUS_GROUP_TOO_LARGE = 0x1
VX_DEV_STATUS_LOOKBACK_TIMEOUT = 0x2
VX_DEV_STATUS_REGION_OVERFLOW = 0x4
VX_BUCKET_BITS = 24
VX_NUM_BUCKETS = 1 << 24

VX_CALL_BUCKET_SORT = 1
VX_CALL_MATCH = 2
VX_CALL_PLOT = 3


class VxPlotParams(C.Structure):
    _fields_ = [("key", C.c_uint8 * 32), ("k", C.c_uint32), ("bucket_bits", C.c_uint32),
                ("match_threshold", C.c_uint64)]


class VxT2Record(C.Structure):
    _fields_ = [("nonce_a", C.c_uint32), ("nonce_b", C.c_uint32), ("hash2", C.c_uint64)]


class VxPlotBuffers(C.Structure):
    _fields_ = [("t1_keys", C.c_void_p), ("t1_nonces", C.c_void_p), ("bucket_offsets", C.c_void_p),
                ("t2", C.c_void_p), ("t2_capacity", C.c_uint64), ("t2_count", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t)]


class VxTuning(C.Structure):
    _fields_ = [("group_bits", C.c_uint32), ("pass1_bits", C.c_uint32), ("group_cap", C.c_uint32),
                ("h1_tiles", C.c_uint32), ("match_chunk_bits", C.c_uint32), ("pass2_bits", C.c_uint32),
                ("fused_sort_match", C.c_uint32), ("pipeline_slices", C.c_uint32),
                ("separate_hash", C.c_uint32), ("region_pct", C.c_uint32), ("hash_slices", C.c_uint32),
                ("tail_slices", C.c_uint32), ("batch_shared_hash", C.c_uint32),
                ("front_passes", C.c_uint32), ("front_subtile", C.c_uint32)]


class VxError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


# (name, restype, argtypes) of every symbol include/vx.h declares.
SYMBOLS = [
    ("vx_default_threshold", C.c_uint64, [C.c_uint32]),
    ("vx_workspace_bytes", C.c_size_t, [C.POINTER(VxPlotParams), C.c_int, C.POINTER(VxTuning)]),
    ("vx_t2_capacity_hint", C.c_uint64, [C.c_uint32, C.c_uint64]),
    ("vx_partition_passes", C.c_uint32, [C.POINTER(VxPlotParams), C.POINTER(VxTuning)]),
    ("vx_hash_slices", C.c_uint32, [C.POINTER(VxPlotParams), C.POINTER(VxTuning)]),
    ("vx_tail_slices", C.c_uint32, [C.POINTER(VxPlotParams), C.POINTER(VxTuning)]),
    ("vx_front_passes", C.c_uint32, [C.POINTER(VxPlotParams), C.POINTER(VxTuning)]),
    ("vx_hash_table1", C.c_int, [C.POINTER(VxPlotParams), C.c_void_p, C.c_void_p]),
    ("vx_bucket_sort", C.c_int, [C.POINTER(VxPlotParams), C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(VxTuning),
                                 C.c_void_p]),
    ("vx_match_table2", C.c_int, [C.POINTER(VxPlotParams), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.c_size_t,
                                  C.POINTER(VxTuning), C.c_void_p]),
    ("vx_plot", C.c_int, [C.POINTER(VxPlotParams), C.POINTER(VxPlotBuffers), C.POINTER(VxTuning),
                          C.c_void_p]),
    ("vx_plot_with_events", C.c_int, [C.POINTER(VxPlotParams), C.POINTER(VxPlotBuffers),
                                      C.POINTER(VxTuning), C.POINTER(C.c_void_p), C.c_void_p]),
    ("vx_plot_batch", C.c_int, [C.POINTER(VxPlotParams), C.POINTER(VxPlotBuffers), C.c_uint32,
                                C.POINTER(VxTuning), C.c_void_p]),
    ("vx_plot_noalloc", C.c_int, [C.POINTER(VxPlotParams), C.POINTER(VxPlotBuffers), C.POINTER(VxTuning),
                                  C.c_void_p, C.c_void_p]),
    ("vx_read_status", C.c_int, [C.c_void_p, C.POINTER(C.c_uint32), C.c_void_p]),
    ("vx_last_error", C.c_char_p, []),
    ("vx_chunk_capacity_hint", C.c_uint64, [C.c_uint32, C.c_uint32, C.c_uint64, C.POINTER(C.c_uint64)]),
    ("vx_chunk_workspace_bytes", C.c_size_t, [C.POINTER(VxPlotParams), C.c_uint32, C.c_uint64,
                                              C.POINTER(VxTuning)]),
    ("vx_plot_chunk", C.c_int, [C.POINTER(VxPlotParams), C.c_uint32, C.c_uint32, C.POINTER(VxPlotBuffers),
                                C.c_uint64, C.c_void_p, C.POINTER(VxTuning), C.c_void_p]),
    ("vx_stage_bytes", C.c_size_t, [C.POINTER(VxPlotParams), C.c_uint32, C.POINTER(VxTuning)]),
    ("vx_stage_plot", C.c_int, [C.POINTER(VxPlotParams), C.c_uint32, C.POINTER(VxTuning), C.c_void_p, C.c_size_t,
                                C.c_void_p]),
    ("vx_staged_chunk_workspace_bytes", C.c_size_t, [C.POINTER(VxPlotParams), C.c_uint32, C.c_uint64,
                                                     C.POINTER(VxTuning)]),
    ("vx_plot_staged_chunk", C.c_int, [C.POINTER(VxPlotParams), C.c_uint32, C.c_uint32, C.c_void_p, C.c_size_t,
                                       C.POINTER(VxPlotBuffers), C.c_uint64, C.c_void_p, C.POINTER(VxTuning),
                                       C.c_void_p]),
    ("vx_egress_create", C.c_int, [C.c_int, C.c_size_t, C.c_uint32, C.POINTER(C.c_void_p)]),
    ("vx_egress_submit", C.c_int, [C.c_void_p, C.POINTER(VxPlotParams), C.c_void_p, C.c_uint64, C.c_void_p,
                                   C.c_void_p, C.POINTER(C.c_uint64)]),
    ("vx_egress_submit_chunk", C.c_int, [C.c_void_p, C.POINTER(VxPlotParams), C.c_uint32, C.c_uint32, C.c_void_p,
                                         C.c_uint64, C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64)]),
    ("vx_egress_wait", C.c_int, [C.c_void_p, C.c_uint64]),
    ("vx_egress_bytes", C.c_uint64, [C.c_void_p]),
    ("vx_egress_destroy", C.c_int, [C.c_void_p]),
]

_lib = None


def lib() -> C.CDLL:
    """The loaded libvx.so; raises if it was never built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"libvx.so not found at {LIB_PATH}: build it with "
                "`python paper_2606_14007_amd/build.py` (there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SYMBOLS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int, where: str) -> None:
    if st != VX_OK:
        raise VxError(st, where, lib().vx_last_error().decode(errors="replace"))


def make_params(key: bytes, k: int, threshold: int | None = None) -> VxPlotParams:
    if len(key) != 32:
        raise ValueError("plot key must be 32 bytes")
    p = VxPlotParams()
    C.memmove(p.key, bytes(key), 32)
    p.k = k
    p.bucket_bits = VX_BUCKET_BITS
    p.match_threshold = vx_default_threshold(k) if threshold is None else int(threshold)
    return p


def make_tuning(group_bits=0, pass1_bits=0, group_cap=0, h1_tiles=0, match_chunk_bits=0,
                pass2_bits=0, fused_sort_match=0, pipeline_slices=0, separate_hash=0,
                region_pct=0, hash_slices=0, tail_slices=0, batch_shared_hash=0,
                front_passes=0, front_subtile=0) -> VxTuning:
    t = VxTuning()
    t.group_bits, t.pass1_bits, t.group_cap = group_bits, pass1_bits, group_cap
    t.h1_tiles, t.match_chunk_bits, t.pass2_bits = h1_tiles, match_chunk_bits, pass2_bits
    t.fused_sort_match, t.pipeline_slices = fused_sort_match, pipeline_slices
    t.separate_hash = separate_hash
    t.region_pct = region_pct
    t.hash_slices = hash_slices
    t.tail_slices = tail_slices
    t.batch_shared_hash = batch_shared_hash
    t.front_passes = front_passes
    t.front_subtile = front_subtile
    return t


def _tref(t):
    return None if t is None else C.byref(t)


# ---- same-named wrappers ------------------------------------------------

def vx_default_threshold(k: int) -> int:
    return int(lib().vx_default_threshold(k))


def vx_workspace_bytes(params: VxPlotParams, which: int, tuning: VxTuning | None = None) -> int:
    return int(lib().vx_workspace_bytes(C.byref(params), which, _tref(tuning)))


def vx_t2_capacity_hint(k: int, threshold: int) -> int:
    return int(lib().vx_t2_capacity_hint(k, threshold))


def vx_partition_passes(params: VxPlotParams, tuning: Optional[VxTuning] = None) -> int:
    return int(lib().vx_partition_passes(C.byref(params), C.byref(tuning) if tuning else None))


def vx_hash_slices(params: VxPlotParams, tuning: Optional[VxTuning] = None) -> int:
    return int(lib().vx_hash_slices(C.byref(params), C.byref(tuning) if tuning else None))


def vx_front_passes(params: VxPlotParams, tuning: Optional[VxTuning] = None) -> int:
    return int(lib().vx_front_passes(C.byref(params), C.byref(tuning) if tuning else None))


def vx_tail_slices(params: VxPlotParams, tuning: Optional[VxTuning] = None) -> int:
    return int(lib().vx_tail_slices(C.byref(params), C.byref(tuning) if tuning else None))


def vx_hash_table1(params: VxPlotParams, d_keys: int, stream: int = 0) -> None:
    _check(lib().vx_hash_table1(C.byref(params), d_keys, stream), "vx_hash_table1")


def vx_bucket_sort(params, d_keys, d_t1_keys, d_t1_nonces, d_offsets, d_ws, ws_bytes,
                   tuning=None, stream: int = 0) -> None:
    _check(lib().vx_bucket_sort(C.byref(params), d_keys, d_t1_keys, d_t1_nonces, d_offsets, d_ws,
                                ws_bytes, _tref(tuning), stream), "vx_bucket_sort")


def vx_match_table2(params, d_t1_keys, d_t1_nonces, d_offsets, d_t2, t2_capacity, d_t2_count,
                    d_ws, ws_bytes, tuning=None, stream: int = 0) -> None:
    _check(lib().vx_match_table2(C.byref(params), d_t1_keys, d_t1_nonces, d_offsets, d_t2,
                                 t2_capacity, d_t2_count, d_ws, ws_bytes, _tref(tuning), stream),
           "vx_match_table2")


def vx_plot(params: VxPlotParams, buffers: VxPlotBuffers, tuning=None, stream: int = 0) -> None:
    _check(lib().vx_plot(C.byref(params), C.byref(buffers), _tref(tuning), stream), "vx_plot")


VX_PLOT_EVENTS = 7


def vx_plot_with_events(params: VxPlotParams, buffers: VxPlotBuffers, events, tuning=None,
                        stream: int = 0) -> None:
    """events: VX_PLOT_EVENTS raw hipEvent_t handles (ints)."""
    if len(events) != VX_PLOT_EVENTS:
        raise ValueError(f"need {VX_PLOT_EVENTS} events")
    arr = (C.c_void_p * VX_PLOT_EVENTS)(*events)
    _check(lib().vx_plot_with_events(C.byref(params), C.byref(buffers), _tref(tuning), arr, stream),
           "vx_plot_with_events")


def vx_plot_batch(params_list, buffers_list, tunings=None, stream: int = 0) -> None:
    n = len(params_list)
    if len(buffers_list) != n or (tunings is not None and len(tunings) != n):
        raise ValueError("params, buffers and tunings must have the same length")
    P = (VxPlotParams * n)(*params_list)
    B = (VxPlotBuffers * n)(*buffers_list)
    T = None if tunings is None else (VxTuning * n)(*tunings)
    _check(lib().vx_plot_batch(P, B, n, T, stream), "vx_plot_batch")


VX_NOALLOC_WORKSPACE_BYTES = 128 << 20


def vx_plot_noalloc(params: VxPlotParams, buffers: VxPlotBuffers, tuning=None, d_status: int = 0,
                    stream: int = 0) -> None:
    """buffers.workspace must be 0 (the library's own array is used)."""
    _check(lib().vx_plot_noalloc(C.byref(params), C.byref(buffers), _tref(tuning), d_status or None, stream),
           "vx_plot_noalloc")


def vx_read_status(d_ws: int, stream: int = 0) -> int:
    out = C.c_uint32(0)
    _check(lib().vx_read_status(d_ws, C.byref(out), stream), "vx_read_status")
    return int(out.value)


def vx_last_error() -> str:
    return lib().vx_last_error().decode(errors="replace")


def vx_chunk_capacity_hint(k: int, chunk_bits: int, threshold: int):
    """(Table-1 capacity, Table-2 capacity) of one chunk; (0, 0) if invalid."""
    t2 = C.c_uint64(0)
    t1 = int(lib().vx_chunk_capacity_hint(k, chunk_bits, threshold, C.byref(t2)))
    return t1, int(t2.value)


def vx_chunk_workspace_bytes(params: VxPlotParams, chunk_bits: int, t1_capacity: int,
                             tuning: Optional[VxTuning] = None) -> int:
    return int(lib().vx_chunk_workspace_bytes(C.byref(params), chunk_bits, t1_capacity, _tref(tuning)))


def vx_plot_chunk(params: VxPlotParams, chunk_bits: int, chunk: int, buffers: VxPlotBuffers, t1_capacity: int,
                  d_t1_count: int, tuning: Optional[VxTuning] = None, stream: int = 0) -> None:
    _check(lib().vx_plot_chunk(C.byref(params), chunk_bits, chunk, C.byref(buffers), t1_capacity, d_t1_count,
                               _tref(tuning), stream), "vx_plot_chunk")


def vx_stage_bytes(params: VxPlotParams, chunk_bits: int, tuning: Optional[VxTuning] = None) -> int:
    return int(lib().vx_stage_bytes(C.byref(params), chunk_bits, _tref(tuning)))


def vx_stage_plot(params: VxPlotParams, chunk_bits: int, d_stage: int, stage_bytes: int,
                  tuning: Optional[VxTuning] = None, stream: int = 0) -> None:
    _check(lib().vx_stage_plot(C.byref(params), chunk_bits, _tref(tuning), d_stage, stage_bytes, stream),
           "vx_stage_plot")


def vx_staged_chunk_workspace_bytes(params: VxPlotParams, chunk_bits: int, t1_capacity: int,
                                    tuning: Optional[VxTuning] = None) -> int:
    return int(lib().vx_staged_chunk_workspace_bytes(C.byref(params), chunk_bits, t1_capacity, _tref(tuning)))


def vx_plot_staged_chunk(params: VxPlotParams, chunk_bits: int, chunk: int, d_stage: int, stage_bytes: int,
                         buffers: VxPlotBuffers, t1_capacity: int, d_t1_count: int,
                         tuning: Optional[VxTuning] = None, stream: int = 0) -> None:
    _check(lib().vx_plot_staged_chunk(C.byref(params), chunk_bits, chunk, d_stage, stage_bytes, C.byref(buffers),
                                      t1_capacity, d_t1_count, _tref(tuning), stream), "vx_plot_staged_chunk")


def vx_egress_create(fd: int, slot_bytes: int, slots: int) -> int:
    """Returns the opaque vx_egress handle (an int)."""
    h = C.c_void_p(None)
    _check(lib().vx_egress_create(fd, slot_bytes, slots, C.byref(h)), "vx_egress_create")
    return int(h.value)


def vx_egress_submit(handle: int, params: VxPlotParams, d_t2: int, t2_capacity: int, d_t2_count: int,
                     stream: int = 0) -> int:
    job = C.c_uint64(0)
    _check(lib().vx_egress_submit(handle, C.byref(params), d_t2, t2_capacity, d_t2_count, stream,
                                  C.byref(job)), "vx_egress_submit")
    return int(job.value)


def vx_egress_submit_chunk(handle: int, params: VxPlotParams, chunk_bits: int, chunk: int, d_t2: int,
                           t2_capacity: int, d_t2_count: int, stream: int = 0) -> int:
    job = C.c_uint64(0)
    _check(lib().vx_egress_submit_chunk(handle, C.byref(params), chunk_bits, chunk, d_t2, t2_capacity, d_t2_count,
                                        stream, C.byref(job)), "vx_egress_submit_chunk")
    return int(job.value)


def vx_egress_wait(handle: int, job: int = 0) -> None:
    _check(lib().vx_egress_wait(handle, job), "vx_egress_wait")


def vx_egress_bytes(handle: int) -> int:
    return int(lib().vx_egress_bytes(handle))


def vx_egress_destroy(handle: int) -> None:
    _check(lib().vx_egress_destroy(handle), "vx_egress_destroy")

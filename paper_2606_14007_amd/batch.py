"""Batched plots: many plots of mixed k as one unit of work (vx_plot_batch),
optionally captured once into a HIP graph and replayed.

Memory plan: every plot owns its outputs (Table 1, offsets, Table 2, count);
workspaces are shared per lane.  Plots are assigned to lanes largest first,
each to the least loaded lane, and every lane gets one workspace sized for
its largest plot; vx_plot_batch runs plots that share a workspace one after
another and different lanes concurrently.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

from . import _native as N
from .plotter import PlotBuffers, PlotOverflow, _dev, _stream, t2_count

LANES = 4


@dataclass
class PlotSpecLike:
    k: int
    key: bytes
    threshold: Optional[int] = None


@dataclass
class Batch:
    specs: list
    params: list
    tunings: Optional[list]
    plots: List[PlotBuffers]
    lane_of_plot: List[int]
    workspaces: List[torch.Tensor]
    graph: Optional[object] = field(default=None, repr=False)

    def footprint_bytes(self) -> int:
        outs = sum(b.nbytes() - b.workspace.numel() for b in self.plots)
        return outs + sum(w.numel() for w in self.workspaces)


def _assign_lanes(work: Sequence[int], lanes: int) -> List[int]:
    order = sorted(range(len(work)), key=lambda i: -work[i])
    load = [0] * lanes
    lane = [0] * len(work)
    for i in order:
        best = min(range(lanes), key=lambda l: load[l])
        lane[i] = best
        load[best] += work[i]
    return lane


def alloc_batch(specs, tunings=None, lanes: int = LANES, device=None) -> Batch:
    """specs: objects with .k, .key (and optionally .threshold)."""
    dev = _dev(device)
    params = [N.make_params(s.key, s.k, getattr(s, "threshold", None)) for s in specs]
    if tunings is not None and len(tunings) != len(specs):
        raise ValueError("one tuning per plot")
    lane_of = _assign_lanes([1 << s.k for s in specs], lanes)
    ws_bytes = [0] * lanes
    for i, p in enumerate(params):
        need = N.vx_workspace_bytes(p, N.VX_CALL_PLOT, tunings[i] if tunings else None)
        if need == 0:
            raise ValueError(f"invalid plot {i}")
        ws_bytes[lane_of[i]] = max(ws_bytes[lane_of[i]], need)
    workspaces = [torch.empty(max(b, 256), dtype=torch.uint8, device=dev) for b in ws_bytes]
    plots = []
    for i, (s, p) in enumerate(zip(specs, params)):
        n = 1 << s.k
        cap = N.vx_t2_capacity_hint(s.k, p.match_threshold)
        plots.append(PlotBuffers(
            k=s.k,
            t1_keys=torch.empty(n, dtype=torch.int64, device=dev),
            t1_nonces=torch.empty(n, dtype=torch.int32, device=dev),
            bucket_offsets=torch.empty(N.VX_NUM_BUCKETS + 1, dtype=torch.int32, device=dev),
            t2=torch.empty((cap, 2), dtype=torch.int64, device=dev),
            t2_count=torch.zeros(1, dtype=torch.int64, device=dev),
            workspace=workspaces[lane_of[i]],
        ))
    return Batch(list(specs), params, tunings, plots, lane_of, workspaces)


def check(batch: Batch, stream=None) -> List[int]:
    """Waits for the batch on `stream` and raises PlotOverflow if any plot's
    Table 2 outgrew its capacity or any workspace's device status word is
    non-zero (vx_plot_batch leaves in each workspace the status bits of every
    plot that used it).  Returns |Table 2| per plot."""
    sh = _stream(stream)
    bad = []
    for lane, ws in enumerate(batch.workspaces):
        st = N.vx_read_status(ws.data_ptr(), sh)
        if st:
            plots = [i for i, l in enumerate(batch.lane_of_plot) if l == lane]
            bad.append(f"device status {st:#x} in the workspace of plots {plots}")
    counts = [t2_count(b) for b in batch.plots]
    for i, (c, b) in enumerate(zip(counts, batch.plots)):
        if c > b.t2_capacity:
            bad.append(f"plot {i} (k={b.k}): Table 2 holds {c} records, capacity {b.t2_capacity}")
    if bad:
        raise PlotOverflow("batch: " + "; ".join(bad))
    return counts


def plot_batch(batch: Batch, stream=None, check_result: bool = False) -> Batch:
    """Enqueue the whole batch (vx_plot_batch) on `stream`; check_result=True
    also waits for it and raises on overflow (check)."""
    N.vx_plot_batch(batch.params, [b.native() for b in batch.plots], batch.tunings, _stream(stream))
    if check_result:
        check(batch, stream)
    return batch


def capture(batch: Batch) -> Batch:
    """Capture the batch into a HIP graph (torch.cuda.CUDAGraph); the
    library's lane streams are created by a first eager run."""
    plot_batch(batch)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plot_batch(batch, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    batch.graph = g
    return batch


def replay(batch: Batch, check_result: bool = False) -> Batch:
    if batch.graph is None:
        raise RuntimeError("batch was not captured")
    batch.graph.replay()
    if check_result:
        check(batch)
    return batch

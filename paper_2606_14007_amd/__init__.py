"""MI355X-native VaultX plotter hot path (arxiv 2606.14007, "VaultxGPU").

The computation lives in libvx.so (hand-written HIP for gfx950 behind the C
ABI in include/vx.h).  This package is its Python binding:

  * `_native`  -- ctypes declarations, same names as the C ABI;
  * `plotter`  -- torch-allocated device buffers and one-call helpers.
"""
from ._native import (VX_BUCKET_BITS, VX_CALL_BUCKET_SORT, VX_CALL_MATCH, VX_CALL_PLOT,
                      VX_DEV_STATUS_GROUP_TOO_LARGE, VX_NUM_BUCKETS, VxError, VxPlotBuffers,
                      VxPlotParams, VxT2Record, VxTuning, lib, make_params, make_tuning,
                      vx_bucket_sort, vx_default_threshold, vx_hash_table1, vx_last_error,
                      vx_match_table2, vx_plot, vx_plot_batch, vx_plot_with_events,
                      VX_PLOT_EVENTS, vx_read_status,
                      vx_partition_passes, vx_hash_slices, vx_tail_slices, vx_front_passes, vx_t2_capacity_hint, vx_workspace_bytes,
                      vx_egress_create, vx_egress_submit, vx_egress_wait, vx_egress_bytes,
                      vx_egress_destroy, vx_chunk_capacity_hint, vx_chunk_workspace_bytes,
                      vx_plot_chunk, vx_stage_bytes, vx_stage_plot, vx_staged_chunk_workspace_bytes,
                      vx_plot_staged_chunk, vx_egress_submit_chunk, vx_plot_noalloc,
                      VX_NOALLOC_WORKSPACE_BYTES)
from .plotter import (T2_DTYPE, ChunkBuffers, PlotBuffers, PlotOverflow, Stage, alloc_chunk, alloc_plot,
                      alloc_stage, check_plot,
                      alloc_staged_chunk, bucket_sort, device_status, plot_staged_chunk, stage_plot, staged_chunks,
                      footprint_bytes, hash_table1, match_table2, plot, plot_chunk, t2_count, t2_records,
                      u32, u64)

__all__ = [n for n in dir() if not n.startswith("_")]

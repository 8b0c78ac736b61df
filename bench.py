#!/usr/bin/env python3
"""Benchmark: one whole k=31 VaultX plot on one MI355X (K=31 plot seconds).

A step is one vx_plot over the seeded k=31 workload (key from SplitMix64
seed 0, 2^31 nonces, default threshold 2^33): keyed BLAKE3 of every nonce,
bucketing by the 24-bit prefix, in-bucket sort, match, Table-2 hashing.  All
buffers are allocated before the timed region.  Stage times come from HIP
events recorded by the library on the plot's stream during the timed steps.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

STAGES = ["hash", "partition1", "partition2", "group_sort", "chunk_sums", "match_emit"]
KERNEL_OF_STAGE = {"hash": "k_hash_scatter", "match_emit": "k_match_emit",
                   "group_sort": "k_groupsort", "partition1": "k_region_scan (pass 1 is in the hash)",
                   "partition2": "k_scatter claiming regions + k_region_bounds + k_colscan (later passes)",
                   "chunk_sums": "k_chunk_sums + k_scan_*"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest() -> str:
    """SHA-256 prefix of the kernel sources' code: comments, blank lines and
    trailing spaces are left out, so that editing a comment keeps the
    counters that were taken on the same code."""
    import re
    h = hashlib.sha256()
    for f in ("kernels.hip", "blake3_device.h", "block_scan.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_2606_14007_amd", "csrc", f), encoding="utf-8") as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            line = re.sub(r"//.*", "", line).rstrip()
            if line:
                h.update(line.encode() + b"\n")
    return h.hexdigest()[:16]


def load_traffic(kernel: str, k: int, launches: int = 1):
    """HBM bytes of `kernel` at size k, from the committed rocprofv3 counter
    summary: per launch, or summed over the `launches` launches of one plot
    where a stage runs the kernel several times (the record names that
    count).  None when absent, taken on other code or on another split."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for ln in open(path):
        ln = ln.strip()
        if not ln or ln.startswith("#"):
            continue
        parts = ln.split()
        if len(parts) >= 5 and parts[0] == kernel and parts[1] == f"k={k}":
            n = int(parts[5].split("=")[1]) if len(parts) >= 6 else 1
            rec = {"sha": parts[2], "fetch": float(parts[3]), "write": float(parts[4]), "n": n}
    if not rec or rec["sha"] != source_digest() or rec["n"] != launches:
        return None
    return rec["fetch"] + rec["write"]


def host_info() -> dict:
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    mem = None
    try:
        for ln in open("/proc/meminfo"):
            if ln.startswith("MemTotal:"):
                mem = round(int(ln.split()[1]) / 2**20, 1)
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)), "cpu_model": model,
            "host_mem_gib": mem}


def cpu_baseline(k_sample: int, target_k: int) -> dict:
    """The plain oracle (C, shares no code with the HIP path) on the host:
    a full k_sample plot on one pinned core, then its thread-split variant
    on every usable core.  Each stage is scaled to target_k: hashing and
    match + H2 by the growth of their work (2^(target_k - k_sample) nonces,
    the |Table 2| ratio of the default thresholds), the bucket + sort stage
    by 2^d * target_k / k_sample (n log n; the insertion sort inside a
    bucket grows faster, so this favours the CPU)."""
    import oracle
    from vx_inputs import derive_key
    key = derive_key(0)
    info = host_info()
    cpus = sorted(os.sched_getaffinity(0))
    d = target_k - k_sample

    def t2_expect(k):
        n = 2.0 ** k
        lam = n / 2.0 ** 24
        t = min(1.0, 2.0 ** (64 - k) / 2.0 ** 40)
        return n * lam * t * (1 - t / 2)

    scale = [2.0 ** d, 2.0 ** d * target_k / k_sample, t2_expect(target_k) / t2_expect(k_sample)]

    def run(threads):
        t0 = time.perf_counter()
        secs, t2n, written = oracle.plot_timed(key, k_sample, threads=threads)
        wall = time.perf_counter() - t0
        if written != t2n:
            raise RuntimeError("oracle Table-2 buffer too small: the timing would skip H2 hashes")
        est = sum(a * b for a, b in zip(secs, scale))
        log(f"cpu baseline, {threads} thread(s): stages {['%.2f' % x for x in secs]} s at k={k_sample} "
            f"(|T2|={t2n}, {wall:.1f} s wall) -> {est:.1f} s per k={target_k} plot")
        return secs, est, t2n

    log(f"cpu baseline: plain oracle, full k={k_sample} plot; host {info}")
    old = os.sched_getaffinity(0)
    os.sched_setaffinity(0, {cpus[0]})   # this thread only: the single-thread oracle runs in it
    try:
        s1, e1, t2n = run(1)
    finally:
        os.sched_setaffinity(0, old)
    sm, em, _ = run(len(cpus))
    stage_names = ["hash", "bucket+sort", "match+H2"]
    return {
        "value": round(em, 2), "unit": "s", "cores": len(cpus), "kind": "oracle",
        "sample": (f"full k={k_sample} plot of the same seeded key (2^{k_sample} H1 + {t2n} H2 hashes, "
                   f"insertion sort per bucket), thread-split oracle on {len(cpus)} host threads, each "
                   f"stage scaled to k={target_k}: hash x{scale[0]:.0f}, bucket+sort "
                   f"x{scale[1]:.1f} (n log n; favours the CPU), match+H2 x{scale[2]:.2f} (|T2|)"),
        "stages_s": {n: round(x, 3) for n, x in zip(stage_names, sm)},
        "single_thread": {"value": round(e1, 2), "unit": "s", "cores": 1,
                          "stages_s": {n: round(x, 3) for n, x in zip(stage_names, s1)}},
        "host": info,
    }


def batched_compare(reps: int, autotuned: bool = False, shared_hash: bool = False) -> dict:
    """The batched workload (32 plots, k uniform in 22..29, keys from
    SplitMix64 seed 4): the same plots one at a time through vx_plot, against
    one vx_plot_batch, eager and replayed as a HIP graph.  Every run is
    checked for overflow and device status; returns times and plots/hour."""
    import torch
    import paper_2606_14007_amd as vx
    from paper_2606_14007_amd import autotune, batch as B
    from vx_inputs import batched_plan

    specs = batched_plan(32)
    tunings = None
    if autotuned:
        cache = autotune.load_cache()
        tun = [autotune.tuned(s.k, cache) for s in specs]
        tunings = [autotune.to_native(t) if t else vx.make_tuning() for t in tun]
        log(f"autotuned plots: {sum(t is not None for t in tun)}/{len(tun)}")
    if shared_hash:
        # every plot may share hash launches with the others (device work list)
        tunings = tunings or [vx.make_tuning() for _ in specs]
        for t in tunings:
            t.batch_shared_hash = 1
    bt = B.alloc_batch(specs, tunings=tunings)
    log(f"batched: {len(specs)} plots, k={sorted(s.k for s in specs)}, "
        f"{bt.footprint_bytes() / 2**30:.1f} GiB on the device")
    sh = torch.cuda.current_stream().cuda_stream
    params = bt.params
    nbs = [b.native() for b in bt.plots]

    def sequential():
        for p, nb in zip(params, nbs):
            vx.vx_plot(p, nb, None, sh)   # plain path, default tuning, one at a time

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_seq = timed(sequential)
    for i, b in enumerate(bt.plots):
        vx.check_plot(b, what=f"sequential plot {i}")
    log(f"sequential: {t_seq * 1e3:.1f} ms for {len(specs)} plots")
    t_bat = timed(lambda: B.plot_batch(bt))
    B.check(bt)
    log(f"batched (eager): {t_bat * 1e3:.1f} ms")
    B.capture(bt)
    t_graph = timed(lambda: B.replay(bt))
    B.check(bt)
    log(f"batched (graph replay): {t_graph * 1e3:.1f} ms")
    n = len(specs)
    best = min(t_bat, t_graph)
    out = {
        "ks": [s.k for s in specs], "footprint_gib": round(bt.footprint_bytes() / 2**30, 1),
        "sequential_ms": round(t_seq * 1e3, 3), "batched_eager_ms": round(t_bat * 1e3, 3),
        "batched_graph_ms": round(t_graph * 1e3, 3), "best_ms": round(best * 1e3, 3),
        "sequential_plots_per_hour": round(n * 3600.0 / t_seq, 1),
        "batched_plots_per_hour": round(n * 3600.0 / best, 1),
        "batched_eager_plots_per_hour": round(n * 3600.0 / t_bat, 1),
        "batched_graph_plots_per_hour": round(n * 3600.0 / t_graph, 1),
        "speedup_vs_sequential": round(t_seq / best, 3),
        "records": sum(1 << s.k for s in specs), "lanes": B.LANES, "autotuned": autotuned,
        "shared_hash": shared_hash,
    }
    del bt
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def bench_batched(args) -> dict:
    """32 plots, k uniform in 22..29, independent keys (SplitMix64 seed 4):
    plots/hour of one batched launch (eager, and replayed as a HIP graph)
    against the same plots one at a time through vx_plot."""
    reps = max(1, args.steps)
    r = batched_compare(reps, bool(args.autotune), bool(args.shared_hash))
    return {
        "metric": "mixed-k plots/hour batched vs plain",
        "value": r["batched_plots_per_hour"],
        "unit": "plots/h",
        "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": r["best_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "batched: 32 plots, k uniform in 22..29, keys from SplitMix64 "
                               "seed 4, default thresholds", "ks": r["ks"],
                   "lanes": r["lanes"], "autotuned": r["autotuned"], "parallelism": "single GPU"},
        **{k: v for k, v in r.items() if k not in ("ks", "lanes", "autotuned")},
    }


def bench_egress(args) -> dict:
    """Plots of one k (default 28) whose Tables 2 leave the device through
    vx_egress as flat plot files: compute alone, compute then egress one
    plot at a time, and egress of plot i overlapped with the computation of
    plot i + 1 (two buffer sets).  The sink is discarded by default (the
    copy path alone: device -> pinned host memory -> writer thread); with
    --egress-dir the files are written there."""
    import torch
    import paper_2606_14007_amd as vx
    from paper_2606_14007_amd import egress as E
    from vx_inputs import derive_key

    k = args.egress_k
    nplots = max(2, args.steps)
    keys = [derive_key(100 + i) for i in range(nplots)]
    sets = [vx.alloc_plot(k) for _ in range(2)]
    fd = -1
    path = None
    if args.egress_dir:
        path = os.path.join(args.egress_dir, f"plots_k{k}.bin")
        fd = E.open_for_append(path)
    eg = E.Egress(fd, slot_bytes=args.egress_slot_mb << 20, slots=args.egress_slots)
    log(f"egress: {nplots} plots at k={k}, sink {'discard' if fd < 0 else path}, "
        f"{args.egress_slots} x {args.egress_slot_mb} MiB pinned staging")
    stream = torch.cuda.current_stream()

    def compute_only():
        for i in range(nplots):
            vx.plot(keys[i], k, buffers=sets[i % 2])

    def sequential():
        for i in range(nplots):
            b = sets[i % 2]
            vx.plot(keys[i], k, buffers=b)
            eg.wait(eg.submit(keys[i], k, b))

    def overlapped():
        jobs = []
        for i in range(nplots):
            b = sets[i % 2]
            if i >= 2:
                eg.wait(jobs[i - 2])     # this buffer set's previous Table 2 is out
            vx.plot(keys[i], k, buffers=b)
            jobs.append(eg.submit(keys[i], k, b))
        eg.wait()

    def timed(fn):
        torch.cuda.synchronize()
        b0 = eg.bytes
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        eg.wait()
        return time.perf_counter() - t0, eg.bytes - b0

    compute_only()
    torch.cuda.synchronize()
    t_comp, _ = timed(compute_only)
    t_seq, by_seq = timed(sequential)
    t_ovl, by_ovl = timed(overlapped)
    # copy path alone: one finished plot egressed with nothing else running
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eg.wait(eg.submit(keys[0], k, sets[0]))
    t_one = time.perf_counter() - t0
    one_bytes = 128 + 16 * vx.t2_count(sets[0])
    eg.close()
    if fd >= 0:
        os.close(fd)
    for b in sets:
        if vx.t2_count(b) > b.t2_capacity:
            raise RuntimeError("Table 2 overflow")
    log(f"compute only {t_comp * 1e3 / nplots:.1f} ms/plot; sequential egress "
        f"{t_seq * 1e3 / nplots:.1f} ms/plot; overlapped {t_ovl * 1e3 / nplots:.1f} ms/plot; "
        f"one Table 2 ({one_bytes / 1e9:.2f} GB) alone {t_one * 1e3:.1f} ms")
    return {
        "metric": f"K={k} plots/hour with Table-2 egress",
        "value": round(nplots * 3600.0 / t_ovl, 1),
        "unit": "plots/h",
        "n_gpus": 1, "steps": nplots, "warmup": 1,
        "ms_per_step": round(t_ovl * 1e3 / nplots, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"k={k} plots, keys from SplitMix64 seeds 100.., Table 2 "
                               f"streamed to {'a discarding sink' if fd < 0 else 'plot files'}",
                   "k": k, "slots": args.egress_slots, "slot_mib": args.egress_slot_mb,
                   "parallelism": "single GPU"},
        "compute_only_plots_per_hour": round(nplots * 3600.0 / t_comp, 1),
        "sequential_egress_plots_per_hour": round(nplots * 3600.0 / t_seq, 1),
        "overlapped_egress_plots_per_hour": round(nplots * 3600.0 / t_ovl, 1),
        "egress_GBps_alone": round(one_bytes / t_one / 1e9, 2),
        "egress_GBps_overlapped": round(by_ovl / t_ovl / 1e9, 2),
        "table2_bytes_per_plot": one_bytes,
    }


def bench_serving(args) -> dict:
    """Poisson plot requests (SplitMix64 seed 5), k uniform in 22..30, at
    about 80% of the plain one-at-a-time service rate; continuous batching
    (4 slots, HBM-footprint admission, jobs of k >= --big-k one at a time
    beside the smaller ones) against the same without size classes and a
    FIFO one-at-a-time server, all on the same arrivals."""
    import torch
    from paper_2606_14007_amd import serve
    from vx_inputs import serving_arrivals

    k_lo, k_hi = 22, 30
    per_k = serve.measure_plain_times(range(k_lo, k_hi + 1), reps=2)
    torch.cuda.empty_cache()
    mean_t = serve.expected_service_time(k_lo, k_hi, per_k)
    rate = 0.8 / mean_t
    log("plain service time per k (ms): " + ", ".join(f"{k}:{t * 1e3:.2f}" for k, t in per_k.items()))
    log(f"mean service time {mean_t * 1e3:.2f} ms -> arrival rate {rate:.1f}/s (80% load)")
    arrivals = serving_arrivals(args.requests, rate)
    budget = int(args.budget_gb * 2**30)

    def run(label, slots, max_bypass, **kw):
        ex = serve.GpuExecutor(slots=slots, budget_bytes=budget)
        st = serve.Server(ex, budget, slots=slots, max_bypass=max_bypass, **kw).run(
            serve.jobs_from_arrivals(arrivals))
        del ex
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        if st.failed():
            raise RuntimeError(f"{label}: {len(st.failed())} jobs reported a device problem")
        log(f"{label}: p50 {st.percentile(50) * 1e3:.1f} ms, p99 {st.percentile(99) * 1e3:.1f} ms, "
            f"{st.plots_per_hour():.0f} plots/h, peak resident {st.max_resident / 2**30:.1f} GiB, "
            f"max concurrent {st.max_concurrent}")
        return st

    cb = run(f"continuous batching, size classes (k >= {args.big_k}: one at a time)", 4, 8,
             big_k=args.big_k, max_big=1)
    flat = run("continuous batching, one class", 4, 8)
    fifo = run("FIFO one at a time", 1, 0)
    return {
        "metric": "plot serving plots/hour (continuous batching, p50/p99 latency) vs FIFO",
        "value": round(cb.plots_per_hour(), 1),
        "unit": "plots/h",
        "n_gpus": 1, "steps": args.requests, "warmup": 0,
        "ms_per_step": round(cb.makespan * 1e3 / args.requests, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"serving: {args.requests} Poisson requests (seed 5), k uniform in "
                               f"{k_lo}..{k_hi}, rate {rate:.1f}/s = 80% of the plain service rate",
                   "slots": 4, "big_k": args.big_k, "max_big": 1, "budget_gib": args.budget_gb,
                   "parallelism": "single GPU"},
        "p50_latency_ms": round(cb.percentile(50) * 1e3, 2),
        "p99_latency_ms": round(cb.percentile(99) * 1e3, 2),
        "one_class_p50_latency_ms": round(flat.percentile(50) * 1e3, 2),
        "one_class_p99_latency_ms": round(flat.percentile(99) * 1e3, 2),
        "one_class_plots_per_hour": round(flat.plots_per_hour(), 1),
        "fifo_p50_latency_ms": round(fifo.percentile(50) * 1e3, 2),
        "fifo_p99_latency_ms": round(fifo.percentile(99) * 1e3, 2),
        "fifo_plots_per_hour": round(fifo.plots_per_hour(), 1),
        "peak_resident_gib": round(cb.max_resident / 2**30, 2),
        "max_concurrent": cb.max_concurrent,
        "plain_ms_per_k": {k: round(t * 1e3, 3) for k, t in per_k.items()},
        "p50_ms_per_k": {k: round(v["p50_ms"], 2) for k, v in cb.by_k().items()},
        "p99_ms_per_k": {k: round(v["p99_ms"], 2) for k, v in cb.by_k().items()},
        "fifo_p50_ms_per_k": {k: round(v["p50_ms"], 2) for k, v in fifo.by_k().items()},
        "fifo_p99_ms_per_k": {k: round(v["p99_ms"], 2) for k, v in fifo.by_k().items()},
    }


def bench_chunked(args) -> dict:
    """One whole plot made as 2^c chunks (default k=32, c=1: 2^32 nonces,
    two chunks of 2^23 buckets; one set of chunk buffers serves both), two
    ways: every chunk hashing all nonces (vx_plot_chunk), and one stage hash
    from which every chunk is made (vx_stage_plot + vx_plot_staged_chunk).
    Seconds per whole plot (the staged way is `value`), and per chunk.  At
    k <= 31 the same plot through vx_plot is timed too."""
    import torch
    import paper_2606_14007_amd as vx
    from vx_inputs import derive_key

    k, c = args.chunk_k, args.chunk_bits
    key = derive_key(0)
    nchunks = 1 << c
    steps = max(1, args.steps)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(nchunks + 2)]

    def run(make_chunk, b, stage_fn=None, timed=False):
        t1 = t2 = 0
        if timed:
            evs[0].record()
        if stage_fn:
            stage_fn()
        if timed:
            evs[1].record()
        for r in range(nchunks):
            make_chunk(r)
            t2n = vx.t2_count(b)  # synchronises; the buffers are reused by the next chunk
            if t2n > b.t2_capacity:
                raise RuntimeError("Table 2 overflow")
            t1 += int(b.t1_count.item())
            t2 += t2n
            if timed:
                evs[r + 2].record()
        return t1, t2

    def measure(label, make_chunk, b, stage_fn=None):
        for _ in range(max(1, args.warmup)):
            run(make_chunk, b, stage_fn)
        if vx.device_status(b.workspace):
            raise RuntimeError("device status")
        part = [0.0] * (nchunks + 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            t1, t2 = run(make_chunk, b, stage_fn, timed=True)
            torch.cuda.synchronize()
            for i in range(nchunks + 1):
                part[i] += evs[i].elapsed_time(evs[i + 1]) / steps
        sec = (time.perf_counter() - t0) / steps
        if t1 != 1 << k:
            raise RuntimeError(f"chunks hold {t1} records, not 2^{k}")
        log(f"k={k} {label}: {sec * 1e3:.1f} ms per plot in {nchunks} chunks "
            f"(stage {part[0]:.1f} ms; chunks {', '.join(f'{x:.1f}' for x in part[1:])} ms)")
        return sec, part, t2

    b = vx.alloc_chunk(k, c)
    log(f"chunked: k={k} in {nchunks} chunks, {b.nbytes() / 2**30:.1f} GiB of chunk buffers")
    rehash_s, rehash_part, t2 = measure("rehash", lambda r: vx.plot_chunk(key, k, c, r, b), b)
    rehash_bytes = b.nbytes()
    del b
    torch.cuda.empty_cache()
    st = vx.alloc_stage(k, c)
    b = vx.alloc_staged_chunk(k, c)
    staged_bytes = b.nbytes() + st.data.numel()
    log(f"staged: {st.data.numel() / 2**30:.1f} GiB stage + {b.nbytes() / 2**30:.1f} GiB of chunk buffers")
    staged_s, staged_part, t2s = measure("staged", lambda r: vx.plot_staged_chunk(key, st, r, b), b,
                                         lambda: vx.stage_plot(key, k, c, st))
    if t2s != t2:
        raise RuntimeError("staged and rehashed chunks differ in |Table 2|")
    out = {
        "metric": f"K={k} plot seconds (chunked)",
        "value": round(staged_s, 5),
        "unit": "s",
        "n_gpus": 1, "steps": steps, "warmup": max(1, args.warmup),
        "ms_per_step": round(staged_s * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"k={k} single plot in {nchunks} chunks of {1 << (24 - c)} buckets",
                   "k": k, "chunk_bits": c, "key_seed": 0, "threshold": f"2^{64 - k}",
                   "parallelism": "single GPU"},
        "staged_stage_ms": round(staged_part[0], 3),
        "staged_chunk_ms": [round(x, 3) for x in staged_part[1:]],
        "rehash_plot_s": round(rehash_s, 5),
        "rehash_chunk_ms": [round(x, 3) for x in rehash_part[1:]],
        "table1_records": 1 << k, "table2_records": t2,
        "staged_device_bytes": staged_bytes, "rehash_device_bytes": rehash_bytes,
        "blake3_hashes_per_s_useful": round(((1 << k) + t2) / staged_s, 1),
    }
    if k <= 31:
        del b, st
        torch.cuda.empty_cache()
        wb = vx.alloc_plot(k)
        vx.plot(key, k, buffers=wb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            vx.plot(key, k, buffers=wb)
        torch.cuda.synchronize()
        ws = (time.perf_counter() - t0) / steps
        log(f"k={k}: {ws * 1e3:.1f} ms as one vx_plot")
        out["whole_plot_ms"] = round(ws * 1e3, 3)
        out["staged_cost_vs_whole"] = round(staged_s / ws, 3)
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--k", type=int, default=31)
    ap.add_argument("--cpu-sample-k", type=int, default=27)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", default="",
                    help="k31: implementation parameters as name=value,... (vx_tuning fields; "
                         "none changes any output), e.g. fused_sort_match=1")
    ap.add_argument("--no-batched", action="store_true",
                    help="k31: skip the batched-vs-sequential part of the line")
    ap.add_argument("--workload", choices=["k31", "batched", "serving", "egress", "chunked"], default="k31",
                    help="k31: one whole plot (the default line); batched: the 32-plot mix; "
                         "serving: Poisson requests through the continuous-batching server; "
                         "egress: Table 2 streamed to plot files; chunked: one plot in chunks")
    ap.add_argument("--chunk-k", type=int, default=32, help="chunked: k of the plot")
    ap.add_argument("--chunk-bits", type=int, default=1, help="chunked: 2^c chunks")
    ap.add_argument("--requests", type=int, default=1000, help="serving: number of requests")
    ap.add_argument("--big-k", type=int, default=28,
                    help="serving: jobs with k at or above this run one at a time")
    ap.add_argument("--egress-k", type=int, default=28, help="egress: k of every plot")
    ap.add_argument("--egress-dir", default=None, help="egress: write plot files here (default: discard)")
    ap.add_argument("--egress-slots", type=int, default=4, help="egress: pinned staging buffers")
    ap.add_argument("--egress-slot-mb", type=int, default=64, help="egress: MiB per staging buffer")
    ap.add_argument("--budget-gb", type=float, default=250.0, help="serving: HBM budget (GiB)")
    ap.add_argument("--autotune", action="store_true",
                    help="batched: use the cached autotuned tuning per k")
    ap.add_argument("--shared-hash", action="store_true",
                    help="batched: let plots share hash launches (device work list) instead of lanes")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 2 GiB device-to-device copy (known bytes) so that "
                         "HBM byte counters can be scaled against it")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only: a plot runs on one MI355X and this build has no "
              f"multi-GPU path (asked for --gpus {args.gpus}, WORLD_SIZE={world}).",
              file=sys.stderr)
        return 2

    if args.workload in ("batched", "serving", "egress", "chunked"):
        import torch
        torch.cuda.set_device(0)
        fn = {"batched": bench_batched, "serving": bench_serving, "egress": bench_egress,
              "chunked": bench_chunked}[args.workload]
        print(json.dumps(fn(args)), flush=True)
        return 0

    import torch
    import paper_2606_14007_amd as vx
    from paper_2606_14007_amd import opcount
    from vx_inputs import derive_key

    k = args.k
    key = derive_key(0)
    T = vx.vx_default_threshold(k)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"device: {torch.cuda.get_device_name(0)}; k={k}; allocating "
        f"{vx.footprint_bytes(k, T) / 2**30:.1f} GiB")
    tun = None
    if args.tuning:
        tun = vx.make_tuning(**{kv.split("=")[0]: int(kv.split("=")[1]) for kv in args.tuning.split(",")})
        log(f"tuning: {args.tuning}")
    bufs = vx.alloc_plot(k, T, tuning=tun, device=dev)
    params = vx.make_params(key, k, T)
    nb = bufs.native()
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream

    if args.calibrate_copy:
        src = torch.empty(1 << 31, dtype=torch.uint8, device=dev).fill_(7)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 2 GiB read + 2 GiB written")
        del src, dst

    for i in range(args.warmup):
        vx.vx_plot(params, nb, tun, sh)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    status = vx.device_status(bufs.workspace)
    if status:
        raise RuntimeError(f"device status {status:#x}")

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(vx.VX_PLOT_EVENTS)]
              for _ in range(args.steps)]
    for row in events:
        for e in row:
            e.record(stream)  # materialise the hipEvent_t handles
    torch.cuda.synchronize()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for row in events:
        vx.vx_plot_with_events(params, nb, [e.cuda_event for e in row], tun, sh)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"timed {args.steps} plots in {t1 - t0:.3f} s")

    t2n = vx.check_plot(bufs, what=f"k={k} plot")   # raises on Table-2 overflow or a device status
    n = 1 << k
    stage_ms = {s: 0.0 for s in STAGES}
    for row in events:
        for i, s in enumerate(STAGES):
            stage_ms[s] += row[i].elapsed_time(row[i + 1]) / args.steps
    event_total = sum(stage_ms.values())
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    plot_s = ms_per_step / 1000.0

    # Rooflines per stage (algorithmic work per launch / event-measured time).
    # VALU work in two forms: algorithmic 32-bit ops (every add, xor and
    # rotate one op), the unit of the target, and vector instructions (a
    # three-input add is one), what the kernels issue.
    h1_ops = opcount.ops_per_h1() * n
    h2_ops = opcount.ops_per_h2() * t2n
    h1_ins = opcount.valu_per_h1() * n
    h2_ins = opcount.valu_per_h2() * t2n
    valu_peak = opcount.MI355X_VALU_LANE_OPS_PER_S
    hbm_peak = opcount.MI355X_HBM_BYTES_PER_S
    npass = vx.vx_partition_passes(params, tun)
    hslices = vx.vx_hash_slices(params, tun)
    tslices = vx.vx_tail_slices(params, tun)
    # With two or more passes the hash kernel also does the first pass (its
    # stage is then only the region scan); a one-pass plot hashes alone.  A
    # plot hashed in slices also does the second pass in the hash launches,
    # and the third where it has one (launch i filing slice i - 2).
    fused_first = npass >= 2
    in_hash = vx.vx_front_passes(params, tun)
    hlaunches = hslices + max(in_hash - 1, 1) if hslices > 1 else 1
    kernel_of = dict(KERNEL_OF_STAGE)
    if not fused_first:
        kernel_of.update(hash="k_hash_table1", partition1="k_digit_hist + k_scatter (pass 1)")
    if hslices > 1 and in_hash == 3:
        kernel_of.update(hash=(f"k_hash_pass x{hlaunches} (hash in {hslices} slices + the second and "
                               "third passes)"),
                         partition1="k_region_scan_slices + k_region_bounds + k_colscan (passes 2-3 are in the hash)",
                         partition2="(in the hash launches)")
    elif hslices > 1:
        kernel_of.update(hash=f"k_hash_pass x{hlaunches} (hash in {hslices} slices + the second pass)",
                         partition1="k_region_scan_slices + k_region_bounds + k_colscan (pass 2 is in the hash)",
                         partition2="k_scatter claiming regions + k_region_bounds + k_colscan (third pass)")
    in_tail = 1 if tslices > 1 and npass == 3 else 0
    if tslices > 1:
        kernel_of.update(match_emit=(f"k_pipe x{tslices + 1 + in_tail} ("
                                     + ("third pass + " if in_tail else "")
                                     + f"group sort + match + H2, pipelined over {tslices} slices)"),
                         group_sort="(in the pipelined tail)", chunk_sums="(sums made by the sort)")
    algo_bytes = {
        "partition1": 0 if fused_first else n * (8 + 12),  # read key, write key+nonce
        # each later pass reads and writes key+nonce
        "partition2": max(0, npass - max(in_hash, 1) - in_tail) * n * (12 + 12),
        # read and write key+nonce, offsets, one pair-count byte per record
        "group_sort": n * (12 + 12 + 1) + (vx.VX_NUM_BUCKETS + 1) * 4,
        "chunk_sums": n * 1,                     # read the count bytes
    }
    stages = {}
    for s in STAGES:
        sec = stage_ms[s] / 1000.0
        ent = {"ms": round(stage_ms[s], 3), "kernel": kernel_of[s]}
        if sec > 0:
            if s in ("hash", "match_emit"):
                ops, ins = (h1_ops, h1_ins) if s == "hash" else (h2_ops, h2_ins)
                ent.update(bound="alu", achieved=ops / sec / 1e12, peak=valu_peak / 1e12,
                           unit="T lane-ops/s",
                           instruction_form={"achieved": round(ins / sec / 1e12, 2),
                                             "frac": round(ins / sec / valu_peak, 4),
                                             "per_hash": opcount.valu_per_h1()})
            elif algo_bytes[s]:
                ent.update(bound="hbm", achieved=algo_bytes[s] / sec / 1e9, peak=hbm_peak / 1e9,
                           unit="GB/s")
            if "peak" in ent:
                ent["frac"] = round(ent["achieved"] / ent["peak"], 4)
                ent["achieved"] = round(ent["achieved"], 2)
        stages[s] = ent
    dom = max(STAGES, key=lambda s: stage_ms[s])
    d = stages[dom]
    traffic = load_traffic(kernel_of[dom].split()[0], k,
                           hlaunches if dom == "hash" else 1)
    alu = d.get("bound") == "alu"
    roofline = {"bound": d.get("bound"), "achieved": d.get("achieved"), "peak": d.get("peak"),
                "unit": "TOP/s" if alu else "GB/s",
                "frac": d.get("frac"), "traffic": traffic, "kernel": d["kernel"], "stage": dom,
                "work_per_launch": (h1_ops if dom == "hash" else h2_ops if dom == "match_emit"
                                    else algo_bytes.get(dom)),
                "work_unit": ("algorithmic 32-bit ops (%d per Table-1 hash, %d per Table-2 hash)"
                              % (opcount.ops_per_h1(), opcount.ops_per_h2()) if alu else "bytes")}
    if alu:
        roofline["instruction_form"] = dict(d["instruction_form"], unit="T VALU lane-instructions/s")
    if traffic and stage_ms[dom] > 0:
        # The same stage against the HBM roof, from the measured bytes: the
        # hash launches that also file the partition passes move them at a
        # rate that bounds them as much as their vector work does.
        bw = traffic / (stage_ms[dom] / 1000.0)
        roofline["hbm_side"] = {"achieved": round(bw / 1e9, 1), "peak": hbm_peak / 1e9, "unit": "GB/s",
                                "frac": round(bw / hbm_peak, 4)}

    # The other two parts of the metric: Blake3 hashes/s (above) and mixed-k
    # plots/hour batched against plain, measured after the k=31 buffers are freed.
    del bufs, nb
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    batched = None
    if not args.no_batched:
        log("batched mix: 32 plots, k 22..29 (seed 4), sequential vs vx_plot_batch ...")
        batched = batched_compare(reps=3)

    out = {
        "metric": "K=31 plot seconds" if k == 31 else f"K={k} plot seconds",
        "value": round(plot_s, 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"k={k} single plot", "k": k, "nonces": n, "key_seed": 0,
                   "threshold": f"2^{64 - k}", "buckets": 1 << 24, "partition_passes": npass,
                   "hash_slices": hslices, "front_passes": in_hash, "tail_slices": tslices, "parallelism": "single GPU"},
        "blake3_hashes_per_s": round((n + t2n) / plot_s, 1),
        "plots_per_hour": round(3600.0 / plot_s, 1),
        "table2_records": t2n,
        "stage_ms": {s: stages[s]["ms"] for s in STAGES},
        "event_total_ms": round(event_total, 3),
        "stages": stages,
        "roofline": roofline,
    }
    if batched:
        out["batched_plots_per_hour"] = batched["batched_plots_per_hour"]
        out["sequential_plots_per_hour"] = batched["sequential_plots_per_hour"]
        out["batched_speedup_vs_sequential"] = batched["speedup_vs_sequential"]
        out["batched"] = batched
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_k, k)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

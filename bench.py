#!/usr/bin/env python3
"""Throughput benchmark of the LOCC crop-collision path on one MI355X.

One step = the whole path (crop, encoder, head, world mapping) over one batch
of synthetic pairs resident in HBM.  Prints one JSON line with pair-queries/s,
per-step latency percentiles, the roofline of the dominant kernel (timed with
HIP events on its launch stream inside the library) and the CPU FP64 oracle
timed on this host on a bounded sample of the same workload.

  python bench.py [--steps K] [--warmup W] [--workload scale|small] [--precision fp32,bf16,fp8,fp8_encoder]

Counter post-processing (turns rocprofv3 --pmc CSV output into a summary):
  python bench.py --summarize-counters FETCH_DIR WRITE_DIR --copy-mib M --kernel NAME
  python bench.py --summarize-sq PASS1_DIR PASS2_DIR --kernel NAME --kernel-match STR
"""

from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-CD queries/sec at 1 GPU (BF16 batched vs FP32 plain); p99 step latency"
UNIT = "pair-queries/s"

# step-latency percentiles are taken over at least this many steps
LATENCY_SAMPLES = 200

# MI355X published peaks
PEAK_HBM_GBPS = 8000.0
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}

CSRC = os.path.join(ROOT, "paper_2304_09439_amd", "csrc")
KERNEL_SOURCES = {
    "crop_fp32": ["crop.hip", "geometry.h"],   # the crop kernel writing float32 rows
    "crop_bf16": ["crop.hip", "geometry.h"],   # ... bf16 rows (BF16 split schedule)
    "crop_fp8": ["crop.hip", "geometry.h"],    # ... bf16 rows (FP8 path)
    "encoder_fp32": ["net_fp32.hip"],
    "head_fp32": ["net_fp32.hip"],
    "fused_bf16": ["fused.hip", "fused.h", "geometry.h", "post.h", "head_bf16.h"],
    # the split schedule's two encoder+head kernels (two workgroups per CU: fused.hip; one: encoder_bf16.hip)
    "encoder_head_bf16": ["fused.hip", "fused.h", "geometry.h", "post.h", "head_bf16.h"],
    "encoder_head_bf16_lds": ["encoder_bf16.hip", "fused.h", "geometry.h", "post.h", "head_bf16.h"],
    "encoder_head_fp8": ["fused_fp8.hip", "fused.h", "post.h"],
    "encoder_fp8_head_bf16": ["fused_fp8.hip", "fused.h", "head_bf16.h", "post.h"],
    "crop_fp8_encoder": ["crop.hip", "geometry.h"],
}
# arithmetic of the encoder and of the head in each network kernel (None: not in that kernel)
KERNEL_PREC = {
    "encoder_fp32": ("fp32", None), "head_fp32": (None, "fp32"),
    "fused_bf16": ("bf16", "bf16"), "encoder_head_bf16": ("bf16", "bf16"), "encoder_head_bf16_lds": ("bf16", "bf16"),
    "encoder_head_fp8": ("fp8", "fp8"),              # encoder layer 1 and head layer 3 are bf16: charged at fp8
    "encoder_fp8_head_bf16": ("fp8", "bf16"),        # encoder layer 1 bf16 charged at fp8 too
}
PATH_DESC = {
    "fp32": "per-step FP32: crop, encoder and head kernels on one stream",
    "bf16": "batched BF16 (schedule chosen by the library's autotuner)",
    "fp8": "batched FP8: crop kernel, then one persistent encoder+head launch (encoder layer 2 and head "
           "layers 1-2 e4m3 x e4m3, encoder layer 1 and head layer 3 bf16; activation scales calibrated "
           "on the first 1,024 pairs)",
    "fp8_encoder": "batched FP8, lower-error variant: crop kernel, then one persistent encoder+head launch "
                   "(encoder layer 2 e4m3 x e4m3, encoder layer 1 and the whole head bf16; the activation scale "
                   "calibrated on the first 1,024 pairs)",
}


def bf16_desc(schedule):
    if not schedule:
        return PATH_DESC["bf16"]
    if schedule["split"]:
        return ("batched BF16: crop kernel, then one persistent encoder+head launch over all pairs "
                f"(autotuned: {schedule})")
    return f"batched BF16: one persistent fused crop+encoder+head launch over all pairs (autotuned: {schedule})"


def workload(name: str):
    from paper_2304_09439_amd import inputs as I
    if name == "scale":
        scene = I.scale_workload()
        return dict(scene=scene, K=128, widths=I.SCALE_WIDTHS, n_points=2048, n_shapes=32,
                    desc="16384 object pairs, 32 procedural shapes (3-6 ellipsoids/boxes) x 2048 surface points, "
                         "K=128, encoder 6-128-256, head 512-512-512-8")
    if name == "small":
        scene = I.small_workload()
        return dict(scene=scene, K=64, widths=I.SMALL_WIDTHS, n_points=1024, n_shapes=160,
                    desc="80 object pairs (64 three-ellipsoid unions + 16 spheres) x 1024 surface points, "
                         "K=64, encoder 6-64-128, head 256-256-256-8")
    raise SystemExit(f"unknown workload {name}")


def per_pair_work(K, widths, n_points):
    """Algorithmic work per pair (fixed 2K encoder rows; padding excluded)."""
    h1, h2, hh = widths.h1, widths.h2, widths.hh
    enc_flops = 2 * (2 * K) * (6 * h1 + h1 * h2)
    head_flops = 2 * (2 * h2 * hh + hh * hh + 8 * hh)
    crop_bytes = 2 * n_points * 12 + 2 * K * 24 + 2 * 32 + 8 + 8   # scan xyz, gather rows, poses, pair, counts
    return dict(enc_flops=enc_flops, head_flops=head_flops, crop_bytes=crop_bytes, contact_bytes=32, K=K,
                row_flops=2 * (6 * h1 + h1 * h2))


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, []) + ["locc_internal.h"]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel: str, workload_name: str):
    """HBM bytes per launch from a committed counter summary, if it was taken on this kernel source."""
    return counter_value(kernel, workload_name, "hbm", "hbm_bytes_per_launch")


# ------------------------------------------------------------------ CPU baseline

_CPU = {}


def _cpu_chunk(rows):
    from threadpoolctl import threadpool_limits
    from oracle import locc_oracle as O
    c = _CPU
    with threadpool_limits(1):
        O.detect_scene(c["scene"], c["w"], c["widths"], c["K"], rows=rows)
    return len(rows)


def cpu_model() -> str:
    """The host CPU's model name as /proc/cpuinfo gives it."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _one_core(scene, w, widths, K, rows):
    """The oracle on `rows` of `scene` in this process with one BLAS thread; pairs/s."""
    from threadpoolctl import threadpool_limits
    from oracle import locc_oracle as O
    with threadpool_limits(1):
        t0 = time.perf_counter()
        O.detect_scene(scene, w, (widths.h1, widths.h2, widths.hh), K, rows=rows)
        dt = time.perf_counter() - t0
    return len(rows) / dt, dt


def cpu_baseline(scene, w, widths, K, n_pairs, small=None, single_pairs=1024):
    """The oracle on the host: the first n_pairs pairs over a fork pool (one BLAS thread per worker, all
    affinity cores up to 16), then on one core the first `single_pairs` pairs of the same workload and, when
    given, the whole small workload (small = (scene, weights, widths, K))."""
    import multiprocessing as mp
    import numpy as np
    _CPU.update(scene=scene, w=w, widths=(widths.h1, widths.h2, widths.hh), K=K)
    n_pairs = min(n_pairs, scene.n_pairs)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    chunks = np.array_split(np.arange(n_pairs), max(workers * 4, 1))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        done = sum(pool.map(_cpu_chunk, chunks))
    dt = time.perf_counter() - t0
    single = {}
    rate, t1 = _one_core(scene, w, widths, K, np.arange(min(single_pairs, scene.n_pairs)))
    single["scale_pairs_0_%d" % min(single_pairs, scene.n_pairs)] = dict(value=round(rate, 1), unit=UNIT,
                                                                        seconds=round(t1, 2))
    if small is not None:
        s_scene, s_w, s_widths, s_K = small
        rate, t1 = _one_core(s_scene, s_w, s_widths, s_K, np.arange(s_scene.n_pairs))
        single["small_all_%d_pairs" % s_scene.n_pairs] = dict(value=round(rate, 1), unit=UNIT, seconds=round(t1, 2))
    return dict(value=done / dt, unit=UNIT, cores=workers, kind="oracle", cpu_model=cpu_model(),
                affinity_cores=len(os.sched_getaffinity(0)),
                sample=f"first {done} pairs of the same workload, float64 NumPy oracle (crop + network + "
                       f"outputs), {workers} worker processes x 1 BLAS thread, {dt:.2f} s wall",
                single_core=single)


# ------------------------------------------------------------------ GPU run

def kernel_entries(kt, work, P, workload_name, steps, precision, full_scan=True, rows=None):
    """Per kernel: average launch duration and the rate of one launch (a step of P pairs may run a kernel
    several times, once per chunk of pairs).

    Encoder kernels are charged the method's own work: `rows` = (valid, tiles), the encoder rows of the
    step's objects, valid = min(count, K) per object (the rows the method defines), tiles = those rows
    rounded up to the 32-row tiles the kernels run.  `frac` is on the valid rows (plus the head on every
    pair); the fixed-2K-row count of the measurement plan and the tile count are reported beside it.
    The crop is charged the HBM bytes it has to move (poses, pair, counts, the 2K rows it writes in this
    path's format); its scans read the shape library from L2 and stop at K members unless member counts
    are requested, so their algorithmic byte rate is reported without a fraction."""
    kernels = {}
    for name, (launches, total_ms) in sorted(kt.items()):
        avg = total_ms / max(launches, 1)
        P_launch = P * steps / max(launches, 1)
        entry = dict(avg_ms=round(avg, 4), launches=int(launches), pairs_per_launch=round(P_launch, 1))
        if name == "crop":
            row_bytes = 32 if precision == "fp32" else 16
            hbm = 2 * 32 + 8 + 8 + 2 * work["K"] * row_bytes
            hbm_rate = hbm * P_launch / (avg * 1e-3) / 1e9
            scan_rate = work["crop_bytes"] * P_launch / (avg * 1e-3) / 1e9
            entry.update(bound="hbm", achieved=round(hbm_rate, 1), peak=PEAK_HBM_GBPS, unit="GB/s",
                         frac=round(hbm_rate / PEAK_HBM_GBPS, 4), hbm_bytes_per_pair=hbm,
                         bytes_basis="HBM bytes a crop moves: poses, pair, counts and the 2K encoder rows it writes; "
                                     "the kernel is bound by the latency of its dependent scan-select-gather chain, "
                                     "not by bandwidth",
                         scan_GBps=round(scan_rate, 1),
                         scan_basis="the measurement plan's algorithmic bytes (full scans of both objects, 2N x 12 B "
                                    "per pair, + 2K gathered rows + poses, pair, counts) per launch time; the scans "
                                    "read the shape library from L2" + (
                                        "" if full_scan else " and stop at K members without member counts"))
        else:
            enc_prec, head_prec = KERNEL_PREC[name]
            enc = enc_prec is not None
            head = work["head_flops"] * P_launch if head_prec else 0.0
            fixed_enc = work["enc_flops"] * P_launch if enc else 0.0
            if enc and rows is not None:
                valid_enc = rows[0] * work["row_flops"] * P_launch / P
                tiles_enc = rows[1] * work["row_flops"] * P_launch / P
            else:
                valid_enc = tiles_enc = fixed_enc

            def peak_of(e):   # the rate at which the kernel's encoder and head work would take their peak time
                t = (e / PEAK_TFLOPS[enc_prec] if enc else 0.0) + (head / PEAK_TFLOPS[head_prec] if head_prec else 0.0)
                return (e + head) / t
            peak = round(peak_of(valid_enc), 1)
            valid, tiles, fixed = valid_enc + head, tiles_enc + head, fixed_enc + head
            rate = lambda f: f / (avg * 1e-3) / 1e12
            entry.update(bound="mfma", achieved=round(rate(valid), 2), peak=peak, unit="TFLOP/s",
                         frac=round(rate(valid) / peak, 4),
                         flops_basis=("encoder rows min(count, K) per object (the method's crop sets) + head on "
                                      "every pair" if enc else "head on every pair"),
                         fixed_2K_TFLOPs=round(rate(fixed), 2), fixed_2K_frac=round(rate(fixed) / peak_of(fixed_enc), 4),
                         tiles_run_TFLOPs=round(rate(tiles), 2), tiles_run_frac=round(rate(tiles) / peak_of(tiles_enc), 4))
            if enc_prec and head_prec and enc_prec != head_prec:
                entry["peak_basis"] = (f"encoder FLOPs at the {enc_prec} peak and head FLOPs at the {head_prec} peak "
                                       "(the rate at which this work would take its time at those peaks)")
            if name.startswith("fused"):  # crop inside: its HBM bytes too
                gbps = (2 * 32 + 8 + 8 + work["contact_bytes"]) * P_launch / (avg * 1e-3) / 1e9
                entry.update(hbm_achieved_GBps=round(gbps, 1), hbm_frac=round(gbps / PEAK_HBM_GBPS, 4))
        key = f"crop_{precision}" if name == "crop" else name
        entry["traffic"] = counter_traffic(key, workload_name)
        issue_ns = counter_value(key, workload_name, "sq", "valu_issue_bound_ns")
        if name == "crop" and issue_ns is not None:
            # the bound the crop can reach: its vector instructions issued back to back on every SIMD
            entry["issue_bound"] = dict(bound_ms=round(issue_ns * 1e-6, 4), frac=round(issue_ns * 1e-6 / avg, 4),
                                        basis="SQ_INSTS_VALU per launch x 4 cycles / (1024 SIMDs x 2.4 GHz), from "
                                              "the committed SQ counter summary of this kernel source")
        busy = counter_value(key, workload_name, "sq", "mfma_busy_frac")
        if busy is not None and name != "crop":
            entry["mfma_busy_frac"] = busy
        kernels[name] = entry
    return kernels


def encoder_rows(counts, K):
    """(valid, tiles): encoder rows min(count, K) summed over the objects of the valid pairs, and the same
    rounded up per object to the 32-row tiles the kernels run."""
    import numpy as np
    c = counts[counts[:, 0] >= 0]
    c = np.clip(c, 0, K)
    return int(c.sum()), int((((c + 31) // 32) * 32).sum())


def time_path(args, scene, K, widths, w, precision, work, workload_name):
    import numpy as np
    import torch
    from paper_2304_09439_amd import binding as B
    wd = (widths.h1, widths.h2, widths.hh)
    ctx = B.context_for_scene(scene, K, wd, w, precision=precision)
    objs, pairs = B.scene_tensors(scene)
    P = scene.n_pairs
    out = torch.empty((P, 8), dtype=torch.float32, device="cuda")
    # the query's outputs are the contacts; the per-object member counts are an optional diagnostic, and
    # without them each object's scan stops once its first K members are known (same contacts)
    counts = torch.empty((P, 2), dtype=torch.int32, device="cuda") if args.member_counts else None
    stream = torch.cuda.current_stream()
    schedule = None
    if precision.startswith("fp8"):
        amax = ctx.calibrate(objs, pairs[:min(P, 1024)])
        print(f"[bench] {precision}: activation maxima {amax.tolist()}", file=sys.stderr, flush=True)
    if precision != "fp32" and args.schedule.get(precision):
        ctx.set_schedule(**args.schedule[precision])   # a schedule given on the command line
        schedule = ctx.get_schedule()
    elif precision != "fp32" and not args.no_autotune:
        schedule, _ = ctx.autotune(objs, pairs, want_counts=counts is not None)   # the library's own autotuner
    for _ in range(args.warmup):
        ctx.detect(objs, pairs, out, counts, want_counts=counts is not None)
    torch.cuda.synchronize()
    print(f"[bench] {precision}: warmup done ({args.warmup} steps), timing {args.steps} steps of {P} pairs",
          file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ctx.detect(objs, pairs, out, counts, want_counts=counts is not None)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-kernel durations: the same number of steps again with the library's per-kernel events (start and
    # stop events attached to the dispatches), kept out of the timed region above because they lengthen a
    # step by about a tenth
    ctx.profile(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        ctx.detect(objs, pairs, out, counts, want_counts=counts is not None)
    torch.cuda.synchronize()
    wall_prof = time.perf_counter() - t1
    ctx.profile(False)
    kt = ctx.profile_read()
    # step latency percentiles from their own run of at least LATENCY_SAMPLES steps, each between two events
    n_lat = 0 if args.profile_run else max(LATENCY_SAMPLES, args.steps)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_lat)]
    for k in range(n_lat):
        ev[k][0].record(stream)
        ctx.detect(objs, pairs, out, counts, want_counts=counts is not None)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    step_ms = np.array([a.elapsed_time(b) for a, b in ev])
    extra = {"latency_samples": n_lat,
             "kernel_timing": dict(steps=args.steps, ms_per_step=round(1000.0 * wall_prof / args.steps, 4),
                                   note="kernel durations from a second run of the same steps with per-kernel "
                                        "events, after the timed region")}
    full = counts
    if counts is None and not args.profile_run:   # the same schedule with member counts (every point tested)
        full = torch.empty((P, 2), dtype=torch.int32, device="cuda")
        ctx.detect(objs, pairs, out, full)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            ctx.detect(objs, pairs, out, full)
        torch.cuda.synchronize()
        extra["ms_per_step_with_member_counts"] = round(1000.0 * (time.perf_counter() - t1) / args.steps, 4)
    if precision == "bf16" and schedule and not args.profile_run:
        extra["schedule_alternatives"] = schedule_alternatives(ctx, objs, pairs, out, counts, schedule, stream,
                                                               args.steps)
    n_bad = ctx.device_errors()
    ctx.close()
    rows = encoder_rows(full.cpu().numpy(), K) if full is not None else None
    ms = 1000.0 * wall / args.steps
    kernels = kernel_entries(kt, work, P, workload_name, args.steps, precision, full_scan=counts is not None,
                             rows=rows)
    return dict(value=round(P / (ms * 1e-3), 1), ms_per_step=round(ms, 4), schedule=schedule,
                p50_step_ms=round(float(np.percentile(step_ms, 50)), 4) if n_lat else None,
                p99_step_ms=round(float(np.percentile(step_ms, 99)), 4) if n_lat else None,
                kernels=kernels, device_errors=int(n_bad), member_counts=bool(args.member_counts), **extra,
                path={"fp32": PATH_DESC["fp32"], "fp8": PATH_DESC["fp8"] + f" (autotuned: {schedule})",
                      "fp8_encoder": PATH_DESC["fp8_encoder"] + f" (autotuned: {schedule})"}.get(
                    precision, bf16_desc(schedule)))


def schedule_alternatives(ctx, objs, pairs, out, counts, best, stream, steps):
    """ms per step of the chosen schedule and of the ones that would overlap or fuse the crop: one fused
    launch (crop inside the network kernel), the split schedule cut into 2 and 4 runs whose crops overlap
    the previous run's network (on the context's second stream), and the same at one network workgroup per
    CU (leaving room on every CU for the next run's crop).  Same pairs, events on the launch stream."""
    import torch
    want = counts is not None
    variants = {"chosen": dict(best), "one_fused_launch": dict(best, split=False, chunks=1, crop_unroll=8),
                "split_2_runs": dict(best, chunks=2), "split_4_runs": dict(best, chunks=4),
                "split_2_runs_1_wg_per_cu": dict(best, chunks=2, wg_per_cu=1)}
    res = {}
    for name, sc in variants.items():
        ctx.set_schedule(**sc)
        for _ in range(3):
            ctx.detect(objs, pairs, out, counts, want_counts=want)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            ctx.detect(objs, pairs, out, counts, want_counts=want)
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = round(e0.elapsed_time(e1) / steps, 4)
    ctx.set_schedule(**best)
    return res


def time_envs(args, envs, w, precision, gpu_broad=False):
    """One simulation step of the uneven-environment workload: H2D of every pose, the step's broad-phase
    pairs and their count from pinned host buffers, then the detect (a replayed HIP graph for the
    batched path, eager launches for the plain FP32 path).  With gpu_broad, H2D of the poses only and
    one replayed graph holding the library's broad phase and the detect on its device count.  Timed
    per step with events."""
    import numpy as np
    import torch
    from paper_2304_09439_amd import binding as B
    widths = envs_widths()
    ctx = B.Context(128, widths, precision=precision)
    ctx.upload_shapes(envs.lib.offsets, envs.lib.pts)
    ctx.upload_weights(w)
    S = envs.n_steps
    n_obj = len(envs.shape)
    cap = max(len(p) for p in envs.pairs)
    objs_h = [torch.from_numpy(B.pack_objects(envs.pos[s], envs.quat[s], envs.shape)).pin_memory() for s in range(S)]
    pairs_h = [torch.from_numpy(np.ascontiguousarray(p)).pin_memory() for p in envs.pairs]
    n_h = [torch.tensor([len(p)], dtype=torch.int32).pin_memory() for p in envs.pairs]
    objs = torch.empty((n_obj, 8), dtype=torch.float32, device="cuda")
    pairs = torch.zeros((cap, 2), dtype=torch.int32, device="cuda")
    n_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = torch.empty((cap, 8), dtype=torch.float32, device="cuda")
    counts = torch.empty((cap, 2), dtype=torch.int32, device="cuda") if args.member_counts else None
    ctx.reserve(cap)
    graph, schedule = None, None
    env_off = torch.from_numpy(envs.env_offsets).cuda()
    count = torch.zeros(2, dtype=torch.int32, device="cuda")
    if precision != "fp32":
        objs.copy_(objs_h[0])
        pairs[:len(envs.pairs[0])].copy_(pairs_h[0])
        if not args.no_autotune:
            schedule, _ = ctx.autotune(objs, pairs[:len(envs.pairs[0])], want_counts=counts is not None)
        if gpu_broad:
            graph = ctx.capture_step_graph(objs, env_off, pairs, count, out, counts)
        else:
            graph = ctx.capture_graph(objs, pairs, n_dev, out, counts)
    stream = torch.cuda.current_stream()

    def step(s):
        P = len(envs.pairs[s])
        objs.copy_(objs_h[s], non_blocking=True)
        if gpu_broad:
            graph.launch()
            return
        pairs[:P].copy_(pairs_h[s], non_blocking=True)
        if graph is not None:
            n_dev.copy_(n_h[s], non_blocking=True)
            graph.launch()
        else:
            ctx.detect(objs, pairs[:P], out[:P], None if counts is None else counts[:P], want_counts=counts is not None)

    # one untimed pass over every step: each step has pinned host buffers of its own, and the first copy out of
    # a pinned buffer pays for mapping it, which a simulation reusing one staging buffer per step would not
    for s in range(S):
        step(s)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(S)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(S):
        ev[s][0].record(stream)
        step(s)
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([a.elapsed_time(b) for a, b in ev])
    total_pairs = sum(len(p) for p in envs.pairs)
    extra = {}
    if gpu_broad:
        # the last step's count against the host list, then the broad phase alone (event-timed launches)
        extra["last_step_count_matches_host"] = count.cpu().tolist() == [len(envs.pairs[-1])] * 2
        ctx.profile(True)
        for s in range(S):
            objs.copy_(objs_h[s], non_blocking=True)
            ctx.broad_phase(objs, env_off, pairs, count)
        torch.cuda.synchronize()
        n_l, tot = ctx.profile_read()["broad_phase"]
        ctx.profile(False)
        extra["broad_phase_ms"] = round(tot / n_l, 5)
    n_bad = ctx.device_errors()
    if graph is not None:
        graph.close()
    ctx.close()
    if gpu_broad:
        path = "HIP graph per step (H2D of poses + replay of broad phase and detect), " + bf16_desc(schedule)
    elif graph is not None:
        path = "HIP graph per step (H2D of poses, pairs and count + replay), " + bf16_desc(schedule)
    else:
        path = "eager per step (H2D of poses and pairs + launches), " + PATH_DESC[precision]
    return dict(value=round(total_pairs / wall, 1), unit=UNIT, steps=S, mean_pairs_per_step=round(total_pairs / S),
                p50_step_ms=round(float(np.percentile(step_ms, 50)), 4),
                p99_step_ms=round(float(np.percentile(step_ms, 99)), 4),
                mean_step_ms=round(float(step_ms.mean()), 4), schedule=schedule, device_errors=int(n_bad),
                path=path, **extra)


def serve_run(B, srv, reqs, arrivals):
    """Submit requests at their arrival times (seconds from start; None = all at once) while polling
    completions.  Returns (per-request latency ms = submit lag + library-measured latency, wall s)."""
    import numpy as np
    n = len(reqs)
    lat = np.zeros(n)
    pending = {}
    t0 = time.perf_counter()
    k = 0
    while k < n or pending:
        now = time.perf_counter() - t0
        while k < n and (arrivals is None or arrivals[k] <= now):
            ids, upd, pairs = reqs[k]
            while True:
                try:
                    rid = srv.submit(ids, upd, pairs)
                    break
                except B.LoccError as e:   # queue full: poll and retry
                    if e.status != B.ERR_BUSY:
                        raise
                    time.sleep(50e-6)
            lag = (time.perf_counter() - t0) - (arrivals[k] if arrivals is not None else 0.0)
            pending[rid] = (k, lag * 1e3)
            k += 1
            now = time.perf_counter() - t0
        # poll the oldest requests first, up to 64 unfinished ones a pass (completions are roughly in
        # submission order; the library stamps each completion itself, so the latency does not depend
        # on when it is polled)
        done, misses = [], 0
        for rid, (j, lag) in pending.items():
            r = srv.poll(rid)
            if r is not None:
                lat[j] = lag + r[2]
                done.append(rid)
            else:
                misses += 1
                if misses == 64:
                    break
        for rid in done:
            del pending[rid]
    return lat, time.perf_counter() - t0


def serve_bench(args, w):
    """Serving workload: Poisson stream of simulation-step requests over resident environments."""
    import numpy as np
    from paper_2304_09439_amd import binding as B
    from paper_2304_09439_amd import inputs as I
    rs = I.request_stream(n_requests=args.serve_requests)
    table = B.pack_objects(rs.pos0, rs.quat0, rs.shape)
    reqs = [(ids, B.pack_objects(pos, quat, rs.shape[ids]), np.ascontiguousarray(pairs))
            for ids, pos, quat, pairs in rs.requests]
    pp = rs.pairs_per_request
    total = int(pp.sum())
    print(f"[bench] serving: {len(reqs)} requests, mean {pp.mean():.1f} pairs, {len(rs.shape)} resident objects",
          file=sys.stderr, flush=True)
    wd = envs_widths()
    max_upd = max(len(r[0]) for r in reqs)

    def server(precision, batching):
        ctx = B.Context(128, wd, precision=precision)
        ctx.upload_shapes(rs.lib.offsets, rs.lib.pts)
        ctx.upload_weights(w)
        return ctx, B.Server(ctx, table, batching=batching, slots=3, max_batch_pairs=32768,
                             max_batch_updates=max(max_upd, 65536), hbm_budget_bytes=8 << 30)

    def summary(lat, wall):
        return dict(p50_latency_ms=round(float(np.percentile(lat, 50)), 4),
                    p99_latency_ms=round(float(np.percentile(lat, 99)), 4),
                    throughput=round(total / wall, 1), unit=UNIT, wall_s=round(wall, 3))

    out = dict(workload=f"{len(reqs)} requests, pairs per request log-uniform in [8, 2000] (mean {pp.mean():.1f}), "
                        f"128 shapes x 4096 points, {len(rs.shape)} resident objects in 4096 environments")
    # saturation of the plain FP32 per-request path sets the offered load
    ctx, srv = server("fp32", False)
    serve_run(B, srv, reqs[:200], None)                      # warm-up
    lat, wall = serve_run(B, srv, reqs, None)
    sat_fp32 = total / wall
    srv.stop()
    ctx.close()
    rate = 0.7 * sat_fp32 / pp.mean()
    arrivals = np.cumsum(np.random.default_rng(44).exponential(1.0 / rate, len(reqs)))
    out["offered_load"] = dict(requests_per_s=round(rate, 1), fraction_of_fp32_saturation=0.7,
                               fp32_per_request_saturated=round(sat_fp32, 1))
    for name, precision, batching in (("fp32_per_request", "fp32", False), ("bf16_batched", "bf16", True)):
        ctx, srv = server(precision, batching)
        serve_run(B, srv, reqs[:200], None)
        lat, wall = serve_run(B, srv, reqs, arrivals)
        st = srv.stats()
        srv.stop()
        res = summary(lat, wall)
        res["batches"] = int(st["batches"])
        out[name] = res
        ctx.close()
    ctx, srv = server("bf16", True)
    serve_run(B, srv, reqs[:200], None)
    st0 = srv.stats()
    lat, wall = serve_run(B, srv, reqs, None)
    st = srv.stats()
    sat = summary(lat, wall)
    busy = st["busy_ms"] - st0["busy_ms"]
    nb = int(st["batches"] - st0["batches"])
    sat.update(batches=nb, requests_per_batch=round(len(reqs) / max(nb, 1), 2), server_busy_ms=round(busy, 3),
               note="requests reach the queue at the rate of the Python submit loop (one ctypes call each), and the "
                    "worker takes whatever is queued as soon as a slot frees, so batches stay small and this "
                    "throughput is bounded by the submit loop, not by the server")
    out["bf16_batched_saturated_submit_loop"] = sat
    out["bf16_batched_saturated"] = serve_capacity(B, srv, reqs, total)
    srv.stop()
    ctx.close()
    return out


def serve_capacity(B, srv, reqs, total):
    """The server's own saturated rate: every request queued by one locc_serve_submit_many call (the flat
    arrays built beforehand), then the wait until the server reports all of them completed.  Latencies
    are the library's (completion minus submission on its clock), one per request."""
    import numpy as np
    arrays = B.Server.pack_requests(reqs)
    st0 = srv.stats()
    t0 = time.perf_counter()
    ids = srv.submit_many_arrays(*arrays)
    t_sub = time.perf_counter() - t0
    n = len(ids)
    while srv.stats()["completed"] - st0["completed"] < n:
        time.sleep(100e-6)
    wall = time.perf_counter() - t0
    st = srv.stats()
    lat = np.array([srv.poll(rid)[2] for rid in ids])
    nb = int(st["batches"] - st0["batches"])
    return dict(throughput=round(total / wall, 1), unit=UNIT, wall_s=round(wall, 4), submit_call_ms=round(1e3 * t_sub, 3),
                p50_latency_ms=round(float(np.percentile(lat, 50)), 4),
                p99_latency_ms=round(float(np.percentile(lat, 99)), 4), latency_samples=int(len(lat)),
                batches=nb, requests_per_batch=round(n / max(nb, 1), 2),
                server_busy_ms=round(st["busy_ms"] - st0["busy_ms"], 3),
                note="all requests queued by one submit_many call, so the rate is the server's (batch formation, "
                     "staging copies, three slots of detect launches, result copies); a request's latency is its "
                     "time in the queue plus its batch")


def voxel_pair_flops():
    """Algorithmic FLOPs per pair of the voxel variant's predictor: the per-object MLP 28-128-128-128 on
    both objects and the pair MLP 128-128-128-128 plus the 128 -> 1 output (cell tests and means are
    float64 compares and float32 adds, not counted)."""
    per_object = 2 * (28 * 128 + 128 * 128 + 128 * 128)
    return 2 * per_object + 2 * (3 * 128 * 128 + 128)


def time_voxel(args, scene):
    """The voxel-embedding variant on the same pairs: shape embeddings computed at upload, then the
    per-pair kernel (logit and probability; counts not requested), timed with events on its stream."""
    import numpy as np
    import torch
    from paper_2304_09439_amd import binding as B
    from paper_2304_09439_amd import inputs as I
    ctx = B.VoxelContext()
    ctx.upload_weights(I.flatten_weights(I.voxel_weights(seed=0)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.upload_shapes(scene.lib.offsets, scene.lib.pts)   # synchronous: host copy + encoder kernels
    encode_ms = 1000.0 * (time.perf_counter() - t0)
    objs, pairs = B.scene_tensors(scene)
    P = scene.n_pairs
    out = torch.empty((P, 2), dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        ctx.detect(objs, pairs, out, want_counts=False)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        ctx.detect(objs, pairs, out, want_counts=False)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([a.elapsed_time(b) for a, b in ev])
    n_bad = ctx.device_errors()
    ctx.close()
    avg = float(step_ms.mean())
    achieved = voxel_pair_flops() * P / (avg * 1e-3) / 1e12
    ms = 1000.0 * wall / args.steps
    return dict(value=round(P / (ms * 1e-3), 1), unit=UNIT, ms_per_step=round(ms, 4),
                p50_step_ms=round(float(np.percentile(step_ms, 50)), 4),
                max_step_ms=round(float(step_ms.max()), 4), step_samples=int(len(step_ms)),
                kernel=dict(name="voxel select + mlp kernels (one step)", avg_ms=round(avg, 4), bound="alu",
                            achieved=round(achieved, 2), peak=PEAK_TFLOPS["fp32"], unit="TFLOP/s",
                            frac=round(achieved / PEAK_TFLOPS["fp32"], 4), flops_per_pair=voxel_pair_flops()),
                shape_encoder_ms=round(encode_ms, 2), device_errors=int(n_bad),
                path="voxel-embedding variant: per-shape embeddings at upload (point MLP, 6^3 cell max, 3D U-Net, "
                     "F=16); per pair a selection kernel (one wave per pair: float64 cell tests, mean embeddings) "
                     "and an MLP kernel (float32 MFMA, 32 pairs per workgroup, pair max, sigmoid)")


def pose_grad_flops(widths):
    """FLOPs per pair of the gradient kernels: the head forward recomputed and its backward to the second
    object's pooled features (2 (2 h2 hh + hh^2 + hh^2 + hh h2)), and the encoder backward at the argmax
    rows (2 h2 channels x h1 units x 12: layer-1 pre-activation and the W1^T product)."""
    h1, h2, hh = widths.h1, widths.h2, widths.hh
    return 2 * (2 * h2 * hh + hh * hh + hh * hh + hh * h2) + 2 * h2 * h1 * 12


def time_pose_grad(args, scene, K, widths, w, precision="fp32"):
    """d logit / d (p, q) of both objects of every pair: crop, encoder with argmax rows (FP32, or the BF16
    split-schedule encoder in a BF16 context), head backward, encoder backward at the argmax rows and the
    float64 chain to the poses."""
    import numpy as np
    import torch
    from paper_2304_09439_amd import binding as B
    wd = (widths.h1, widths.h2, widths.hh)
    ctx = B.context_for_scene(scene, K, wd, w, precision=precision)
    objs, pairs = B.scene_tensors(scene)
    P = scene.n_pairs
    grad = torch.empty((P, 14), dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        ctx.pose_gradients(objs, pairs, grad)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    wall, step_ms, kt, _ = timed_then_profiled(ctx, lambda: ctx.pose_gradients(objs, pairs, grad), args.steps,
                                               stream)
    n_bad = ctx.device_errors()
    ctx.close()
    kernels = {name: dict(avg_ms=round(tot / max(n, 1), 4), launches=int(n)) for name, (n, tot) in sorted(kt.items())}
    g = kernels.get("pose_grad")
    if g:
        achieved = pose_grad_flops(widths) * P / (g["avg_ms"] * 1e-3) / 1e12
        g.update(bound="alu", achieved=round(achieved, 2), peak=PEAK_TFLOPS["fp32"], unit="TFLOP/s",
                 frac=round(achieved / PEAK_TFLOPS["fp32"], 4), flops_per_pair=pose_grad_flops(widths))
    ms = 1000.0 * wall / args.steps
    return dict(value=round(P / (ms * 1e-3), 1), unit="pair-gradients/s", ms_per_step=round(ms, 4),
                p50_step_ms=round(float(np.percentile(step_ms, 50)), 4),
                max_step_ms=round(float(step_ms.max()), 4), step_samples=int(len(step_ms)), kernels=kernels,
                device_errors=int(n_bad),
                path=("FP32: crop (with index sets), encoder recording argmax rows, head backward (32 pairs per "
                      "workgroup), encoder backward at the argmax rows and float64 chain to the poses")
                if precision == "fp32" else
                ("BF16 context: crop (float32 and bf16 rows, index sets), the BF16 split-schedule encoder recording "
                 "argmax rows and pooled features, then the FP32 path's head backward, encoder backward at the "
                 "argmax rows and float64 chain to the poses"))


def train_flops(widths):
    """FLOPs per pair of the training kernels (the crop and the forward encoder are timed apart): the
    head forward and backward (u1, u2, du1, dz), the head weight gradients (dH3[0], dH2, dH1) and the
    encoder weight gradients at the argmax rows of both objects (14 multiply-adds per hidden unit)."""
    h1, h2, hh = widths.h1, widths.h2, widths.hh
    head = 2 * (2 * h2 * hh + hh * hh + hh * hh + hh * 2 * h2)
    wgrad = 2 * (hh + hh * hh + hh * 2 * h2)
    enc = 2 * (2 * h2 * h1 * 14)
    return head + wgrad + enc


def time_train(args):
    """Training throughput of the FP32 network (64-128 / 256-256-256, K = 64) on 4096 labelled sphere
    pairs per step: crop, encoder with argmax rows, then the training kernels (loss, gradients, Adam,
    repacking)."""
    import numpy as np
    import torch
    from paper_2304_09439_amd import binding as B
    from paper_2304_09439_amd import inputs as I
    wd = I.Widths(64, 128, 256)
    sc, y = I.sphere_training_set(n_pairs=4096)
    ctx = B.context_for_scene(sc, 64, (wd.h1, wd.h2, wd.hh), I.flatten_weights(I.gaussian_weights(wd, seed=1)),
                              precision="fp32")
    objs, pairs = B.scene_tensors(sc)
    lab = torch.from_numpy(y).cuda()
    loss = torch.empty(2, dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        ctx.train_step(objs, pairs, lab, loss=loss)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    wall, step_ms, kt, _ = timed_then_profiled(ctx, lambda: ctx.train_step(objs, pairs, lab, loss=loss), args.steps,
                                               stream)
    last = loss.cpu().numpy().tolist()
    ctx.close()
    kernels = {name: dict(avg_ms=round(tot / max(n, 1), 4), launches=int(n)) for name, (n, tot) in sorted(kt.items())}
    P = sc.n_pairs
    t = kernels.get("train")
    if t:
        achieved = train_flops(wd) * P / (t["avg_ms"] * 1e-3) / 1e12
        t.update(bound="alu", achieved=round(achieved, 2), peak=PEAK_TFLOPS["fp32"], unit="TFLOP/s",
                 frac=round(achieved / PEAK_TFLOPS["fp32"], 4), flops_per_pair=train_flops(wd))
    ms = 1000.0 * wall / args.steps
    return dict(value=round(P / (ms * 1e-3), 1), unit="training pairs/s", batch=P, ms_per_step=round(ms, 4),
                p50_step_ms=round(float(np.percentile(step_ms, 50)), 4), kernels=kernels,
                loss_after=last, path="FP32 training step: crop, encoder with argmax rows, head forward/backward "
                                      "on matrix cores, fixed-order weight-gradient reductions, Adam, repacking")


def timed_then_profiled(ctx, step, steps, stream):
    """steps calls of step() timed (wall clock and per-step events, no per-kernel events), then as many again
    with the library's per-kernel events for the kernel durations.  Returns (wall s, step ms array, kernel
    totals, wall s of the profiled run)."""
    import numpy as np
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        step()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.profile(True)
    t1 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall_prof = time.perf_counter() - t1
    ctx.profile(False)
    return wall, np.array([a.elapsed_time(b) for a, b in ev]), ctx.profile_read(), wall_prof


def envs_widths():
    from paper_2304_09439_amd import inputs as I
    wd = I.SCALE_WIDTHS
    return (wd.h1, wd.h2, wd.hh)


def run(args):
    from paper_2304_09439_amd import inputs as I

    W = workload(args.workload)
    scene, K, widths = W["scene"], W["K"], W["widths"]
    w = I.flatten_weights(I.gaussian_weights(widths, seed=0))
    cpu = None
    if not args.no_cpu_baseline:
        small = None
        if args.workload == "scale":
            S = workload("small")
            small = (S["scene"], I.flatten_weights(I.gaussian_weights(S["widths"], seed=0)), S["widths"], S["K"])
        cpu = cpu_baseline(scene, w, widths, K, args.cpu_pairs, small=small)   # before the GPU is touched

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    work = per_pair_work(K, widths, W["n_points"])
    precisions = args.precision.split(",")
    paths = {p: time_path(args, scene, K, widths, w, p, work, args.workload) for p in precisions}
    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)   # one elementwise kernel: copy_mib read + copy_mib written
        torch.cuda.synchronize()

    primary = "bf16" if "bf16" in paths else precisions[0]
    main_path = paths[primary]
    kernels = main_path["kernels"]
    dominant = max(kernels, key=lambda k: kernels[k]["avg_ms"])
    d = kernels[dominant]
    roofline = dict(kernel=dominant, bound=d["bound"], achieved=d["achieved"], peak=d["peak"], unit=d["unit"],
                    frac=d["frac"], traffic=d["traffic"])
    for k in ("flops_basis", "fixed_2K_frac", "tiles_run_frac"):
        if k in d:
            roofline[k] = d[k]
    line = dict(
        metric=METRIC, value=main_path["value"], unit=UNIT, n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=main_path["ms_per_step"], higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32" if primary == "fp32" else primary, data="synthetic",
        config=dict(workload=W["desc"], pairs=scene.n_pairs, K=K, points_per_shape=W["n_points"],
                    outputs="contacts (logit, point, normal, depth)" + (" and member counts" if args.member_counts
                                                                        else "; member counts not requested"),
                    shapes=W["n_shapes"], precision=primary, geometry="f64", path=main_path["path"]),
        p50_step_ms=main_path["p50_step_ms"], p99_step_ms=main_path["p99_step_ms"],
        roofline=roofline, kernels=kernels, cpu_baseline=cpu, device_errors=main_path["device_errors"],
        paths={p: {k: v for k, v in r.items()} for p, r in paths.items()},
    )
    if "fp32" in paths and primary != "fp32":
        line["speedup_vs_fp32_plain"] = round(main_path["value"] / paths["fp32"]["value"], 3)
    if not args.no_voxel:
        line["voxel_variant"] = time_voxel(args, scene)
    if not args.no_pose_grad:
        line["pose_gradients"] = time_pose_grad(args, scene, K, widths, w)
        line["pose_gradients"]["bf16"] = time_pose_grad(args, scene, K, widths, w, precision="bf16")
    if not args.no_train:
        line["training"] = time_train(args)
    if args.serve_requests > 0:
        line["serving"] = serve_bench(args, w)
    if args.env_steps > 0:
        envs = I.env_workload(steps=args.env_steps)
        print(f"[bench] uneven environments: {len(envs.shape)} objects, "
              f"{sum(len(p) for p in envs.pairs) / envs.n_steps:.0f} pairs per step", file=sys.stderr, flush=True)
        line["environments"] = dict(
            workload=f"4096 environments, 1-40 objects each ({len(envs.shape)} objects) from the 32-shape library, "
                     f"cube side {envs.side:.3f} m, {args.env_steps} jittered steps; pairs from a host broad "
                     f"phase ahead of time, or from the library's broad phase inside the step",
            **{p: time_envs(args, envs, w, p) for p in precisions if p in ("fp32", "bf16")})
        if "bf16" in precisions:
            line["environments"]["bf16_gpu_broad_phase"] = time_envs(args, envs, w, "bf16", gpu_broad=True)
    print(json.dumps(line), flush=True)


# ------------------------------------------------------------------ counters

def _counter_means(directory):
    """{kernel name: mean counter value per dispatch} from rocprofv3 counter CSV files."""
    import csv
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {directory}")
    acc = {}
    for f in files:
        with open(f) as fh:
            for row in csv.DictReader(fh):
                name = row.get("Kernel_Name") or row.get("Kernel-Name") or ""
                val = float(row.get("Counter_Value") or row.get("Counter-Value") or 0.0)
                disp = row.get("Dispatch_Id") or row.get("Dispatch-Id") or str(len(acc))
                acc.setdefault(name, {}).setdefault(disp, 0.0)
                acc[name][disp] += val
    return {k: sum(v.values()) / len(v) for k, v in acc.items()}


N_SIMD = 1024          # 256 compute units x 4 SIMDs
CLOCK_GHZ = 2.4        # published peak engine clock


def _sq_means(directory, needle):
    """(kernel name, {counter: mean per dispatch}, mean dispatch duration ns or None) of the dispatches whose
    kernel name contains needle, from rocprofv3 counter CSV files."""
    import csv
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {directory}")
    acc, dur, name_seen = {}, {}, None
    for f in files:
        with open(f) as fh:
            for row in csv.DictReader(fh):
                name = row.get("Kernel_Name") or ""
                if needle not in name:
                    continue
                name_seen = name
                disp = row.get("Dispatch_Id") or str(len(dur))
                acc.setdefault(row["Counter_Name"], {}).setdefault(disp, 0.0)
                acc[row["Counter_Name"]][disp] += float(row["Counter_Value"])
                t0, t1 = row.get("Start_Timestamp"), row.get("End_Timestamp")
                if t0 and t1:
                    dur[disp] = float(t1) - float(t0)
    if not acc:
        raise SystemExit(f"no dispatch of a kernel matching {needle!r} under {directory}")
    means = {c: sum(v.values()) / len(v) for c, v in acc.items()}
    n = max(len(v) for v in acc.values())
    return name_seen, means, (sum(dur.values()) / len(dur) if dur else None), n


def summarize_sq(args):
    """SQ counters of one kernel from one or more rocprofv3 --pmc runs (one pass each), as means per dispatch,
    with the derived vector-issue bound and matrix-core busy fraction."""
    merged, name, dur, n = {}, None, None, 0
    for d in args.summarize_sq:
        nm, means, du, nd = _sq_means(d, args.kernel_match)
        name = name or nm
        dur = dur or du
        n = max(n, nd)
        merged.update(means)
    print(f"kernel {args.kernel} ({name})")
    print(f"source_sha256 {source_hash(args.kernel)}")
    print(f"dispatches {n}")
    if dur:
        print(f"duration_ns_mean {dur:.0f}")
    for c in sorted(merged):
        print(f"{c} {merged[c]:.0f}")
    if "SQ_INSTS_VALU" in merged:
        # every wave64 vector instruction occupies its SIMD's vector unit for at least 4 cycles
        print(f"valu_issue_bound_ns {merged['SQ_INSTS_VALU'] * 4 / (N_SIMD * CLOCK_GHZ):.0f}")
    if "SQ_INSTS_VALU" in merged and "SQ_INSTS_MFMA" in merged and merged["SQ_INSTS_MFMA"] > 0:
        print(f"valu_per_mfma {merged['SQ_INSTS_VALU'] / merged['SQ_INSTS_MFMA']:.2f}")
    if dur and "SQ_VALU_MFMA_BUSY_CYCLES" in merged:
        print(f"mfma_busy_frac {merged['SQ_VALU_MFMA_BUSY_CYCLES'] / (N_SIMD * CLOCK_GHZ * dur):.3f}")
    if "SQ_WAIT_ANY" in merged and "SQ_WAVE_CYCLES" in merged:
        print(f"wait_any_frac {merged['SQ_WAIT_ANY'] / merged['SQ_WAVE_CYCLES']:.3f}")


def counter_value(kernel: str, workload_name: str, kind: str, key: str):
    """A value from a committed counter summary (profiles/<kernel>_<workload>_<kind>_counters.txt), if it was
    taken on this kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload_name}_{kind}_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) >= 2 and not line.startswith("#"):
                vals[parts[0]] = parts[1]
    if vals.get("source_sha256") != source_hash(kernel) or key not in vals:
        return None
    return float(vals[key])


def summarize_counters(args):
    fetch = _counter_means(args.summarize_counters[0])
    write = _counter_means(args.summarize_counters[1])

    def pick(table, needle):
        hits = [(k, v) for k, v in table.items() if needle in k]
        if not hits:
            raise SystemExit(f"no kernel matching {needle!r}; kernels: {list(table)}")
        return max(hits, key=lambda kv: kv[1])

    copy_bytes = args.copy_mib * (1 << 20)
    ck, cf = pick(fetch, args.copy_kernel)
    _, cw = pick(write, args.copy_kernel)
    f_scale = copy_bytes / (cf * 1024.0)   # counters are KiB per dispatch
    w_scale = copy_bytes / (cw * 1024.0)
    kk, kf = pick(fetch, args.kernel_match)
    _, kw = pick(write, args.kernel_match)
    fetch_b = kf * 1024.0 * f_scale
    write_b = kw * 1024.0 * w_scale
    print(f"kernel {args.kernel} ({kk})")
    print(f"source_sha256 {source_hash(args.kernel)}")
    short = ck.split("(")[0].split("<")[0].replace("void ", "")
    print(f"copy_kernel torch.neg ({short}) copy_bytes {copy_bytes}")
    print(f"fetch_scale {f_scale:.4f} write_scale {w_scale:.4f}")
    print(f"fetch_kib_per_dispatch {kf:.1f} write_kib_per_dispatch {kw:.1f}")
    print(f"hbm_bytes_per_launch {fetch_b + write_b:.0f}")
    print(f"hbm_fetch_bytes_per_launch {fetch_b:.0f} hbm_write_bytes_per_launch {write_b:.0f}")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="scale", choices=["scale", "small"])
    ap.add_argument("--schedule", action="append", default=[], metavar="PREC:WG,CLAIM,DYN,SPLIT,UNROLL,CHUNKS",
                    help="fix the schedule of a batched path instead of autotuning it, e.g. bf16:2,16,1,1,4,2 "
                         "(repeatable; used to profile the schedule a previous run picked)")
    ap.add_argument("--precision", default="fp32,bf16,fp8,fp8_encoder",
                    help="comma list of paths to time: fp32 (per-step), bf16 (batched, the headline), fp8 (batched)")
    ap.add_argument("--member-counts", action="store_true",
                    help="request the per-object member counts in the timed steps (full scans of both objects)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default schedule")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests of the serving workload (0 = skip)")
    ap.add_argument("--env-steps", type=int, default=200,
                    help="simulation steps of the uneven-environment workload to time (0 = skip)")
    ap.add_argument("--cpu-pairs", type=int, default=16384)
    ap.add_argument("--no-voxel", action="store_true", help="skip the voxel-embedding variant's leg")
    ap.add_argument("--no-pose-grad", action="store_true", help="skip the pose-gradient leg")
    ap.add_argument("--no-train", action="store_true", help="skip the training leg")
    ap.add_argument("--copy-mib", type=int, default=0, help="also run a plain device copy of this size")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-sq", nargs="+", metavar="DIR", help="summarise SQ counter passes of --kernel")
    ap.add_argument("--profile-run", action="store_true",
                    help="time only the warm-up and timed steps of each path (no latency samples, member-count "
                         "leg or schedule alternatives), for runs under a profiler")
    ap.add_argument("--kernel", default="encoder_fp32")
    ap.add_argument("--kernel-match", default="encoder_fp32_kernel")
    ap.add_argument("--copy-kernel", default="neg_kernel")
    args = ap.parse_args()
    sched = {}
    for item in args.schedule:
        prec, vals = item.split(":")
        wg, claim, dyn, split, unroll, chunks = (int(v) for v in vals.split(","))
        sched[prec] = dict(wg_per_cu=wg, claim=claim, dynamic=bool(dyn), split=bool(split), crop_unroll=unroll,
                           chunks=chunks)
    args.schedule = sched
    if args.summarize_counters:
        return summarize_counters(args)
    if args.summarize_sq:
        return summarize_sq(args)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the LOCC path has no "
              f"multi-GPU mode in this build", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only; launch it without a multi-rank launcher", file=sys.stderr)
        sys.exit(2)
    run(args)


if __name__ == "__main__":
    main()

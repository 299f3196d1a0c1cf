#!/usr/bin/env python3
"""Benchmark of the MI355X SBR radio-map path (one GPU).

Headline workload ("large"): seeded fBm terrain (513 x 513 vertices over
2 x 2 km) plus 2,000 buildings with facades and roofs split into <= 4 m quads,
1,021,074 triangles of concrete, glass and metal; isotropic V-pol transmitter
40 m above the terrain at the origin, f = 3.5 GHz, N_S = 1e8 rays, max depth
L = 8, 1000 x 1000 cells of 2 m at z = 1.5 m.

One timed step = one rt_radio_map call: zero the map, launch every ray, trace
all its segments through the LBVH, reflect, deposit.  The metric is traced
segments ("ray-bounces", one closest-hit query each) per second, counted on
the device.  Inputs are resident in HBM before timing starts.

Before timing, rt_tune picks the launch configuration (tree width, launch
order, workgroup size, deposit strategy, refill threshold) on a spread sample
of the same lattice; its time is reported separately.

Printed: one JSON line with the metric, a roofline object for the forward
kernel, and the FP64 oracle timed on a strided sample of the same lattice on
the host cores.  Roofline: the forward kernel issues VALU instructions on
about 92 % of its cycles and moves about 2 % of the HBM peak (the 326 MB of
tree, triangles and normals are served from the vector L1 caches, the L2
and the 256 MB MALL), so it is reported against the VALU issue rate (256
CUs x 64 lanes x 2.4 GHz = 39.3 T FP32 lane-operations/s) with an
algorithmic operation count per segment (see
ALU_OPS below); the algorithmic HBM byte model and the measured DRAM bytes
are reported beside it ("hbm_model").  Side legs: the Manhattan city (1e7
rays, L = 5), differentiation and batching ratios, transmit arrays, slab
walls with refraction, diffuse reflection, Russian roulette, 64 rooftop
transmitters on both scenes, and the time per map against N_S (up to 1e9)
and the number of transmit antennas (up to 512).
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SBR radio map M ray-bounces/s; fwd+bwd/fwd and batched vs plain at 1e-3 tol"
HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one FP32 lane-op each
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic FP32 operations per unit of work (the arithmetic the method needs,
# one op per add/mul/fma/min/max/compare):
#   slab test of one child box against a ray with precomputed inverse
#     direction: 6 fma + 3 min + 3 max + 2 combine + 1 compare = 15
#   watertight triangle test: 9 sub + 6 shear + 9 (U,V,W) + 3 scale + 5 (T) +
#     1 div + 6 sign/range tests + 6 = 45
#   per segment: ray set-up, plane crossing and weight, bounce (basis,
#     Fresnel with complex sqrt and divisions, 2x2 complex update) = 250
ALU_OPS = {"child_box": 15, "tri": 45, "segment": 250}
# Algorithmic bytes (HBM byte model): per binary node visit 2 child boxes +
# 2 refs = 56 B (a 4-wide node: 4 boxes + 4 refs = 112 B), per triangle test
# 3 vertices + id = 40 B, per deposit a 4 B read-modify-write = 8 B
NODE_BYTES = {2: 56, 4: 112}
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "forward_manhattan_counters.json")
PROFILE_COUNTERS_LARGE = os.path.join(ROOT, "profiles", "forward_large_counters.json")
KERNEL_SOURCES = ["paper_2504_21719_amd/csrc/sbr_forward.hip", "paper_2504_21719_amd/csrc/sbr_common.h",
                  "paper_2504_21719_amd/csrc/rt_device.h"]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="wall time budget of the oracle sample")
    ap.add_argument("--cpu-workers", type=int, default=0, help="oracle processes (default: min(16, host cores))")
    ap.add_argument("--no-extras", action="store_true", help="skip the fwd+bwd and batched ratio legs")
    ap.add_argument("--no-manhattan", action="store_true", help="skip the Manhattan legs")
    ap.add_argument("--no-tune", action="store_true", help="use the untuned launch defaults")
    ap.add_argument("--launch", default="", help="width,order,block,deposit,refill: apply to the headline "
                                                 "workload instead of tuning")
    ap.add_argument("--calib-copy", action="store_true", help="also run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--profile-steps", type=int, default=0, help="only run N forward steps (for rocprofv3)")
    ap.add_argument("--profile-large", type=int, default=0,
                    help="only run N forward steps of the 1 M-triangle workload (for rocprofv3)")
    ap.add_argument("--profile-legs", type=int, default=0,
                    help="only run N repetitions of the adjoint and batched legs (for rocprofv3)")
    ap.add_argument("--large-counters", action="store_true",
                    help="with --ingest-counters: the CSVs are of a --profile-large run")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn rocprofv3 FETCH_SIZE / WRITE_SIZE counter CSVs of a --profile-steps --calib-copy "
                         "run into the per-launch traffic record, then exit")
    ap.add_argument("--trace-summary", metavar="KERNEL_TRACE_CSV",
                    help="average duration of the headline's forward dispatches in a rocprofv3 kernel trace of "
                         "a run with --no-extras --no-manhattan --no-cpu-baseline and the same --steps, then exit")
    return ap.parse_args()


CALIB_COPY_BYTES = (64 << 20) * 4


def ingest_counters(fetch_csv, write_csv, large=False):
    """Per-launch HBM traffic of the forward kernel from two counter runs.

    Each run holds the forward dispatches and three plain device copies of
    CALIB_COPY_BYTES; a counter's scale factor is the copy's true byte count
    over what the counter reports for it."""
    import csv
    out = {"kernel_source_sha": kernel_source_sha(), "kernel": "k_forward (single transmitter, 4-wide tree)",
           "workload": "large: 1,021,074 triangles, 1e8 rays, L = 8" if large else "manhattan, 1e7 rays, L = 5"}
    for path, counter, key in ((fetch_csv, "FETCH_SIZE", "fetch"), (write_csv, "WRITE_SIZE", "write")):
        with open(path) as f:
            rows = [r for r in csv.DictReader(f) if r["Counter_Name"] == counter]
        fwd = [float(r["Counter_Value"]) for r in rows if "k_forward<false, 0" in r["Kernel_Name"]]
        copies = sorted((int(r["Grid_Size"]), float(r["Counter_Value"])) for r in rows
                        if "copyBuffer" in r["Kernel_Name"])[-3:]
        if not fwd or len(copies) < 3:
            raise SystemExit("%s: no forward dispatches or calibration copies" % path)
        copy_kib = sum(v for _, v in copies) / 3
        factor = CALIB_COPY_BYTES / 1024.0 / copy_kib
        kib = sum(fwd) / len(fwd)
        out[key + "_kib_raw"] = round(kib, 3)
        out[key + "_copy_kib_raw"] = round(copy_kib, 3)
        out[key + "_factor"] = round(factor, 4)
        out[key + "_bytes_per_launch"] = int(round(kib * 1024 * factor))
        out[key + "_dispatches"] = len(fwd)
    out["calibration_factor"] = {"fetch": out["fetch_factor"], "write": out["write_factor"]}
    with open(PROFILE_COUNTERS_LARGE if large else PROFILE_COUNTERS, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def trace_summary(path, steps):
    """Durations of the forward dispatches of the headline's timed steps.

    In a run with --no-extras --no-manhattan --no-cpu-baseline the last
    2 * steps forward dispatches are the timed steps followed by the
    kernel-only timing (accumulate = 1); earlier ones are the autotuner's
    candidates, the counting pass and the warm-up."""
    import csv
    with open(path) as f:
        rows = [r for r in csv.DictReader(f) if "k_forward<false, 0, true, false>" in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    if len(rows) < 2 * steps:
        raise SystemExit("%s: %d forward dispatches, fewer than 2 x %d" % (path, len(rows), steps))
    out = {"kernel": "k_forward<false, MODE_SINGLE, wide, not extended>", "dispatches": len(rows)}
    for name, sel in (("timed_steps", rows[-2 * steps:-steps]), ("kernel_only", rows[-steps:])):
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in sel]
        r0 = sel[0]
        out[name] = {"n": len(d), "avg_us": round(sum(d) / len(d), 1), "min_us": round(min(d), 1),
                     "max_us": round(max(d), 1), "grid": int(r0.get("Grid_Size_X", r0.get("Grid_Size", 0))),
                     "workgroup": int(r0.get("Workgroup_Size_X", r0.get("Workgroup_Size", 0)))}
    print(json.dumps(out))
    return out


_T0 = time.perf_counter()


def _progress(msg):
    """One line on stderr per finished leg (the JSON result goes to stdout)."""
    print("[bench %6.1f s] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.trace_summary:
        trace_summary(args.trace_summary, args.steps)
        return
    if args.ingest_counters:
        ingest_counters(*args.ingest_counters, large=args.large_counters)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the map would be "
              "all-reduced over RCCL after tracing disjoint ray ranges).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2504_21719_amd as rt
    import scenegen as sg

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.profile_large:
        lc = sg.large_config()
        ls = rt.scene_from_mesh(lc.scene)
        le = torch.tensor(lc.scene.eps_r, dtype=torch.float32, device=dev)
        lg = torch.tensor(lc.scene.sigma, dtype=torch.float32, device=dev)
        lo = torch.empty((1, lc.plane.H, lc.plane.W), dtype=torch.float32, device=dev)
        if args.launch:
            rt.rt_set_launch_config(ls, *[int(x) for x in args.launch.split(",")])
        else:
            rt.rt_tune(ls, le, lg, lc.tx, lc.plane, lc.params, 4_000_000, lo)
        for _ in range(args.profile_large):
            rt.rt_radio_map(ls, le, lg, lc.tx, lc.plane, lc.params, lo)
        if args.calib_copy:
            a = torch.empty(CALIB_COPY_BYTES // 4, dtype=torch.float32, device=dev)
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
        torch.cuda.synchronize()
        inf = ls.info()
        print(json.dumps({"profile_large": args.profile_large, "launch": "%d,%d,%d,%d,%d" % (
            inf.tuned_width, inf.tuned_order, inf.tuned_block, inf.tuned_deposit, inf.tuned_refill)}))
        return
    if args.profile_legs:
        profile_legs(rt, sg, dev, args.profile_legs)
        return
    if args.profile_steps:
        # Manhattan forward steps only (for rocprofv3)
        cfg = sg.manhattan_config()
        scene, eps, sig, out, _ = setup_plain(rt, cfg, dev, args.launch, args.no_tune, 2_000_000)
        for _ in range(args.profile_steps):
            rt.rt_radio_map(scene, eps, sig, cfg.tx, cfg.plane, cfg.params, out)
        if args.calib_copy:
            a = torch.empty(CALIB_COPY_BYTES // 4, dtype=torch.float32, device=dev)
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps,
                          "calib_copy_bytes": CALIB_COPY_BYTES if args.calib_copy else 0}))
        return

    # ---- headline: the 1.02 M-triangle scene
    lc = sg.large_config()
    scene, eps, sig, out, tune_s = setup_plain(rt, lc, dev, args.launch, args.no_tune, 4_000_000)
    info = scene.info()
    width = info.tuned_width or 4
    n_seg, n_cross, n_node, n_tri = device_counts(rt, scene, eps, sig, lc, out)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        rt.rt_radio_map(scene, eps, sig, lc.tx, lc.plane, lc.params, out)
    torch.cuda.synchronize()
    # timed region: exactly `steps` steps, synchronised on both sides
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        rt.rt_radio_map(scene, eps, sig, lc.tx, lc.plane, lc.params, out)
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [s.elapsed_time(e) for s, e in ev]
    ms_per_step = wall * 1e3 / args.steps
    value = n_seg / (ms_per_step * 1e-3) / 1e6
    kern_ms = kernel_ms(rt, scene, eps, sig, lc, out, stream, args.steps)
    tr = traffic_from_profile(PROFILE_COUNTERS_LARGE)
    roof = rooflines(n_seg, n_cross, n_node, n_tri, width, kern_ms, tr,
                     note="tree + triangles about %d MB: larger than the L2 caches, partly held in the 256 MB MALL"
                     % (info.device_bytes >> 20))
    if tr:
        # bytes that crossed to DRAM per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE), against the HBM peak
        mb = tr["fetch_bytes"] + tr["write_bytes"]
        roof["hbm_model"]["measured_traffic"] = {"bytes_per_launch": mb,
                                                 "GB/s": round(mb / (kern_ms * 1e-3) / 1e9, 1),
                                                 "frac": round(mb / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                                 "source": tr["source"]}
    result = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "M ray-bounces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "large: seeded fBm terrain + 2,000 subdivided buildings, %s triangles (concrete, "
                               "glass, metal), iso V-pol Tx 40 m above the terrain at the origin, 3.5 GHz, 1e8 "
                               "Fibonacci rays, max depth 8, 1000x1000 cells of 2 m at z=1.5 m"
                               % format(lc.scene.n_triangles, ","),
                   "n_rays": lc.params.n_rays, "max_depth": lc.params.max_depth,
                   "n_triangles": lc.scene.n_triangles, "cells": [lc.plane.H, lc.plane.W],
                   "parallelism": "single GPU"},
        "segments_per_step": n_seg,
        "crossings_per_step": n_cross,
        "event_ms_per_step_median": round(float(np.median(step_ms)), 4),
        "build_ms": round(info.build_ms, 3),
        "bvh_depth": info.bvh_depth,
        "tuned": tuned_record(info, tune_s),
        "roofline": roof,
    }
    result["hbm_model"] = result["roofline"].pop("hbm_model")
    _progress("headline done: %.1f M ray-bounces/s, %.3f ms/step" % (value, ms_per_step))
    if not args.no_extras:
        try:
            result["large_extras"] = large_extras(rt, sg, lc, scene, eps, sig, dev, out)
        except rt.RtError as e:
            result["large_extras_error"] = str(e)
        _progress("large-scene extras done")
    del scene, out
    torch.cuda.empty_cache()

    # ---- side legs on the Manhattan city
    if not args.no_manhattan:
        cfg = sg.manhattan_config()
        try:
            mscene, meps, msig, mout, mtune = setup_plain(rt, cfg, dev, "", args.no_tune, 2_000_000)
            result["manhattan"] = manhattan_leg(rt, cfg, mscene, meps, msig, mout, mtune, dev)
            _progress("manhattan leg done")
            if not args.no_extras:
                result.update(extra_legs(rt, sg, cfg, mscene, meps, msig, dev))
                _progress("ratio legs done")
                result["array"] = array_leg(rt, sg, cfg, mscene, meps, msig, mout)
                _progress("array leg done")
                result["n_s_sweep"] = n_s_leg(rt, sg, cfg, mscene, meps, msig, mout)
                _progress("N_S sweep done")
                result["refraction"] = refraction_leg(rt, sg, cfg, dev, mout)
                _progress("refraction leg done")
                result["diffuse"] = diffuse_leg(rt, sg, cfg, mscene, meps, msig, dev, mout)
                _progress("diffuse leg done")
        except rt.RtError as e:
            result["manhattan_error"] = str(e)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(lc, args.cpu_seconds, args.cpu_workers)
        _progress("cpu baseline done")

    print(json.dumps(result), flush=True)


def profile_legs(rt, sg, dev, reps):
    """`reps` repetitions of each kernel the ratio legs run, for rocprofv3:
    forward with a tape plus the adjoint (differentiation workload), 64
    rooftop transmitters in one batched call on the Manhattan city and on the
    1.02 M-triangle scene, and 16 material samples forward + backward in one
    batched call (geometry pass + per-sample field pass)."""
    import numpy as np
    import torch
    cfg = sg.manhattan_config()
    scene, eps, sig, _, _ = setup_plain(rt, cfg, dev, "", False, 2_000_000)
    dc = sg.diff_config()
    H, W = dc.plane.H, dc.plane.W
    m = torch.empty((1, H, W), dtype=torch.float32, device=dev)
    tape = rt.rt_tape_create(dc.params)
    g = torch.randn((1, H, W), dtype=torch.float32, device=dev)
    ge, gs, go = (torch.empty(n, dtype=torch.float32, device=dev) for n in (2, 2, 3))
    for _ in range(reps):
        rt.rt_radio_map(scene, eps, sig, dc.tx, dc.plane, dc.params, m, tape=tape)
        rt.rt_radio_map_backward(scene, eps, sig, dc.tx, dc.plane, dc.params, tape, g, ge, gs, go)
    torch.cuda.synchronize()
    del tape
    _progress("adjoint leg done")
    txs, budgets = sg.rooftop_transmitters(64, seed=5, buildings=sg.manhattan_buildings(cfg.scene))
    maps = torch.empty((len(txs), 1, H, W), dtype=torch.float32, device=dev)
    for _ in range(reps):
        rt.rt_radio_map_batched(scene, eps[None], sig[None], txs, budgets, cfg.plane,
                                sg.Params(cfg.params.freq_hz, 1, 5), maps)
    torch.cuda.synchronize()
    _progress("batched transmitters (Manhattan) done")
    # the per-transmitter loop the batched call is compared with, once, in
    # budget order (the trace then pairs each call with its budget)
    for k in np.argsort(-np.asarray(budgets), kind="stable"):
        rt.rt_radio_map(scene, eps, sig, txs[k], cfg.plane, sg.Params(cfg.params.freq_hz, int(budgets[k]), 5),
                        maps[k])
    torch.cuda.synchronize()
    del maps
    _progress("per-transmitter loop (Manhattan) done")
    S = 16
    E, Sg = sg.random_materials(cfg.scene, S, seed=5)
    eS = torch.tensor(E, dtype=torch.float32, device=dev)
    sS = torch.tensor(Sg, dtype=torch.float32, device=dev)
    maps = torch.empty((1, S, H, W), dtype=torch.float32, device=dev)
    gm = torch.randn((1, S, H, W), dtype=torch.float32, device=dev)
    grads = torch.empty((1, S, 2 * cfg.scene.n_materials + 3), dtype=torch.float32, device=dev)
    for _ in range(reps):
        rt.rt_radio_map_batched(scene, eS, sS, [dc.tx], [1_000_000], dc.plane, sg.Params(cfg.params.freq_hz, 1, 5),
                                maps, grad_maps=gm, grads=grads)
    torch.cuda.synchronize()
    del maps, gm, scene
    torch.cuda.empty_cache()
    _progress("batched material samples done")
    lc = sg.large_config()
    ls, le, lg, _, _ = setup_plain(rt, lc, dev, "", False, 4_000_000)
    txs, budgets = sg.rooftop_transmitters(64, seed=5, buildings=sg.large_buildings())
    maps = torch.empty((len(txs), 1, lc.plane.H, lc.plane.W), dtype=torch.float32, device=dev)
    for _ in range(reps):
        rt.rt_radio_map_batched(ls, le[None], lg[None], txs, budgets, lc.plane, sg.Params(lc.params.freq_hz, 1, 5),
                                maps)
    torch.cuda.synchronize()
    _progress("batched transmitters (large scene) done")
    print(json.dumps({"profile_legs": reps, "large_batched_rays": int(np.sum(budgets))}))


def setup_plain(rt, cfg, dev, launch, no_tune, tune_rays):
    """Scene, materials and map of one workload, with the launch configuration
    applied (``launch`` = "width,order,block,deposit,refill") or tuned."""
    import torch
    scene = rt.scene_from_mesh(cfg.scene)
    eps = torch.tensor(cfg.scene.eps_r, dtype=torch.float32, device=dev)
    sig = torch.tensor(cfg.scene.sigma, dtype=torch.float32, device=dev)
    out = torch.empty((1, cfg.plane.H, cfg.plane.W), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if launch:
        rt.rt_set_launch_config(scene, *[int(x) for x in launch.split(",")])
    elif not no_tune:
        rt.rt_tune(scene, eps, sig, cfg.tx, cfg.plane, cfg.params, tune_rays, out)
    torch.cuda.synchronize()
    return scene, eps, sig, out, time.perf_counter() - t0


def device_counts(rt, scene, eps, sig, cfg, out):
    """Segments, crossings, node visits and triangle tests of one pass."""
    import numpy as np
    import torch
    stats = torch.zeros(8, dtype=torch.int64, device=out.device)
    rt.rt_radio_map(scene, eps, sig, cfg.tx, cfg.plane, cfg.params, out, stats=stats)
    torch.cuda.synchronize()
    st = stats.cpu().numpy().astype(np.int64)
    if st[4] != 0:
        raise SystemExit("traversal stack overflow or bad node reference reported by the forward kernel")
    return int(st[0]), int(st[1]), int(st[2]), int(st[3])


def tuned_record(info, tune_s):
    return {"width": info.tuned_width or 4, "order": "coherent" if info.tuned_order != 2 else "lattice",
            "block": info.tuned_block, "deposit": "wave" if info.tuned_deposit == 2 else "atomic",
            "refill": info.tuned_refill, "tune_s": round(tune_s, 3),
            "launch": "%d,%d,%d,%d,%d" % (info.tuned_width, info.tuned_order, info.tuned_block,
                                          info.tuned_deposit, info.tuned_refill)}


def manhattan_leg(rt, cfg, scene, eps, sig, out, tune_s, dev, reps=20):
    """The Manhattan city (10 x 10 blocks, 1,202 triangles, 1e7 rays, L = 5,
    1 m cells): the tree stays in the L2 caches."""
    import torch
    info = scene.info()
    width = info.tuned_width or 4
    n_seg, n_cross, n_node, n_tri = device_counts(rt, scene, eps, sig, cfg, out)
    t = _time(lambda: rt.rt_radio_map(scene, eps, sig, cfg.tx, cfg.plane, cfg.params, out), reps, 3)
    kern = kernel_ms(rt, scene, eps, sig, cfg, out, torch.cuda.current_stream(), reps)
    r = rooflines(n_seg, n_cross, n_node, n_tri, width, kern, traffic_from_profile())
    return {"workload": "manhattan: seeded 10x10-block city, 1,202 triangles, iso V-pol Tx at (0,0,30) m, 3.5 GHz, "
                        "1e7 Fibonacci rays, max depth 5, 1000x1000 cells of 1 m at z=1.5 m",
            "value": round(n_seg / (t * 1e-3) / 1e6, 3), "unit": "M ray-bounces/s", "ms_per_step": round(t, 4),
            "segments_per_step": n_seg, "crossings_per_step": n_cross, "build_ms": round(info.build_ms, 3),
            "bvh_depth": info.bvh_depth, "tuned": tuned_record(info, tune_s),
            "roofline": r}


def kernel_ms(rt, scene, eps, sig, cfg, out, stream, steps):
    """Average duration of the forward launch alone: with accumulate = 1 a call
    queues only the work-counter reset (one thread) and the launch-order
    rotations (a few hundred threads) besides the forward kernel."""
    import numpy as np
    import torch
    evk = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for s, e in evk:
        s.record(stream)
        rt.rt_radio_map(scene, eps, sig, cfg.tx, cfg.plane, cfg.params, out, accumulate=1)
        e.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([s.elapsed_time(e) for s, e in evk]))


def rooflines(n_seg, n_cross, n_node, n_tri, width, kern_ms, traffic,
              note="the Manhattan tree and triangles stay in L2: this is a model, not DRAM traffic"):
    """ALU roofline (primary) and the algorithmic HBM byte model for the forward kernel."""
    ops = ALU_OPS["child_box"] * width * n_node + ALU_OPS["tri"] * n_tri + ALU_OPS["segment"] * n_seg
    alg_bytes = NODE_BYTES[width] * n_node + 40 * n_tri + 8 * n_cross
    t = kern_ms * 1e-3
    alu = ops / t / 1e12
    hbm = alg_bytes / t / 1e9
    return {"bound": "alu", "achieved": round(alu, 3), "peak": round(ALU_PEAK_TOPS, 2), "unit": "T lane-ops/s",
            "frac": round(alu / ALU_PEAK_TOPS, 4),
            "traffic": (traffic["fetch_bytes"] + traffic["write_bytes"]) if traffic else None,
            "traffic_detail": traffic,
            "op_unit": "one FP32 VALU lane-operation (add/mul/min/max/compare); peak = 256 CUs x 64 lanes x 2.4 GHz",
            "kernel": "k_forward", "kernel_ms": round(kern_ms, 4), "alg_ops_per_launch": int(ops),
            "ops_model": "%d per child box x %d children per node visit + %d per triangle test + %d per segment" % (
                ALU_OPS["child_box"], width, ALU_OPS["tri"], ALU_OPS["segment"]),
            "node_visits": n_node, "tri_tests": n_tri, "tree_width": width,
            "hbm_model": {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(hbm / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": int(alg_bytes),
                          "byte_model": "%d B per node visit + 40 B per triangle test + 8 B per deposit" % NODE_BYTES[width],
                          "note": note}}


def traffic_from_profile(path=PROFILE_COUNTERS):
    try:
        with open(path) as f:
            pc = json.load(f)
        if pc.get("kernel_source_sha") == kernel_source_sha():
            return {"fetch_bytes": pc["fetch_bytes_per_launch"], "write_bytes": pc["write_bytes_per_launch"],
                    "calibration_factor": pc.get("calibration_factor"),
                    "source": os.path.relpath(path, ROOT)}
    except (OSError, KeyError, ValueError):
        pass
    return None


def large_extras(rt, sg, cfg, scene, eps, sig, dev, out, reps=3):
    """Side legs on the 1.02 M-triangle scene: Russian roulette from depth 2
    (p_max 0.5) against the plain run; 64 rooftop transmitters with ray
    budgets log-uniform in [1e5, 1e7] (L = 5, 64 x 1000 x 1000 maps) in one
    batched call against the per-transmitter loop of rt_radio_map calls on one
    stream (same outputs, one synchronisation); 16 material samples forward +
    backward in one batched call against 16 taped forwards and adjoints."""
    import dataclasses
    import numpy as np
    import torch
    res = {}
    n_seg = device_counts(rt, scene, eps, sig, cfg, out)[0]
    t = _time(lambda: rt.rt_radio_map(scene, eps, sig, cfg.tx, cfg.plane, cfg.params, out), reps, 1)
    prr = dataclasses.replace(cfg.params, rr_depth=2, rr_p_max=0.5, seed=1)
    seg_rr = device_counts(rt, scene, eps, sig, dataclasses.replace(cfg, params=prr), out)[0]
    t_rr = _time(lambda: rt.rt_radio_map(scene, eps, sig, cfg.tx, cfg.plane, prr, out), reps, 1)
    res["roulette"] = {"setting": "Russian roulette from depth 2, p_max 0.5", "plain_ms": round(t, 3),
                       "plain_segments": n_seg, "ms_per_step": round(t_rr, 3), "segments_per_step": seg_rr,
                       "speedup": round(t / t_rr, 3)}
    txs, budgets = sg.rooftop_transmitters(64, seed=5, buildings=sg.large_buildings())
    T = len(txs)
    maps = torch.empty((T, 1, cfg.plane.H, cfg.plane.W), dtype=torch.float32, device=dev)
    params = sg.Params(cfg.params.freq_hz, 1, 5)
    plist = [sg.Params(cfg.params.freq_hz, int(b), 5) for b in budgets]

    def plain_loop():
        for k in range(T):
            rt.rt_radio_map(scene, eps, sig, txs[k], cfg.plane, plist[k], maps[k])

    def batched():
        rt.rt_radio_map_batched(scene, eps[None], sig[None], txs, budgets, cfg.plane, params, maps)

    t_plain = _time(plain_loop, reps, 1)
    t_batch = _time(batched, reps, 1)
    res["batched_tx_over_plain"] = {"workload": "64 rooftop Tx (roof centre + 3 m), budgets log-uniform in "
                                                "[1e5, 1e7], %d rays, L = 5" % int(np.sum(budgets)),
                                    "batched_ms": round(t_batch, 3), "plain_loop_ms": round(t_plain, 3),
                                    "ratio": round(t_plain / t_batch, 3)}
    del maps
    # 16 material samples forward + backward from the headline transmitter
    # (1e6 rays, L = 5): one batched call against 16 taped forwards + adjoints
    S, n_rays = 16, 1_000_000
    H, W = cfg.plane.H, cfg.plane.W
    E, Sg = sg.random_materials(cfg.scene, S, seed=5)
    eS = torch.tensor(E, dtype=torch.float32, device=dev)
    sS = torch.tensor(Sg, dtype=torch.float32, device=dev)
    p1 = sg.Params(cfg.params.freq_hz, n_rays, 5)
    smaps = torch.empty((1, S, H, W), dtype=torch.float32, device=dev)
    gm = torch.randn((1, S, H, W), dtype=torch.float32, device=dev)
    grads = torch.empty((1, S, 2 * cfg.scene.n_materials + 3), dtype=torch.float32, device=dev)
    nm = cfg.scene.n_materials
    ge, gs, go = (torch.empty(n, dtype=torch.float32, device=dev) for n in (nm, nm, 3))
    tape = rt.rt_tape_create(p1)
    es_list = [eS[k].contiguous() for k in range(S)]
    ss_list = [sS[k].contiguous() for k in range(S)]
    g_list = [gm[0, k][None].contiguous() for k in range(S)]

    def plain_samples():
        for k in range(S):
            rt.rt_radio_map(scene, es_list[k], ss_list[k], cfg.tx, cfg.plane, p1, smaps[0, k][None], tape=tape)
            rt.rt_radio_map_backward(scene, es_list[k], ss_list[k], cfg.tx, cfg.plane, p1, tape, g_list[k], ge, gs, go)

    def batched_samples():
        rt.rt_radio_map_batched(scene, eS, sS, [cfg.tx], [n_rays], cfg.plane, sg.Params(cfg.params.freq_hz, 1, 5),
                                smaps, grad_maps=gm, grads=grads)

    t_ps = _time(plain_samples, reps, 1)
    t_bs = _time(batched_samples, reps, 1)
    res["batched_samples_over_plain"] = {"workload": "16 material samples forward + backward, headline Tx, "
                                                     "1e6 rays, L = 5", "batched_ms": round(t_bs, 3),
                                         "plain_loop_ms": round(t_ps, 3), "ratio": round(t_ps / t_bs, 3)}
    del smaps, gm, tape
    torch.cuda.empty_cache()
    return res


def extra_legs(rt, sg, cfg, scene, eps, sig, dev, reps=5):
    """Ratio legs on the same GPU, each against its plain per-call loop.

    * fwd+bwd / fwd: differentiation workload (Manhattan, 1e6 rays, L = 4,
      directional V-pol Tx at yaw 30 deg, pitch -10 deg): forward with a tape
      plus the adjoint, over the forward without a tape;
    * batched vs plain, 64 transmitters: seeded rooftop Tx with budgets
      log-uniform in [1e5, 1e7], L = 5, 64 x 1000 x 1000 maps; one batched
      call vs 64 rt_radio_map calls on one stream (same outputs, one sync);
    * batched vs plain, 16 material samples fwd + bwd: differentiation Tx,
      1e6 rays, L = 5; one batched call vs 16 forward-with-tape + backward.
    """
    import numpy as np
    import torch
    out = {}
    # ---- fwd+bwd / fwd
    dc = sg.diff_config()
    H, W = dc.plane.H, dc.plane.W
    m = torch.empty((1, H, W), dtype=torch.float32, device=dev)
    tape = rt.rt_tape_create(dc.params)
    g = torch.randn((1, H, W), dtype=torch.float32, device=dev)
    ge = torch.empty(2, dtype=torch.float32, device=dev)
    gs = torch.empty(2, dtype=torch.float32, device=dev)
    go = torch.empty(3, dtype=torch.float32, device=dev)

    def fwd():
        rt.rt_radio_map(scene, eps, sig, dc.tx, dc.plane, dc.params, m)

    def fwdbwd():
        rt.rt_radio_map(scene, eps, sig, dc.tx, dc.plane, dc.params, m, tape=tape)
        rt.rt_radio_map_backward(scene, eps, sig, dc.tx, dc.plane, dc.params, tape, g, ge, gs, go)

    t_f = _time(fwd, reps)
    t_fb = _time(fwdbwd, reps)
    out["fwd_bwd_over_fwd"] = round(t_fb / t_f, 3)
    out["diff_fwd_ms"] = round(t_f, 4)
    out["diff_fwd_bwd_ms"] = round(t_fb, 4)
    del tape

    # ---- 64 transmitters, uneven budgets
    txs, budgets = sg.rooftop_transmitters(64, seed=5, buildings=sg.manhattan_buildings(cfg.scene))
    T = len(txs)
    maps = torch.empty((T, 1, cfg.plane.H, cfg.plane.W), dtype=torch.float32, device=dev)
    params = sg.Params(cfg.params.freq_hz, 1, 5)
    plist = [sg.Params(cfg.params.freq_hz, int(b), 5) for b in budgets]

    def plain_loop():
        for t in range(T):
            rt.rt_radio_map(scene, eps, sig, txs[t], cfg.plane, plist[t], maps[t])

    def batched():
        rt.rt_radio_map_batched(scene, eps[None], sig[None], txs, budgets, cfg.plane, params, maps)

    t_plain = _time(plain_loop, reps, 1)
    t_batch = _time(batched, reps, 1)
    out["batched_tx_over_plain"] = round(t_plain / t_batch, 3)
    out["batched_tx_ms"] = round(t_batch, 3)
    out["plain_tx_loop_ms"] = round(t_plain, 3)
    out["batched_tx_rays"] = int(np.sum(budgets))
    del maps

    # ---- 16 material samples, forward + backward
    S = 16
    E, Sg = sg.random_materials(cfg.scene, S, seed=5)
    eS = torch.tensor(E, dtype=torch.float32, device=dev)
    sS = torch.tensor(Sg, dtype=torch.float32, device=dev)
    ptx = sg.Params(cfg.params.freq_hz, 1, 5)
    p1 = sg.Params(cfg.params.freq_hz, 1_000_000, 5)
    maps = torch.empty((1, S, H, W), dtype=torch.float32, device=dev)
    gm = torch.randn((1, S, H, W), dtype=torch.float32, device=dev)
    grads = torch.empty((1, S, 2 * cfg.scene.n_materials + 3), dtype=torch.float32, device=dev)
    tape = rt.rt_tape_create(p1)
    es_list = [eS[k].contiguous() for k in range(S)]
    ss_list = [sS[k].contiguous() for k in range(S)]
    g_list = [gm[0, k][None].contiguous() for k in range(S)]

    def plain_samples():
        for k in range(S):
            rt.rt_radio_map(scene, es_list[k], ss_list[k], dc.tx, dc.plane, p1, maps[0, k][None], tape=tape)
            rt.rt_radio_map_backward(scene, es_list[k], ss_list[k], dc.tx, dc.plane, p1, tape, g_list[k], ge, gs, go)

    def batched_samples():
        rt.rt_radio_map_batched(scene, eS, sS, [dc.tx], [1_000_000], dc.plane, ptx, maps, grad_maps=gm, grads=grads)

    t_ps = _time(plain_samples, reps, 1)
    t_bs = _time(batched_samples, reps, 1)
    out["batched_samples_over_plain"] = round(t_ps / t_bs, 3)
    out["batched_samples_ms"] = round(t_bs, 3)
    out["plain_samples_loop_ms"] = round(t_ps, 3)
    return out


def array_leg(rt, sg, cfg, scene, eps, sig, out, sizes=(1, 16, 64, 256, 1024)):
    """Synthetic transmit arrays (the paper's radio-map timing sweep over the
    number of transmit antennas): the Manhattan workload with a half-wavelength
    uniform linear array along x, steered to x-cosine 0.5, for several sizes."""
    import math
    import numpy as np
    lam = 299792458.0 / cfg.params.freq_hz
    res = {"workload": "manhattan, 1e7 rays, L = 5, ULA along x, half-wavelength spacing, steered to x-cosine 0.5",
           "ms": {}, "M ray-bounces/s": {}}
    st = None
    for n in sizes:
        base = sg.linear_array(n, 0.5 * lam)
        u = np.exp(-2j * math.pi * base.positions[:, 0] / lam * 0.5) / math.sqrt(n)
        tx = sg.Tx(cfg.tx.pos, array=sg.TxArray(base.positions, u.astype(np.complex64)))
        t = _time(lambda: rt.rt_radio_map(scene, eps, sig, tx, cfg.plane, cfg.params, out), 3, 1)
        if st is None:
            import torch
            stats = torch.zeros(8, dtype=torch.int64, device=out.device)
            rt.rt_radio_map(scene, eps, sig, tx, cfg.plane, cfg.params, out, stats=stats)
            st = int(stats[0])
        res["ms"][str(n)] = round(t, 3)
        res["M ray-bounces/s"][str(n)] = round(st / (t * 1e-3) / 1e6, 1)
    return res


def n_s_leg(rt, sg, cfg, scene, eps, sig, out, n_rays=(10 ** 6, 10 ** 7, 10 ** 8, 10 ** 9), sizes=(1, 64, 512)):
    """Time per radio map against the number of samples N_S and the number of
    transmit antennas, the shape of the paper's radio-map timing experiment
    (Sec. "Radio Map Solver": one source 20 m above the ground of a street
    scene, N_S up to 1e9, arrays of up to 512 antennas): the Manhattan city
    stands in for the street scene, with an isotropic V-pol source at
    (0, 0, 20) m and, for several antennas, a half-wavelength uniform linear
    array along x steered to x-cosine 0.5."""
    import math
    import numpy as np
    import torch
    lam = 299792458.0 / cfg.params.freq_hz
    pos = (0.0, 0.0, 20.0)
    res = {"workload": "manhattan (street-scene stand-in), iso V-pol source at (0, 0, 20) m, L = %d, %dx%d cells "
                       "of %g m; ULA along x, half-wavelength spacing, steered to x-cosine 0.5"
                       % (cfg.params.max_depth, cfg.plane.W, cfg.plane.H, cfg.plane.dx),
           "ms": {}, "M ray-bounces/s": {}, "segments": {}}
    for N in n_rays:
        p = sg.Params(cfg.params.freq_hz, int(N), cfg.params.max_depth)
        stats = torch.zeros(8, dtype=torch.int64, device=out.device)
        rt.rt_radio_map(scene, eps, sig, sg.Tx(pos), cfg.plane, p, out, stats=stats)
        torch.cuda.synchronize()
        seg = int(stats[0])
        res["segments"]["%.0e" % N] = seg
        for n in sizes:
            if n == 1:
                tx = sg.Tx(pos)
            else:
                base = sg.linear_array(n, 0.5 * lam)
                u = np.exp(-2j * math.pi * base.positions[:, 0] / lam * 0.5) / math.sqrt(n)
                tx = sg.Tx(pos, array=sg.TxArray(base.positions, u.astype(np.complex64)))
            reps = 2 if N >= 10 ** 9 else 3
            t = _time(lambda: rt.rt_radio_map(scene, eps, sig, tx, cfg.plane, p, out), reps, 1)
            key = "N_S=%.0e,N_A=%d" % (N, n)
            res["ms"][key] = round(t, 3)
            res["M ray-bounces/s"][key] = round(seg / (t * 1e-3) / 1e6, 1)
    return res


def refraction_leg(rt, sg, cfg, dev, out, launch=""):
    """Finite-thickness walls and refraction: the Manhattan workload (1e7 rays,
    L = 5) with 20 cm concrete and 10 mm glass slabs, every hit sampling
    reflection or transmission, against slab reflection only and the plain
    half-space path on the same scene.  The buildings' bottom faces are left
    out (they coincide with the ground, which transmitted rays could reach)."""
    import torch
    sc = sg.with_thickness(sg.manhattan_scene(bottoms=False))
    scene = rt.scene_from_mesh(sc)
    if launch:
        rt.rt_set_launch_config(scene, *[int(x) for x in launch.split(",")])
    else:
        rt.rt_tune(scene, torch.tensor(sc.eps_r, dtype=torch.float32, device=dev),
                   torch.tensor(sc.sigma, dtype=torch.float32, device=dev), cfg.tx, cfg.plane, cfg.params,
                   2_000_000, out)
    eps = torch.tensor(sc.eps_r, dtype=torch.float32, device=dev)
    sig = torch.tensor(sc.sigma, dtype=torch.float32, device=dev)
    thk = torch.tensor(sc.thickness, dtype=torch.float32, device=dev)
    res = {"workload": "manhattan without building bottoms (%d triangles), 1e7 rays, L = 5, "
                       "slabs: concrete 0.2 m, glass 0.01 m" % sc.n_triangles}
    for name, p, t in (("refraction", sg.Params(cfg.params.freq_hz, cfg.params.n_rays, cfg.params.max_depth,
                                                 refraction=1, seed=1), thk),
                       ("slab_reflection", cfg.params, thk),
                       ("half_space", cfg.params, None)):
        stats = torch.zeros(8, dtype=torch.int64, device=dev)
        rt.rt_radio_map(scene, eps, sig, cfg.tx, cfg.plane, p, out, stats=stats, thickness=t)
        seg = int(stats[0])
        ms = _time(lambda: rt.rt_radio_map(scene, eps, sig, cfg.tx, cfg.plane, p, out, thickness=t), 5, 1)
        res[name] = {"ms": round(ms, 3), "segments": seg, "M ray-bounces/s": round(seg / (ms * 1e-3) / 1e6, 1)}
    # forward with a tape + adjoint over forward: the differentiation
    # transmitter (directional, yaw 30 deg, pitch -10 deg), 1e6 rays, L = 4
    dc = sg.diff_config()
    pd = sg.Params(dc.params.freq_hz, dc.params.n_rays, dc.params.max_depth, refraction=1, seed=1)
    m = torch.empty((1, dc.plane.H, dc.plane.W), dtype=torch.float32, device=dev)
    tape = rt.rt_tape_create(pd)
    g = torch.randn((1, dc.plane.H, dc.plane.W), dtype=torch.float32, device=dev)
    ge = torch.empty(2, dtype=torch.float32, device=dev)
    gs = torch.empty(2, dtype=torch.float32, device=dev)
    go = torch.empty(3, dtype=torch.float32, device=dev)

    def fwd():
        rt.rt_radio_map(scene, eps, sig, dc.tx, dc.plane, pd, m, thickness=thk)

    def fwdbwd():
        rt.rt_radio_map(scene, eps, sig, dc.tx, dc.plane, pd, m, tape=tape, thickness=thk)
        rt.rt_radio_map_backward(scene, eps, sig, dc.tx, dc.plane, pd, tape, g, ge, gs, go, thickness=thk)

    t_f = _time(fwd, 5)
    t_fb = _time(fwdbwd, 5)
    res["fwd_bwd_over_fwd"] = {"workload": "same scene and slabs, refraction, directional Tx (yaw 30, pitch -10 "
                                           "deg), 1e6 rays, L = 4", "fwd_ms": round(t_f, 4),
                               "fwd_bwd_ms": round(t_fb, 4), "ratio": round(t_fb / t_f, 3)}
    del tape
    # batched transmitters with refraction: the 64 rooftop transmitters of the
    # plain batched leg, one call against the per-transmitter loop
    txs, budgets = sg.rooftop_transmitters(64, seed=5, buildings=sg.manhattan_buildings(sg.manhattan_scene()))
    T = len(txs)
    maps = torch.empty((T, 1, cfg.plane.H, cfg.plane.W), dtype=torch.float32, device=dev)
    pb = sg.Params(cfg.params.freq_hz, 1, cfg.params.max_depth, refraction=1, seed=1)
    plist = [sg.Params(cfg.params.freq_hz, int(b), cfg.params.max_depth, refraction=1, seed=1) for b in budgets]

    def plain_loop():
        for t in range(T):
            rt.rt_radio_map(scene, eps, sig, txs[t], cfg.plane, plist[t], maps[t], thickness=thk)

    def batched():
        rt.rt_radio_map_batched(scene, eps[None], sig[None], txs, budgets, cfg.plane, pb, maps, thickness=thk)

    t_plain = _time(plain_loop, 3, 1)
    t_batch = _time(batched, 3, 1)
    res["batched_tx_over_plain"] = {"workload": "64 rooftop Tx, %d rays, same slabs, refraction" % int(sum(budgets)),
                                    "batched_ms": round(t_batch, 3), "plain_loop_ms": round(t_plain, 3),
                                    "ratio": round(t_plain / t_batch, 3)}
    return res


def diffuse_leg(rt, sg, cfg, scene, eps, sig, dev, out):
    """Diffuse reflection: the Manhattan workload (1e7 rays, L = 5) with
    scattering coefficients S = 0.4 (concrete) and 0.2 (glass) and
    cross-polarisation shares K_x = 0.1 and 0.3, Lambertian pattern; every
    hit samples specular or diffuse reflection.  Also forward + adjoint over
    forward for the differentiation transmitter with the same materials."""
    import torch
    sca = torch.tensor([0.4, 0.2], dtype=torch.float32, device=dev)
    xpd = torch.tensor([0.1, 0.3], dtype=torch.float32, device=dev)
    p = sg.Params(cfg.params.freq_hz, cfg.params.n_rays, cfg.params.max_depth, seed=1)
    stats = torch.zeros(8, dtype=torch.int64, device=dev)
    rt.rt_radio_map(scene, eps, sig, cfg.tx, cfg.plane, p, out, stats=stats, scattering=sca, xpd=xpd)
    seg = int(stats[0])
    ms = _time(lambda: rt.rt_radio_map(scene, eps, sig, cfg.tx, cfg.plane, p, out, scattering=sca, xpd=xpd), 5, 1)
    res = {"workload": "manhattan, 1e7 rays, L = 5, Lambertian S = 0.4 / 0.2, K_x = 0.1 / 0.3 (concrete / glass)",
           "ms": round(ms, 3), "segments": seg, "M ray-bounces/s": round(seg / (ms * 1e-3) / 1e6, 1)}
    # forward with a tape + adjoint over forward: the differentiation
    # transmitter (directional, yaw 30 deg, pitch -10 deg), 1e6 rays, L = 4
    dc = sg.diff_config()
    pd = sg.Params(dc.params.freq_hz, dc.params.n_rays, dc.params.max_depth, seed=1)
    m = torch.empty((1, dc.plane.H, dc.plane.W), dtype=torch.float32, device=dev)
    tape = rt.rt_tape_create(pd)
    g = torch.randn((1, dc.plane.H, dc.plane.W), dtype=torch.float32, device=dev)
    ge = torch.empty(2, dtype=torch.float32, device=dev)
    gs = torch.empty(2, dtype=torch.float32, device=dev)
    go = torch.empty(3, dtype=torch.float32, device=dev)

    def fwd():
        rt.rt_radio_map(scene, eps, sig, dc.tx, dc.plane, pd, m, scattering=sca, xpd=xpd)

    def fwdbwd():
        rt.rt_radio_map(scene, eps, sig, dc.tx, dc.plane, pd, m, tape=tape, scattering=sca, xpd=xpd)
        rt.rt_radio_map_backward(scene, eps, sig, dc.tx, dc.plane, pd, tape, g, ge, gs, go, scattering=sca, xpd=xpd)

    t_f = _time(fwd, 5)
    t_fb = _time(fwdbwd, 5)
    res["fwd_bwd_over_fwd"] = {"workload": "same materials, directional Tx (yaw 30, pitch -10 deg), 1e6 rays, L = 4",
                               "fwd_ms": round(t_f, 4), "fwd_bwd_ms": round(t_fb, 4), "ratio": round(t_fb / t_f, 3)}
    return res


def _time(fn, reps=10, warm=2):
    """Average ms per call of fn() on the current stream (HIP events)."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def _oracle_chunks(job):
    """One oracle process: strided chunks of the lattice until the deadline."""
    import numpy as np
    import oracle
    cfg, offsets, stride, per_chunk, deadline = job
    segs = rays = 0
    for c in offsets:
        if time.time() >= deadline:
            break
        ids = c + stride * np.arange(per_chunk, dtype=np.int64)
        r = oracle.radio_map(cfg.scene, cfg.tx, cfg.plane, cfg.params, ray_ids=ids)
        segs += r.segments
        rays += ids.size
    return segs, rays


def cpu_baseline(cfg, seconds, workers=0):
    """FP64 oracle over a strided sample of the same lattice on the host cores.

    The sample is a set of chunks, chunk c holding rays c, c + 1e6, c + 2e6,
    ... (100 rays spread over the whole 1e8-ray lattice); `workers` oracle
    processes take interleaved chunks until `seconds` of wall time have
    passed.  The oracle itself is single-threaded brute force: every segment
    tests all 1.02 M triangles.
    """
    import multiprocessing as mp
    import oracle
    N = cfg.params.n_rays
    per_chunk = 100
    stride = N // per_chunk
    workers = int(workers or min(16, os.cpu_count() or 1))
    oracle.lib()   # built before forking
    gc.collect()   # collected before forking, so that no finalizer runs in a worker
    w0 = time.perf_counter()
    deadline = time.time() + seconds
    jobs = [(cfg, list(range(w, stride, workers)), stride, per_chunk, deadline) for w in range(workers)]
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_oracle_chunks, jobs)
    wall = time.perf_counter() - w0
    segs = sum(p[0] for p in parts)
    rays = sum(p[1] for p in parts)
    return {"value": round(segs / wall / 1e6, 6), "unit": "M ray-bounces/s", "cores": workers, "kind": "oracle",
            "sample": "%d rays of the 1e8-ray lattice (chunks of 100 rays 1e6 apart, interleaved over %d "
                      "single-threaded FP64 brute-force oracle processes), %d segments, %.1f s wall"
                      % (rays, workers, segs, wall),
            "per_core_segments_per_s": round(segs / wall / workers, 2),
            "host_cpu": _cpu_model(), "host_nproc": os.cpu_count()}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()

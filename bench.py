#!/usr/bin/env python3
"""Throughput of the Lagrangian-point tracking step on one MI355X.

One step = host-cell search + interpolation + spreading of every point of the
workload (8 bubbles' markers and 10^7 uniform particles on a band-refined
l 7->10 octree, FP32, fixed-point spreading) in one batched persistent pass
(with the in-step sort: 12 kernels on one stream).  Inputs are resident in
HBM before timing starts.

Prints one JSON line: points/s, the dominant kernel's achieved bandwidth
against the HBM peak (roofline), the FP64 oracle timed on a bounded sample on
the host cores (cpu_baseline), and side measurements (tree build, plain FP64
GPU path, spreading modes, error against the oracle).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "Lagrangian points located+interpolated+spread /s"
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_k_batch_cfg2.json")

# Algorithmic bytes (compulsory I/O, each input read once, each output
# written once): per point pos + id + vel + force; per touched leaf its key
# and level, its field row and its spread row.
BYTES_PER_POINT = {"f32": 12 + 4 + 12 + 12, "f64": 24 + 4 + 24 + 24}
BYTES_PER_LEAF = {"f32": 9 + 12 + 12, "f64": 9 + 24 + 24}


COPY_BYTES = 1 << 30


def write_traffic(args, fetch_csv, write_csv):
    """Per-launch HBM bytes of k_batch from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), each scaled by what the same counter reads for the 1 GiB
    calibration copy (which reads and writes exactly COPY_BYTES)."""
    import csv

    def per_kernel(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        batch = [float(r["Counter_Value"]) for r in rows if "k_batch" in r["Kernel_Name"]]
        copies = [float(r["Counter_Value"]) for r in rows if "copy" in r["Kernel_Name"].lower()]
        if not batch or not copies:
            raise SystemExit(f"{path}: no k_batch or copy dispatch with {counter}")
        return sum(batch) / len(batch), max(copies)

    fb, fc = per_kernel(fetch_csv, "FETCH_SIZE")
    wb, wc = per_kernel(write_csv, "WRITE_SIZE")
    ff = (COPY_BYTES / 1024.0) / fc
    fw = (COPY_BYTES / 1024.0) / wc
    rec = {"kernel": "k_batch", "config": args.config, "dtype": args.dtype, "mode": args.mode,
           "kernel_hash": kernel_source_hash(),
           "fetch_kib_per_launch": fb, "write_kib_per_launch": wb,
           "copy_fetch_kib": fc, "copy_write_kib": wc, "factor_fetch": ff, "factor_write": fw,
           "fetch_bytes": fb * 1024 * ff, "write_bytes": wb * 1024 * fw,
           "bytes_per_launch": int(fb * 1024 * ff + wb * 1024 * fw)}
    os.makedirs(os.path.dirname(PROFILE_TRAFFIC), exist_ok=True)
    with open(PROFILE_TRAFFIC, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# The library's sources and its build flags: a stored traffic record applies
# while they are unchanged.
def kernel_source_hash() -> str:
    import glob
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2605_20565_amd")
    files = sorted(glob.glob(os.path.join(pkg, "csrc", "*.hip")) + glob.glob(os.path.join(pkg, "csrc", "*.h")))
    for p in files + [os.path.join(pkg, "build.py"), os.path.join(ROOT, "include", "octrack.h")]:
        with open(p, "rb") as f:
            h.update(os.path.basename(p).encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def workload_desc(w, cfg):
    lv = np.bincount(w.tree.levels, minlength=w.tree.l_max + 1)[w.tree.l_min:]
    return {
        "workload": f"cfg{cfg}",
        "tree": f"band-refined octree l {w.tree.l_min}->{w.tree.l_max}, {w.tree.n_leaves} leaves "
                f"(per level {lv.tolist()}), periodic unit cube",
        "points": int(w.n_points),
        "instances": int(len(w.instances) - 1),
        "markers": int(sum(w.instances[i + 1] - w.instances[i] for i, k in enumerate(w.kinds) if k == "markers")),
        "ops": "locate+interpolate+spread",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--scale", type=float, default=1.0, help="multiplies the particle count")
    ap.add_argument("--dtype", choices=["f32", "f64"], default="f32")
    ap.add_argument("--mode", choices=["fixed", "atomic"], default="fixed")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--no-sort", action="store_true", help="process points in input order (no in-step sort)")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (use --block/--tile/--grid)")
    ap.add_argument("--host-major", action="store_true",
                    help="sorted plans use the host-major pass instead of the per-point pass")
    ap.add_argument("--presort-shift", type=int, default=0,
                    help="with --presorted: order by host id >> shift (6 mimics the in-step binning)")
    ap.add_argument("--presorted", action="store_true",
                    help="store the points in host-leaf order before timing (the layout a simulation that keeps "
                         "its particles sorted maintains) and run without the in-step sort")
    ap.add_argument("--cpu-sample", type=int, default=3_000_000, help="points in the oracle's timed sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip side measurements")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the side measurements on workloads 3 and 4 (about two minutes of generation)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with one 1 GiB device copy (reference kernel for rocprofv3 byte counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU: turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE) of a "
                         "--copy-calibration run into the per-launch traffic record under profiles/")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(args, *args.traffic_from)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding paragraph of the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import paper_2605_20565_amd as ot

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    dt = torch.float32 if args.dtype == "f32" else torch.float64

    t0 = time.time()
    w = synth.workload(args.config, scale=args.scale)
    log(f"[bench] workload cfg{args.config}: {w.tree.n_leaves} leaves, {w.n_points} points "
        f"({time.time() - t0:.1f}s to generate)")

    # ---- inputs resident in HBM --------------------------------------------
    anchors = torch.from_numpy(w.tree.anchors.astype(np.int32)).to(dev)
    levels = torch.from_numpy(w.tree.levels).to(dev)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    tree = ot.Tree.from_anchors(anchors, levels, w.tree.l_min, w.tree.l_max, w.tree.periodic)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - tb) * 1e3
    info = tree.info()
    log(f"[bench] tree built in {build_ms:.1f} ms; table {info.table_levels} levels, {info.table_bytes / 2**20:.1f} MiB")

    pos = torch.from_numpy(w.points).to(dev, dt)
    force = torch.from_numpy(w.forces).to(dev, dt)
    field = tree.permute_rows(torch.from_numpy(w.field).to(dev, dt))
    if args.presorted:
        order = torch.argsort(tree.locate(pos).long() >> args.presort_shift, stable=True)
        pos, force = pos[order].contiguous(), force[order].contiguous()
        args.no_sort = True
    n = pos.shape[0]
    ids = torch.empty(n, dtype=torch.int32, device=dev)
    vel = torch.empty((n, 3), dtype=dt, device=dev)
    fout = torch.empty((tree.n_leaves, 3), dtype=dt, device=dev)
    offsets = [int(v) for v in w.instances]
    ops = [ot.OT_OP_LOCATE | ot.OT_OP_INTERPOLATE | ot.OT_OP_SPREAD] * (len(offsets) - 1)
    shape = {"block": args.block, "tile": args.tile, "grid": args.grid, "sort_points": not args.no_sort,
             "host_major": args.host_major}
    tune_ms = None
    if not args.no_tune:
        from paper_2605_20565_amd import tune as tuner
        cands = [c for c in tuner.default_candidates(n) if not (args.no_sort and c.sort_points)]
        t_t = time.perf_counter()
        best, timings = tuner.tune(tree, offsets, ops, pos, field, force, dt, args.mode, candidates=cands, reps=3,
                                   cache_path=None, log=log)
        tune_ms = timings
        shape = {"block": best.block, "tile": best.tile, "grid": best.grid, "sort_points": best.sort_points,
                 "host_major": args.host_major}
        log(f"[bench] tuned in {time.perf_counter() - t_t:.1f}s: {best.label()}")
    plan = ot.BatchPlan(tree, offsets, ops, dtype=dt, mode=args.mode, **shape)
    n_tiles, grid = plan.shape()

    def step():
        plan.run(pos, field=field, force=force, ids=ids, vel=vel, field_out=fout)

    # ---- timed region: K steps back to back ----------------------------------
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = n * args.steps / elapsed
    log(f"[bench] {ms_per_step:.3f} ms/step, {value:.4g} points/s")

    # ---- dominant kernel duration: HIP events around it on its stream -------
    plan.set_timing(True)
    step()
    torch.cuda.synchronize()
    kms = []
    for _ in range(args.steps):
        step()
        torch.cuda.synchronize()
        kms.append(plan.last_kernel_ms())
    plan.set_timing(False)
    kernel_ms = float(np.mean(kms))
    hm_windows, hm_handed = plan.windows()

    # touched leaves: leaves that receive a weight from at least one point
    ones = torch.ones_like(pos)
    touched = int(torch.count_nonzero(tree.spread(ones, pos, mode="atomic").abs().sum(dim=1)).item())
    alg_bytes = n * BYTES_PER_POINT[args.dtype] + touched * BYTES_PER_LEAF[args.dtype]
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        with open(PROFILE_TRAFFIC) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == kernel_source_hash() and tr.get("dtype") == args.dtype \
                and tr.get("mode") == args.mode and tr.get("config") == args.config:
            traffic = tr.get("bytes_per_launch")
    step_gbps = alg_bytes / (ms_per_step * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": "k_hm + k_batch" if args.host_major else "k_batch", "kernel_ms": round(kernel_ms, 4),
                "algorithmic_bytes": int(alg_bytes), "touched_leaves": touched,
                "step_achieved": round(step_gbps, 1), "step_frac": round(step_gbps / HBM_PEAK_GBPS, 4)}
    log(f"[bench] k_batch {kernel_ms:.3f} ms, {achieved:.0f} GB/s algorithmic ({achieved / HBM_PEAK_GBPS:.1%} of peak); "
        f"whole step {step_gbps:.0f} GB/s ({step_gbps / HBM_PEAK_GBPS:.1%})")

    extra = {}
    if not args.no_extra:
        extra = side_measurements(args, w, tree, pos, force, field, plan, step, dev, dt, ot, torch, shape)

    if args.presorted:
        log("[bench] presorted input: not the headline layout")
    out = {
        "metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {**workload_desc(w, args.config), "precision": args.dtype, "spread_mode": args.mode,
                   "point_order": "host-leaf order (pre-sorted)" if args.presorted else "random (as generated)",
                   "path": "batched persistent kernel" + (", in-step sort of points by host leaf"
                                                          if shape["sort_points"] else ""),
                   "block": shape["block"] or "library default", "tile": shape["tile"] or "library default",
                   "tiles": n_tiles, "workgroups": grid, "autotuned": not args.no_tune,
                   "host_major_windows": hm_windows, "windows_to_per_point_pass": hm_handed},
        "roofline": roofline,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    out.update(extra)
    out["build_tree_ms"] = round(build_ms, 2)
    if args.copy_calibration:
        a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if tune_ms is not None:
        out["tuning_ms_per_step"] = tune_ms
    out["kernel_source"] = kernel_source_hash()
    print(json.dumps(out), flush=True)


def side_measurements(args, w, tree, pos, force, field, plan, step, dev, dt, ot, torch, shape):
    res = {}
    n = pos.shape[0]

    def timeit(fn, reps):
        fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) * 1e3 / reps

    # plain FP64 GPU path (one fused launch, FP64 atomics), the speedup's denominator
    p64 = torch.from_numpy(w.points).to(dev, torch.float64)
    f64 = torch.from_numpy(w.forces).to(dev, torch.float64)
    fl64 = tree.permute_rows(torch.from_numpy(w.field).to(dev, torch.float64))
    i64 = torch.empty(n, dtype=torch.int32, device=dev)
    v64 = torch.empty((n, 3), dtype=torch.float64, device=dev)
    o64 = torch.empty((tree.n_leaves, 3), dtype=torch.float64, device=dev)
    ms64 = timeit(lambda: tree.track(p64, field=fl64, force=f64, mode="atomic", ids=i64, vel=v64, field_out=o64),
                  max(3, args.steps // 2))
    res["fp64_plain"] = {"ms_per_step": round(ms64, 4), "value": n / (ms64 * 1e-3), "spread_mode": "atomic",
                         "path": "one fused launch per step"}
    ms_main = timeit(step, max(3, args.steps // 2))
    res["speedup_vs_fp64_plain"] = round(ms64 / ms_main, 3)
    # the batched path in FP64 (FIXED, sorted), same launch shape as the measured step
    pl64 = ot.BatchPlan(tree, [int(v) for v in w.instances], [7] * (len(w.instances) - 1), dtype=torch.float64,
                        mode="fixed", block=shape["block"], tile=shape["tile"], grid=shape["grid"],
                        sort_points=shape["sort_points"])
    ms64b = timeit(lambda: pl64.run(p64, field=fl64, force=f64, ids=i64, vel=v64, field_out=o64),
                   max(3, args.steps // 2))
    pl64.close()
    res["fp64_batched"] = {"ms_per_step": round(ms64b, 4), "value": n / (ms64b * 1e-3), "spread_mode": "fixed"}
    res["speedup_vs_fp64_batched"] = round(ms64b / ms_main, 3)
    del p64, f64, fl64, i64, v64, o64

    # one plain fused launch per instance (the alternative to one batched pass)
    offs = [int(v) for v in w.instances]
    ids_p = torch.empty(n, dtype=torch.int32, device=dev)
    vel_p = torch.empty((n, 3), dtype=dt, device=dev)
    fo_p = torch.empty((tree.n_leaves, 3), dtype=dt, device=dev)

    def per_instance():
        for i in range(len(offs) - 1):
            a, b = offs[i], offs[i + 1]
            tree.track(pos[a:b], field=field, force=force[a:b], mode=args.mode, ids=ids_p[a:b], vel=vel_p[a:b],
                       field_out=fo_p, accumulate=i > 0)
    res["per_instance_launches"] = {"launches": len(offs) - 1, "ms_per_step": round(timeit(per_instance, 3), 4)}

    # spreading modes on the batched FP32 path
    modes = {}
    for mode in ("fixed", "atomic"):
        pl = ot.BatchPlan(tree, [int(v) for v in w.instances], [7] * (len(w.instances) - 1), dtype=dt, mode=mode,
                          block=args.block, tile=args.tile, grid=args.grid, sort_points=not args.no_sort)
        ids = torch.empty(n, dtype=torch.int32, device=dev)
        vel = torch.empty((n, 3), dtype=dt, device=dev)
        fo = torch.empty((tree.n_leaves, 3), dtype=dt, device=dev)
        modes[mode] = round(timeit(lambda: pl.run(pos, field=field, force=force, ids=ids, vel=vel, field_out=fo),
                                   max(3, args.steps // 2)), 4)
        pl.close()
    res["spread_mode_ms_per_step"] = modes

    # FIXED mode is bitwise reproducible: five runs of the batched plan
    outs = []
    for _ in range(5):
        ids = torch.empty(n, dtype=torch.int32, device=dev)
        vel = torch.empty((n, 3), dtype=dt, device=dev)
        fo = torch.empty((tree.n_leaves, 3), dtype=dt, device=dev)
        plan.run(pos, field=field, force=force, ids=ids, vel=vel, field_out=fo)
        torch.cuda.synchronize()
        outs.append((ids.clone(), vel.clone(), fo.clone()))
    res["fixed_bitwise_repro_5_runs"] = args.mode == "fixed" and all(
        all(torch.equal(a.view(torch.uint8) if a.is_floating_point() else a,
                        b.view(torch.uint8) if b.is_floating_point() else b) for a, b in zip(outs[0], o))
        for o in outs[1:])
    del outs

    # multi-direct forcing (5 iterations) on the workload's bubble markers
    res["mdf"] = mdf_measure(w, tree, field, dev, dt, args.mode, torch, timeit)

    # point-particle step (trilinear, drag, AB2, relocation) on the workload's particle groups
    res["particle_step"] = particle_measure(w, tree, field, dev, dt, torch, timeit)

    # migration phase I: relocation after a sub-cell move, owners under an 8-way leaf partition
    res["migration"] = migration_measure(w, tree, pos, dev, torch, timeit)

    # differentiable pair on 10^6 markers over the workload's bubbles (workload 5's shape)
    res["backward_1e6_markers"] = backward_measure(w, tree, field, dev, dt, args.mode, ot, torch, timeit)

    # launch latency on the small workload 1 (11k points; latency bound, so no roofline figure)
    res["config1_latency_us"] = config1_latency(dev, dt, args.mode, ot, torch, timeit)
    # workload 1 as its configuration states it: the plain method in FP64
    res["config1_fp64_latency_us"] = config1_latency(dev, torch.float64, args.mode, ot, torch, timeit)

    # copy bandwidth for context
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    cms = timeit(lambda: b.copy_(a), 10)
    res["copy_GBps"] = round(2 * a.numel() * 4 / (cms * 1e-3) / 1e9, 1)
    del a, b

    # error against the oracle on a sample of the same inputs
    res["error_vs_oracle"] = oracle_check(w, tree, dev, dt, torch)
    if not args.no_workloads and args.config == 2:
        del ids_p, vel_p, fo_p
        torch.cuda.empty_cache()
        res["workload3"] = workload3_measure(args, dev, ot, torch, timeit)
        torch.cuda.empty_cache()
        res["workload4"] = workload4_measure(args, dev, ot, torch, timeit)
        torch.cuda.empty_cache()
    return res


def _touched(tree, P):
    ones = P.new_ones(P.shape)
    return int((tree.spread(ones, P, mode="atomic").abs().sum(dim=1) > 0).sum().item())


def _roof(n, touched, ms, dtype):
    gbps = (n * BYTES_PER_POINT[dtype] + touched * BYTES_PER_LEAF[dtype]) / (ms * 1e-3) / 1e9
    return {"algorithmic_GBps": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBPS, 4)}


def _workload_on_gpu(w, dev, dt, ot, torch):
    tree = ot.Tree.from_anchors(torch.from_numpy(w.tree.anchors.astype(np.int32)).to(dev),
                                torch.from_numpy(w.tree.levels).to(dev), w.tree.l_min, w.tree.l_max, w.tree.periodic)
    P = torch.from_numpy(w.points).to(dev, dt)
    F = torch.from_numpy(w.forces).to(dev, dt)
    U = tree.permute_rows(torch.from_numpy(w.field).to(dev, dt))
    return tree, P, F, U


def workload3_measure(args, dev, ot, torch, timeit):
    """Workload 3 (256 bubbles of log-uniform size + 64 particle groups, 320
    uneven instances): one batched, sorted pass against one
    plain fused launch per instance, FP32 FIXED."""
    import synth
    t0 = time.time()
    w = synth.workload(3)
    log(f"[bench] workload cfg3: {w.tree.n_leaves} leaves, {w.n_points} points ({time.time() - t0:.1f}s)")
    tree, P, F, U = _workload_on_gpu(w, dev, torch.float32, ot, torch)
    n = P.shape[0]
    offs = [int(v) for v in w.instances]
    ids = torch.empty(n, dtype=torch.int32, device=dev)
    vel = torch.empty_like(P)
    fo = torch.empty_like(U)
    # the launch shape from the autotuner's sorted candidates, as for the headline step
    from paper_2605_20565_amd import tune as tuner
    ops = [7] * (len(offs) - 1)
    cands = [c for c in tuner.default_candidates(n) if c.sort_points]
    best, _ = tuner.tune(tree, offs, ops, P, U, F, torch.float32, "fixed", candidates=cands, reps=3, cache_path=None)
    plan = ot.BatchPlan(tree, offs, ops, dtype=torch.float32, mode="fixed", sort_points=True, block=best.block,
                        tile=best.tile, grid=best.grid, host_major=args.host_major)
    ms_b = timeit(lambda: plan.run(P, field=U, force=F, ids=ids, vel=vel, field_out=fo), 10)
    plan.close()

    def per_instance():
        for i in range(len(offs) - 1):
            a, b = offs[i], offs[i + 1]
            tree.track(P[a:b], field=U, force=F[a:b], mode="fixed", ids=ids[a:b], vel=vel[a:b], field_out=fo,
                       accumulate=i > 0)
    ms_i = timeit(per_instance, 2)
    touched = _touched(tree, P)
    out = {"leaves": int(tree.n_leaves), "points": int(n), "instances": len(offs) - 1,
           "batched_ms_per_step": round(ms_b, 4), "batched_points_per_s": n / (ms_b * 1e-3),
           "per_instance_launches_ms_per_step": round(ms_i, 4), "batched_speedup": round(ms_i / ms_b, 2),
           "batched_shape": best.label(),
           "touched_leaves": touched, "batched_roofline": _roof(n, touched, ms_b, "f32"),
           "path": "batched persistent kernel, in-step sort; FP32, FIXED"}
    tree.close()
    return out


def workload4_measure(args, dev, ot, torch, timeit):
    """Workload 4 (10^8 particles in Gaussian shells, sigma = 2 finest dx,
    ~26 per finest leaf in the bands): FIXED vs FP32-atomic vs FP64 batched
    spreading steps, FIXED's bitwise reproducibility over 5 runs, and the
    error against the oracle on a 10^7-point subsample of the same points."""
    import synth
    t0 = time.time()
    w = synth.workload(4)
    log(f"[bench] workload cfg4: {w.tree.n_leaves} leaves, {w.n_points} points ({time.time() - t0:.1f}s)")
    tree, P, F, U = _workload_on_gpu(w, dev, torch.float32, ot, torch)
    n = P.shape[0]
    offs = [int(v) for v in w.instances]
    ops = [7] * (len(offs) - 1)
    ids = torch.empty(n, dtype=torch.int32, device=dev)
    vel = torch.empty_like(P)
    fo = torch.empty_like(U)
    touched = _touched(tree, P)
    res = {"leaves": int(tree.n_leaves), "points": int(n), "touched_leaves": touched}
    for mode in ("fixed", "atomic"):
        pl = ot.BatchPlan(tree, offs, ops, dtype=torch.float32, mode=mode, sort_points=True,
                          host_major=args.host_major)
        ms = timeit(lambda: pl.run(P, field=U, force=F, ids=ids, vel=vel, field_out=fo), 5)
        res[f"f32_{mode}"] = {"ms_per_step": round(ms, 3), "points_per_s": n / (ms * 1e-3),
                              **_roof(n, touched, ms, "f32")}
        if mode == "fixed":
            outs = []
            for _ in range(5):
                pl.run(P, field=U, force=F, ids=ids, vel=vel, field_out=fo)
                torch.cuda.synchronize()
                outs.append(fo.view(torch.int32).clone())
            res["fixed_bitwise_repro_5_runs"] = all(torch.equal(outs[0], o) for o in outs[1:])
            del outs
        pl.close()
    # FP64 batched (FIXED)
    P64, F64 = P.double(), F.double()
    U64 = tree.permute_rows(torch.from_numpy(w.field).to(dev, torch.float64))
    vel64, fo64 = torch.empty_like(P64), torch.empty_like(U64)
    pl = ot.BatchPlan(tree, offs, ops, dtype=torch.float64, mode="fixed", sort_points=True,
                      host_major=args.host_major)
    ms = timeit(lambda: pl.run(P64, field=U64, force=F64, ids=ids, vel=vel64, field_out=fo64), 3)
    pl.close()
    res["f64_fixed"] = {"ms_per_step": round(ms, 3), "points_per_s": n / (ms * 1e-3), **_roof(n, touched, ms, "f64")}
    del P64, F64, U64, vel64, fo64, vel, fo
    torch.cuda.empty_cache()
    # the oracle on a 10^7-point subsample (FP32-rounded inputs, the same batched path on the subsample)
    import oracle
    rng = np.random.default_rng(404)
    m = min(10_000_000, n)
    sel = np.sort(rng.choice(n, size=m, replace=False))
    pts = w.points[sel].astype(np.float32).astype(np.float64)
    frc = w.forces[sel].astype(np.float32).astype(np.float64)
    o = oracle.Tree.from_anchors(w.tree.anchors, w.tree.levels, w.tree.l_min, w.tree.l_max, w.tree.periodic)
    fld = o.permute_rows(w.field).astype(np.float32).astype(np.float64)
    Ps, Fs = torch.from_numpy(pts).to(dev, torch.float32), torch.from_numpy(frc).to(dev, torch.float32)
    Us = torch.from_numpy(fld).to(dev, torch.float32)
    pl = ot.BatchPlan(tree, [0, m], [7], dtype=torch.float32, mode="fixed", sort_points=True,
                      host_major=args.host_major)
    ids_s = torch.empty(m, dtype=torch.int32, device=dev)
    vel_s, fo_s = torch.empty_like(Ps), torch.empty_like(Us)
    pl.run(Ps, field=Us, force=Fs, ids=ids_s, vel=vel_s, field_out=fo_s)
    torch.cuda.synchronize()
    pl.close()
    t1 = time.time()
    want_ids = o.locate(pts)
    Uo, S = o.interpolate(fld, pts, with_scale=True)
    fo_o, Sf, cnt, A = o.spread(frc, pts, with_scale=True)
    log(f"[bench] oracle on the cfg4 subsample: {time.time() - t1:.1f}s")
    mm = float(np.abs(frc).max())
    _, E = math.frexp(m * mm)
    _, Ef = math.frexp(mm)
    q = math.ldexp(1.0, -min(62 - E, 51 - Ef))
    eu = np.abs(vel_s.cpu().double().numpy() - Uo) / np.maximum(S, 1e-300)
    bound = 1e-5 * Sf + 2.0 ** -110 * A + cnt[:, None] * 0.5 * q
    got = fo_s.cpu().double().numpy()
    touched_s = Sf > 0
    ef = np.abs(got - fo_o) / np.maximum(bound, 1e-300)
    res["error_vs_oracle_1e7_subsample"] = {
        "sample": m, "ids_mismatch": int((ids_s.cpu().numpy() != want_ids).sum()),
        "interp_scaled_max": float(eu.max()), "interp_tol": 1e-5,
        "spread_err_over_bound_max": float(ef[touched_s].max()),
        "spread_scaled_p99": float(np.percentile((np.abs(got - fo_o) / np.maximum(Sf, 1e-300))[touched_s], 99))}
    tree.close()
    return res


def particle_measure(w, tree, field, dev, dt, torch, timeit):
    idx = [i for i, k in enumerate(w.kinds) if k == "particles"]
    if not idx:
        return None
    sel = np.concatenate([np.arange(w.instances[i], w.instances[i + 1]) for i in idx])
    X = torch.from_numpy(np.ascontiguousarray(w.points[sel])).to(dev, dt)
    V = torch.zeros_like(X)
    VP = torch.zeros_like(X)
    AP = torch.zeros_like(X)
    ids = tree.locate(X)
    prm = dict(dt0=1e-3, r_p=1e-3, rho_p=2.5, rho_f=1.0, nu=1e-3, g=(0.0, 0.0, -1.0))
    tree.particle_step(field, X, V, VP, AP, ids, first=True, **prm)
    n = int(X.shape[0])
    # algorithmic bytes of a step: the four state arrays read and written, the
    # new host ids written, every leaf's field row read once
    nbytes = n * (8 * 3 * X.element_size() + 4) + field.numel() * field.element_size()
    ms = timeit(lambda: tree.particle_step(field, X, V, VP, AP, ids, **prm), 10)
    # host-ordered state (ot_particle_sort), the layout a simulation keeps by
    # re-sorting every few steps; the sort's own time is reported beside it
    from paper_2605_20565_amd import lib as otlib
    work = torch.empty(otlib.ot_particle_sort_workspace_bytes(n), dtype=torch.uint8, device=dev)
    outs = tuple(torch.empty_like(X) for _ in range(4))
    ms_sort = timeit(lambda: tree.particle_sort(X, V, VP, AP, out=outs, work=work), 5)
    Xs, Vs, VPs, APs, ids_s, _ = tree.particle_sort(X, V, VP, AP, out=outs, work=work)
    ms_sorted = timeit(lambda: tree.particle_step(field, Xs, Vs, VPs, APs, ids_s, **prm), 10)
    return {"particles": n, "ms_per_step": round(ms, 4), "particles_per_s": n / (ms * 1e-3),
            "algorithmic_bytes_per_step": nbytes,
            "hbm_frac": round(nbytes / (ms * 1e-3) / (HBM_PEAK_GBPS * 1e9), 4),
            "host_ordered_ms_per_step": round(ms_sorted, 4),
            "host_ordered_hbm_frac": round(nbytes / (ms_sorted * 1e-3) / (HBM_PEAK_GBPS * 1e9), 4),
            "sort_ms": round(ms_sort, 4)}


def backward_measure(w, tree, field, dev, dt, mode, ot, torch, timeit, per_body=125_000):
    """Interpolation of the leaf field at 10^6 markers (125k per bubble) and its backward: the field's
    gradient is the spread of the upstream gradient, the markers' the phi' contraction."""
    import synth
    if not w.spheres:
        return None
    X = torch.from_numpy(np.concatenate([synth.fibonacci_sphere(s, per_body) for s in w.spheres])).to(dev, dt)
    g = torch.randn(X.shape, generator=torch.Generator(device=dev).manual_seed(5), device=dev, dtype=dt)
    n = X.shape[0]
    U = torch.empty_like(X)
    gf = torch.empty_like(field)
    gx = torch.empty_like(X)
    fwd = timeit(lambda: tree.interpolate(field, X, out=U), 20)
    bwd = timeit(lambda: tree.interp_backward(field, g, X, mode=mode, grad_field=gf, grad_pos=gx), 20)
    spr = timeit(lambda: tree.spread(g, X, mode=mode, out=gf), 20)
    gpo = timeit(lambda: tree.grad_pos(field, g, X, out=gx), 20)
    Xr = X.clone().requires_grad_(True)
    ur = field.clone().requires_grad_(True)

    def autograd_step():
        (ot.interpolate(tree, ur, Xr, mode=mode) * g).sum().backward()
        Xr.grad = None
        ur.grad = None
    full = timeit(autograd_step, 10)
    touched = int((gf != 0).any(dim=1).sum())
    # the same pair as batched plans with the in-run sort of the markers by host leaf
    fplan = ot.BatchPlan(tree, [0, n], [ot.OT_OP_INTERPOLATE], dtype=dt, mode=mode, sort_points=True)
    bplan = ot.BatchPlan(tree, [0, n], [ot.OT_OP_SPREAD | ot.OT_OP_GRAD_POS], dtype=dt, mode=mode,
                         sort_points=True)
    fwd_s = timeit(lambda: fplan.run(X, field=field, vel=U), 20)
    bwd_s = timeit(lambda: bplan.run(X, field=field, force=g, field_out=gf, grad=gx), 20)
    fplan.close()
    bplan.close()
    b = dt.itemsize
    per_marker = 5 * 3 * b + 2 * 4   # forward pos, id, U; backward g, pos, id, grad_X
    per_leaf = 3 * 3 * b + 9         # field forward and backward, grad_field, key and level
    alg = n * per_marker + touched * per_leaf
    t_best = min(fwd, fwd_s) + min(bwd, bwd_s)   # the faster path of each direction
    return {"markers": n, "touched_leaves": touched, "spread_mode": mode, "forward_ms": round(fwd, 4),
            "backward_one_pass_ms": round(bwd, 4), "backward_separate_spread_ms": round(spr, 4),
            "backward_separate_grad_pos_ms": round(gpo, 4), "autograd_fwd_bwd_ms": round(full, 4),
            "batched_sorted_forward_ms": round(fwd_s, 4), "batched_sorted_backward_ms": round(bwd_s, 4),
            "markers_per_s_fwd_bwd": n / (t_best * 1e-3),
            "best_path": {"forward": "batched, sorted" if fwd_s < fwd else "plain",
                          "backward": "batched, sorted" if bwd_s < bwd else "plain one-pass"},
            "algorithmic_GBps": round(alg / (t_best * 1e-3) / 1e9, 1),
            "algorithmic_bytes": {"per_marker": per_marker, "per_touched_leaf": per_leaf}}


def migration_measure(w, tree, pos, dev, torch, timeit, P=8):
    n = pos.shape[0]
    dx = 1.0 / (1 << w.tree.l_max)
    g = torch.Generator(device=dev).manual_seed(3)
    moved_pos = torch.remainder(pos + 0.3 * dx * torch.randn(pos.shape, generator=g, device=dev, dtype=pos.dtype), 1.0)
    ids0 = tree.locate(pos)
    ids = ids0.clone()

    def reloc():
        ids.copy_(ids0)
        tree.relocate(moved_pos, ids, count=False)
    moved = tree.relocate(moved_pos, ids0.clone())
    reloc_ms = timeit(reloc, 10)
    copy_ms = timeit(lambda: ids.copy_(ids0), 10)
    out = torch.empty_like(ids0)
    locate_ms = timeit(lambda: tree.locate(moved_pos, out=out), 10)
    split = tree.leaf_splitters(P)
    owner_ms = timeit(lambda: tree.find_owner(split, moved_pos), 10)
    _, counts = tree.find_owner(split, moved_pos)
    return {"points": n, "displacement": "0.3 dx_finest rms per axis", "moved": moved,
            "relocate_ms": round(reloc_ms - copy_ms, 4), "full_locate_ms": round(locate_ms, 4),
            "owners": P, "find_owner_ms": round(owner_ms, 4), "per_owner_counts": counts.cpu().tolist()}


def mdf_measure(w, tree, field, dev, dt, mode, torch, timeit, n_iter=5):
    idx = [i for i, k in enumerate(w.kinds) if k == "markers"]
    if not idx:
        return None
    sel = np.concatenate([np.arange(w.instances[i], w.instances[i + 1]) for i in idx])
    P = torch.from_numpy(np.ascontiguousarray(w.points[sel])).to(dev, dt)
    tgt = torch.zeros_like(P)   # bodies at rest: the forcing drives the slip to zero
    u = field.clone()
    work = torch.empty(max(1, int(tree_mdf_bytes(tree, P))), dtype=torch.uint8, device=dev)
    ms = timeit(lambda: tree.mdf(u, P, tgt, n_iter, mode=mode, inplace=True, work=work), 10)
    # the same call captured once in a HIP graph and replayed
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        tree.mdf(u, P, tgt, n_iter, mode=mode, inplace=True, work=work)
    ms_graph = timeit(g.replay, 10)
    del g
    # the bodies' IBM force and torque from the marker forces (per-body sums)
    import paper_2605_20565_amd as ot
    _, f_lag, _ = tree.mdf(u, P, tgt, n_iter, mode=mode, work=work)
    offs = np.concatenate([[0], np.cumsum([w.instances[i + 1] - w.instances[i] for i in idx])])
    cen = torch.tensor([w.spheres[i].centre for i in range(len(idx))], dtype=dt, device=dev)
    us = timeit(lambda: ot.body_sums(f_lag, P, offs, cen, 1.0), 20) * 1e3
    # the mean IBM force over the domain, subtracted from the leaf force field
    # (deterministic FP64 reduction over all leaves, then the subtraction)
    _, _, f_eul = tree.mdf(u, P, tgt, n_iter, mode=mode, work=work)
    fm_work = torch.empty(ot.lib.ot_force_mean_workspace_bytes(), dtype=torch.uint8, device=dev)
    us_mean = timeit(lambda: tree.force_mean(f_eul, subtract=True, work=fm_work), 20) * 1e3
    return {"markers": int(P.shape[0]), "iterations": n_iter, "ms_per_step": round(ms, 4),
            "ms_per_iteration": round(ms / n_iter, 4), "graph_replay_ms_per_step": round(ms_graph, 4),
            "spread_mode": mode,
            "body_force_torque_us": round(us, 1), "bodies": len(idx),
            "force_mean_subtract_us": round(us_mean, 1), "leaves": int(tree.n_leaves)}


def tree_mdf_bytes(tree, P):
    import paper_2605_20565_amd as ot
    code = ot.OT_F32 if P.dtype.itemsize == 4 else ot.OT_F64
    return ot.lib.ot_mdf_workspace_bytes(tree._h, P.shape[0], code)


def config1_latency(dev, dt, mode, ot, torch, timeit):
    import synth
    w1 = synth.workload(1)
    t1 = ot.Tree.from_anchors(torch.from_numpy(w1.tree.anchors.astype(np.int32)).to(dev),
                              torch.from_numpy(w1.tree.levels).to(dev), w1.tree.l_min, w1.tree.l_max, w1.tree.periodic)
    P = torch.from_numpy(w1.points).to(dev, dt)
    F = torch.from_numpy(w1.forces).to(dev, dt)
    U = t1.permute_rows(torch.from_numpy(w1.field).to(dev, dt))
    n = P.shape[0]
    ids = torch.empty(n, dtype=torch.int32, device=dev)
    vel = torch.empty((n, 3), dtype=dt, device=dev)
    fo = torch.empty((t1.n_leaves, 3), dtype=dt, device=dev)
    plain = timeit(lambda: t1.track(P, field=U, force=F, mode=mode, ids=ids, vel=vel, field_out=fo), 50)
    offs = [int(v) for v in w1.instances]
    pl = ot.BatchPlan(t1, offs, [7] * (len(offs) - 1), dtype=dt, mode=mode)
    batched = timeit(lambda: pl.run(P, field=U, force=F, ids=ids, vel=vel, field_out=fo), 50)
    pl.close()
    pg = ot.BatchPlan(t1, offs, [7] * (len(offs) - 1), dtype=dt, mode=mode, graph=True)
    graph = timeit(lambda: pg.run(P, field=U, force=F, ids=ids, vel=vel, field_out=fo), 50)
    pg.close()
    return {"points": n, "leaves": t1.n_leaves, "plain_fused_launch": round(plain * 1e3, 1),
            "batched": round(batched * 1e3, 1), "batched_graph_replay": round(graph * 1e3, 1)}


def oracle_check(w, tree, dev, dt, torch, n_sample=20000):
    import oracle
    rng = np.random.default_rng(123)
    sel = np.sort(rng.choice(w.n_points, size=min(n_sample, w.n_points), replace=False))
    npdt = np.float32 if dt == torch.float32 else np.float64
    pts = w.points[sel].astype(npdt).astype(np.float64)
    frc = w.forces[sel].astype(npdt).astype(np.float64)
    o = oracle.Tree.from_anchors(w.tree.anchors, w.tree.levels, w.tree.l_min, w.tree.l_max, w.tree.periodic)
    fld = o.permute_rows(w.field).astype(npdt).astype(np.float64)
    P, F, Fd = (torch.from_numpy(x).to(dev, dt) for x in (pts, frc, fld))
    ids, vel, fo = tree.track(P, field=Fd, force=F, mode="fixed")
    U, S = o.interpolate(fld, pts, with_scale=True)
    f, Sf, cnt, A = o.spread(frc, pts, with_scale=True)
    eu = np.abs(vel.cpu().numpy() - U) / np.maximum(S, 1e-300)
    # spreading: per leaf against tol * sum|w F| + 2^-110 sum|F| (the oracle's
    # binary128 weights' absolute precision) + half a fixed-point quantum per contribution
    m = float(np.abs(frc).max())
    _, E = math.frexp(len(frc) * m)
    _, Ef = math.frexp(m)
    q = math.ldexp(1.0, -min(62 - E, 51 - Ef))
    tol = 1e-5 if dt == torch.float32 else 1e-12
    bound = tol * Sf + 2.0 ** -110 * A + cnt[:, None] * 0.5 * q
    ef = np.abs(fo.cpu().numpy() - f) / np.maximum(bound, 1e-300)
    touched = Sf > 0
    return {"sample": int(len(sel)), "ids_mismatch": int((ids.cpu().numpy() != o.locate(pts)).sum()),
            "interp_scaled_max": float(eu.max()), "interp_tol": tol,
            "spread_err_over_bound_max": float(ef[touched].max()),
            "spread_scaled_p99": float(np.percentile((np.abs(fo.cpu().numpy() - f) / np.maximum(Sf, 1e-300))[touched], 99))}


def cpu_baseline(w, n_sample):
    """The FP64 oracle (plain C, OpenMP over points; spreading into per-thread
    fields merged in thread order) on a bounded sample of the workload."""
    import oracle
    o = oracle.Tree.from_anchors(w.tree.anchors, w.tree.levels, w.tree.l_min, w.tree.l_max, w.tree.periodic)
    fld = o.permute_rows(w.field)
    rng = np.random.default_rng(7)
    m = min(n_sample, w.n_points)
    sel = np.sort(rng.choice(w.n_points, size=m, replace=False))
    pts = np.ascontiguousarray(w.points[sel])
    frc = np.ascontiguousarray(w.forces[sel])
    t = time.perf_counter()
    o.locate(pts)
    o.interpolate(fld, pts)
    o.spread(frc, pts)
    el = time.perf_counter() - t
    threads = oracle.num_threads()
    log(f"[bench] oracle: {m} points in {el:.1f}s on {threads} threads")
    # the same on one thread, on a tenth of the sample
    m1 = max(1, m // 10)
    oracle.set_num_threads(1)
    t = time.perf_counter()
    o.locate(pts[:m1])
    o.interpolate(fld, pts[:m1])
    o.spread(frc[:m1], pts[:m1])
    el1 = time.perf_counter() - t
    oracle.set_num_threads(threads)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": m / el, "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": f"{m} points drawn uniformly from the {w.n_points}-point workload, full tree; "
                      f"locate+interpolate+spread in FP64, {el:.1f}s",
            "single_thread_value": m1 / el1, "single_thread_sample": f"first {m1} points of the sample, {el1:.1f}s",
            "cpu_model": model, "nproc": os.cpu_count()}


if __name__ == "__main__":
    main()

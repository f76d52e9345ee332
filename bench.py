"""Benchmark of the axion-coupled Yee step on one MI355X.

Default workload: the 3D focused-pulse + counter-propagating axion packet run
(512^3 cells, lambda/12, FP32 fields, Mur EM and outflow axion boundaries),
advanced by the fused one-pass kernel.  One step = one full leapfrog step of
every field (E0/B0, axion, E1/B1, boundaries); diagnostics are recorded every
100 steps inside the timed region.

Printed: one JSON line with the throughput (Gcell-updates/s), the HBM roofline
of the fused kernel (algorithmic bytes per launch / mean launch time from HIP
events on the run's stream), the unfused path for comparison, and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def words_per_cell(ndim):
    """State words one cell-update reads and writes once: every stored EM
    component read and written, phi read at two levels and written once."""
    em = {1: 8, 2: 9, 3: 12}[ndim]
    return 2 * em + 3


def workload(name):
    from paper_2406_16796_amd import workloads as W
    if name == "3d":
        cfg = W.focused_3d()
    elif name == "2d":
        cfg = W.gaussian_2d()
    elif name == "1d":
        cfg = W.plane_wave_1d()
    else:
        raise SystemExit("unknown workload " + name)
    return cfg


def cells(cfg):
    n = cfg["n"]
    return int(n[0]) * int(n[1]) * int(n[2])


def time_path(axf, torch, cfg, precision, path, steps, warmup, diag_every):
    run = axf.Run(cfg, precision=precision, path=path, diag_every=diag_every)
    run.step(max(warmup, 1))
    run.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.step(steps)
    run.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms, launches = run.last_step_timing()
    rec = run.diag_now()
    del run
    torch.cuda.empty_cache()
    return wall, ev_ms, launches, rec


def cpu_baseline(cfg, target_s=15.0):
    """The FP64 oracle on a bounded sample: the same workload on a grid cut
    down to a few 10^5-10^6 cells, timed over whole steps."""
    from oracle.oracle import Oracle
    sample = dict(cfg)
    ndim = sum(1 for v in cfg["n"] if v > 1)
    side = {3: 64, 2: 512, 1: 4096}[ndim]
    n = [min(int(v), side) if v > 1 else 1 for v in cfg["n"]]
    sample["n"] = n
    sample["slab_hi"] = min(int(cfg.get("slab_hi", n[0])), n[0])
    sample["slab_lo"] = min(int(cfg.get("slab_lo", 0)), n[0])
    o = Oracle(sample)
    o.step(1)
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < target_s and steps < 1000:
        o.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    nc = n[0] * n[1] * n[2]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": nc * steps / dt / 1e9, "unit": "Gcell-updates/s", "cores": threads, "kind": "oracle",
            "sample": "%s grid of the same workload, %d steps, FP64, %.1f s" % ("x".join(map(str, n)), steps, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="3d", choices=["3d", "2d", "1d"])
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--diag-every", type=int, default=100)
    ap.add_argument("--plain-steps", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this build runs on one GPU only (--gpus %d requested); multi-GPU sharding is "
              "described in DESIGN.md but not built" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_16796_amd import axf
    torch.cuda.set_device(0)
    cfg = workload(args.workload)
    prec = axf.F32 if args.precision == "f32" else axf.F64
    esize = 4 if prec == axf.F32 else 8
    ndim = sum(1 for v in cfg["n"] if v > 1)
    nc = cells(cfg)

    # whole hot path (fused step + diagnostics at the configured cadence)
    wall, ev_ms, launches, rec = time_path(axf, torch, cfg, prec, axf.PATH_AUTO, args.steps, args.warmup,
                                           args.diag_every)
    value = nc * args.steps / wall / 1e9
    # the dominant kernel alone: fused launches only, HIP events on the run's stream
    _, k_ms, k_launches, _ = time_path(axf, torch, cfg, prec, axf.PATH_AUTO, args.steps, 2, 0)
    per_launch_s = k_ms / 1e3 / max(k_launches, 1)
    algo_bytes = words_per_cell(ndim) * esize * nc
    achieved = algo_bytes / per_launch_s / 1e9
    traffic = None
    # unfused path for comparison
    p_wall, p_ms, p_launches, _ = time_path(axf, torch, cfg, prec, axf.PATH_PLAIN, args.plain_steps, 2, 0)
    plain_value = nc * args.plain_steps / p_wall / 1e9

    line = {
        "metric": "Gcell-updates/s (fused step; % of HBM roofline)",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": cfg.get("name"), "ndim": ndim, "n": cfg["n"], "dx": cfg["dx"][0], "dt": cfg["dt"],
            "m": cfg["m"], "g": cfg["g"], "em_bc": "mur", "axion_bc": cfg["ax_bc"][0],
            "diag_every": args.diag_every, "path": "fused",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_fused", "bytes_per_launch": algo_bytes, "mean_launch_ms": round(per_launch_s * 1e3, 4),
            "launches": k_launches,
        },
        "plain": {"value": round(plain_value, 3), "unit": "Gcell-updates/s",
                  "ms_per_step": round(p_wall / args.plain_steps * 1e3, 4),
                  "launches_per_step": round(p_launches / max(args.plain_steps, 1), 2),
                  "speedup_fused": round(value / plain_value, 3) if plain_value > 0 else None},
        "diag": {"p_gen": rec["p_gen"], "p_conv": rec["p_conv"], "finite": rec["finite"]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark of the axion-coupled Yee step on one MI355X.

Default workload: the 3D focused-pulse run (512^3 cells at lambda/12, dt =
0.95 dx / sqrt(3)): a focused Gaussian laser (waist 6 lambda, FWHM 10
lambda, E along z) entering through the x_min Mur face and a counter-
propagating Gaussian axion packet (k = 1, width 5 lambda, amplitude 1e-3),
m = 0.3, g = 1e-4, uniform B0 along z, Mur EM and outflow axion boundaries,
FP32 fields, advanced by the one-pass march (one interior launch and one
boundary-frame launch per step).  One step is one full leapfrog step of
every field (zero-order E/B, axion, first-order E/B, Mur and axion
boundaries, laser injection); the energy and probability diagnostics are
recorded every 100 steps inside the timed region.

Printed: one JSON line with the whole-path throughput (Gcell-updates/s), the
HBM roofline of the step (algorithmic bytes per step over the mean step time
from HIP events on the run's stream; measured HBM traffic from the committed
rocprofv3 counter summary when it matches the kernel source), the unfused
path for comparison, the 2D 4096^2 Gaussian-pulse run in FP32 and FP64 (its
fraction from counted HBM bytes: a pass advances four steps), a device copy
for the achievable bandwidth, and the FP64 CPU oracle timed on a bounded
sample of the same workload on one host thread and on all of them.

Other modes:
  --profile-only          the device copy and the fused steps only (the command
                          the rocprofv3 counter passes run)
  --pmc-summary F W       turn the FETCH_SIZE and WRITE_SIZE counter CSVs of two
                          rocprofv3 --pmc runs of --profile-only into the traffic
                          summary under profiles/
  --trace-summary S       turn the kernel_stats CSV of a rocprofv3 --kernel-trace
                          --stats run of this script into the summary under profiles/
"""
import argparse
import csv
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# built-in shape of the 2D wavefront step: (steps per pass, rows per interior
# wavefront, prefetch distance, rows per frame wavefront)
DEFAULT_WAVE_SHAPE = {"f32": (4, 16, 2, 8), "f64": (4, 16, 1, 8)}
COPY_BYTES = 1 << 30
CSRC = "paper_2406_16796_amd/csrc/"
COMMON_SOURCES = [CSRC + "axf_stencil.h", CSRC + "axf_internal.h", "paper_2406_16796_amd/build.py"]
# workload -> (generator, file tag of the step kernels, kernel-name patterns of
# one step's launches ({T} = float or double, {NW} = row wavefronts per march
# workgroup), sources those kernels are built from)
WORKLOADS = {
    "2d": ("gaussian_2d", "k_wave2d", ["k_wave2d_pass<{T}", "k_wave2d_int<{T}", "k_wave2d<{T}"],
           [CSRC + "axf_fused.hip", CSRC + "axf_fused.h"] + COMMON_SOURCES),
    "3d": ("focused_3d", "k_march3d", ["k_march3d<{T},{NW},0>", "k_march3d<{T},{NW},1>", "k_march3d<{T},{NW},2>"],
           [CSRC + "axf_march3d.hip", CSRC + "axf_fused.h"] + COMMON_SOURCES),
    "1d": ("plane_wave_1d", "k_wave1d", ["k_wave1d<{T},256>"],
           [CSRC + "axf_wave1d.hip", CSRC + "axf_fused.h"] + COMMON_SOURCES),
    "fps": ("weak_laser_plasma_2d", "k_push", ["k_push<{T}>", "k_jzero<{T}>"],
            [CSRC + "axf_particles.hip", CSRC + "axf_kernels.h"] + COMMON_SOURCES),
    "window": ("gaussian_2d_window", "k_win_rows", ["k_win_rows<{T}", "k_win_xghosts<{T}>"],
               [CSRC + "axf_window.hip"] + COMMON_SOURCES),
}
# words of each cell a window move reads and writes in 2D (E0x, E0y, B0z, E1,
# B1, phi at two levels); the boundary planes that move with them are left out
WINDOW_WORDS_2D = 11
# particle state words a push reads (x, y, u, x1, y1, u1, w) and writes (all but w)
PARTICLE_WORDS = 11 + 10


def pattern_label(p):
    return p if p.endswith(">") else p + ",...>"


# row wavefronts per workgroup of the 3D march by storage precision
MARCH_NW = {"f32": 8, "f64": 6}


def step_patterns(name, precision):
    """Kernel-name patterns (spaces removed) of one step's launches."""
    t = "float" if precision == "f32" else "double"
    return [p.replace("{T}", t).replace("{NW}", str(MARCH_NW[precision])) for p in WORKLOADS[name][2]]


def words_per_cell(ndim):
    """State words one cell-update reads and writes once: every stored EM
    component read and written, phi read at two levels and written once."""
    em = {1: 8, 2: 9, 3: 12}[ndim]
    return 2 * em + 3


def workload(name):
    from paper_2406_16796_amd import workloads as W
    return getattr(W, WORKLOADS[name][0])()


def workload_tag(cfg, precision):
    n = [int(v) for v in cfg["n"] if int(v) > 1]
    return "%s_%s_%s" % (cfg["name"], "x".join(map(str, n)), precision)


def kernel_source_hash(name):
    h = hashlib.sha256()
    for rel in WORKLOADS[name][3]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_file(tag, kernel):
    return os.path.join(ROOT, "profiles", "%s_%s_hbm_traffic.md" % (kernel, tag))


def read_traffic(name, tag, kernel):
    """HBM bytes per launch from the committed counter summary, or None when
    it is missing or was taken on another version of the kernel source."""
    path = traffic_file(tag, kernel)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- `") and "=" in line:
                k, v = line[3:].split("`", 1)[0].split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash(name):
        return None
    return float(vals["traffic_bytes_per_launch"])


def device_copy(torch):
    """A plain device copy of COPY_BYTES: the calibration kernel of the
    counter passes and the achievable HBM bandwidth on this GPU."""
    n = COPY_BYTES // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        torch.neg(src, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * COPY_BYTES / (ms * 1e-3) / 1e9


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
    fused = run.uses_fused()
    del run
    torch.cuda.empty_cache()
    return wall, ev_ms, launches, rec, fused


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, target_s=12.0):
    """The FP64 oracle on a bounded sample: the same workload on a grid cut
    down to a few 10^5 cells, timed over whole steps, on every thread the
    OpenMP runtime gives it (OMP_NUM_THREADS) and on one thread."""
    from oracle.oracle import Oracle
    sample = dict(cfg)
    ndim = sum(1 for v in cfg["n"] if v > 1)
    side = {3: 64, 2: 512, 1: 4096}[ndim]
    n = [min(int(v), side) if v > 1 else 1 for v in cfg["n"]]
    sample["n"] = n
    sample["slab_hi"] = min(int(cfg.get("slab_hi", n[0])), n[0])
    sample["slab_lo"] = min(int(cfg.get("slab_lo", 0)), n[0])
    nc = n[0] * n[1] * n[2]
    out = {}
    for label, threads in (("all", None), ("one", 1)):
        if threads is None:
            Oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1))
        else:
            Oracle.set_threads(threads)
        o = Oracle(sample)
        o.step(1)
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < target_s and steps < 1000:
            o.step(1)
            steps += 1
        dt = time.perf_counter() - t0
        out[label] = (nc * steps / dt / 1e9, o.threads(), steps, dt)
        o.close()
    v, th, steps, dt = out["all"]
    v1, _, steps1, dt1 = out["one"]
    return {"value": round(v, 5), "unit": "Gcell-updates/s", "cores": th, "kind": "oracle",
            "sample": "%s cells of the same workload (FP64, same boundaries and sources), %d whole steps in %.1f s "
                      "on %d threads" % ("x".join(map(str, n)), steps, dt, th),
            "cpu_model": cpu_model(),
            "one_thread": {"value": round(v1, 5), "cores": 1,
                           "sample": "the same sample, %d whole steps in %.1f s" % (steps1, dt1)}}


def leg_1d(axf, torch):
    """The 4096-cell 1D conversion run (FP64, 3000 steps, CW laser, periodic
    axion, Mur EM), fused passes against the unfused phase sequence, both
    timed whole with HIP events on the run's stream."""
    from paper_2406_16796_amd import workloads as W
    cfg = W.plane_wave_1d()
    steps = int(cfg["steps"])
    out = {"workload": workload_tag(cfg, "f64"), "steps": steps}
    for label, path in (("fused", axf.PATH_FUSED), ("plain", axf.PATH_PLAIN)):
        _, ms, launches, rec, _ = time_path(axf, torch, cfg, axf.F64, path, steps, 2, 0)
        out[label] = {"ms": round(ms, 3), "launches": launches,
                      "Gcell_s": round(int(cfg["n"][0]) * steps / (ms * 1e-3) / 1e9, 3), "p_gen": rec["p_gen"]}
    out["fused_speedup"] = round(out["plain"]["ms"] / out["fused"]["ms"], 2)
    out["p_bitwise_equal"] = out["fused"]["p_gen"] == out["plain"]["p_gen"]
    return out


def fps_late_start(cfg):
    """First step of the late window of the weak-laser plasma: the pulse
    centre three quarters of the way across the grid, every particle behind
    it perturbed to first order."""
    return int((cfg["t_center"] + 0.75 * cfg["n"][0] * cfg["dx"][0]) / cfg["dt"])


def leg_fps(axf, torch, steps=1000):
    """The weak-laser plasma of Sec. III.D (12000 x 100 cells, one cold
    electron per cell, FP32): the step with the particles against the same
    grid in vacuum, both timed with HIP events on the run's stream.  The
    difference is the particle kernels' share of a step (the push and the
    zeroing of the current arrays); the push moves PARTICLE_WORDS words of
    particle state per particle.

    The push leaves out the atomic additions of zero terms, and a particle
    the laser has not reached has a zero first-order state, so the share
    depends on how much of the plasma the laser has swept.  Two windows of
    `steps` steps are timed: at the start ("early", the pulse entering the
    plasma) and once the pulse centre has crossed three quarters of the grid
    ("late", every particle behind it perturbed); the roofline figure is the
    late one."""
    from paper_2406_16796_amd import workloads as W
    out = {}
    late0 = fps_late_start(W.weak_laser_plasma_2d(plasma=True))
    for phase, advance in (("early", 2), ("late", late0)):
        res = {"start_step": advance}
        for label, plasma in (("plasma", True), ("vacuum", False)):
            cfg = W.weak_laser_plasma_2d(plasma=plasma)
            _, ms, launches, rec, _ = time_path(axf, torch, cfg, axf.F32, axf.PATH_AUTO, steps, advance, 0)
            res[label] = {"ms_per_step": round(ms / steps, 5), "launches_per_step": round(launches / steps, 2)}
            if plasma:
                npart = (cfg["plasma_hi"] - cfg["plasma_lo"]) * cfg["n"][1] * cfg["ppc"][0] * cfg["ppc"][1]
                out["workload"] = workload_tag(cfg, "f32")
                out["particles"] = npart
        dt_s = (res["plasma"]["ms_per_step"] - res["vacuum"]["ms_per_step"]) * 1e-3
        res["particle_ms_per_step"] = round(dt_s * 1e3, 5)
        res["particle_pushes_per_s"] = round(out["particles"] / dt_s, 1) if dt_s > 0 else None
        out[phase] = res
    dt_s = out["late"]["particle_ms_per_step"] * 1e-3
    gbs = out["particles"] * PARTICLE_WORDS * 4 / dt_s / 1e9 if dt_s > 0 else None
    out["particle_roofline"] = {"bound": "hbm", "achieved": round(gbs, 1) if gbs else None, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4) if gbs else None,
                                "bytes_per_particle": PARTICLE_WORDS * 4, "window": "late"}
    return out


def window_moves(cfg, n0, n1):
    """Window moves between steps n0 and n1 (the library's schedule: the
    window stands win_cells * floor((t - win_t0) / (win_cells dx)) columns
    along at t = n dt, and has not moved before win_t0)."""
    def target(n):
        t = n * cfg["dt"]
        if n < 1 or t < cfg["win_t0"]:
            return 0
        return int(math.floor((t - cfg["win_t0"]) / (cfg["win_cells"] * cfg["dx"][0])))
    return target(n1) - target(n0)


def window_points(cfg):
    """Storage points of a 2D grid (node counts: n + 1 along a Mur axis)."""
    from paper_2406_16796_amd import workloads as W
    return math.prod(int(cfg["n"][d]) + (1 if cfg["em_bc"][d] == W.EM_MUR else 0) for d in range(2))


def leg_window(axf, torch, steps=600):
    """The moving window of Sec. III.B on the 4096^2 FP32 Gaussian-pulse run:
    the run with a move every 8 columns against the same run standing, both
    timed with HIP events on the run's stream.  The difference over the
    moves in the timed steps is the cost of one move; a move reads and
    writes WINDOW_WORDS_2D words of every cell."""
    from paper_2406_16796_amd import workloads as W
    out = {}
    warm = 8
    for label, cfg in (("static", W.gaussian_2d()), ("window", W.gaussian_2d_window(8))):
        _, ms, launches, _, _ = time_path(axf, torch, cfg, axf.F32, axf.PATH_AUTO, steps, warm, 0)
        out[label] = {"ms_per_step": round(ms / steps, 5)}
        if label == "window":
            out["workload"] = workload_tag(cfg, "f32")
            moves = window_moves(cfg, warm, warm + steps)
            nn = window_points(cfg)
            out["moves"] = moves
            per_move = (out["window"]["ms_per_step"] - out["static"]["ms_per_step"]) * steps / moves
            out["ms_per_move"] = round(per_move, 4)
            gbs = 2 * WINDOW_WORDS_2D * 4 * nn / (per_move * 1e-3) / 1e9 if per_move > 0 else None
            out["move_roofline"] = {"bound": "hbm", "achieved": round(gbs, 1) if gbs else None, "peak": HBM_PEAK_GBS,
                                    "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4) if gbs else None,
                                    "bytes_per_move": 2 * WINDOW_WORDS_2D * 4 * nn}
    return out


def leg_2d(axf, torch, precision, steps=200):
    """The 2D Gaussian-pulse run (4096^2, lambda/16) through the fused 2D
    wavefront kernel in one storage precision (the FP32 vs FP64 comparison of
    that configuration).  A pass of that kernel advances several steps per
    read of the state, so its HBM fraction is taken from the counted bytes of
    the committed counter summary over the measured step time; the
    algorithmic-equivalent rate (one full read and write of the state per
    step) is given beside it and may exceed the peak."""
    cfg = workload("2d")
    prec = axf.F64 if precision == "f64" else axf.F32
    esize = 8 if precision == "f64" else 4
    nc = int(cfg["n"][0]) * int(cfg["n"][1]) * int(cfg["n"][2])
    _, ms, launches, _, fused = time_path(axf, torch, cfg, prec, axf.PATH_AUTO, steps, 4, 0)
    step_s = ms / 1e3 / steps
    equiv = words_per_cell(2) * esize * nc / step_s / 1e9
    tag = workload_tag(cfg, precision)
    traffic = read_traffic("2d", tag, WORKLOADS["2d"][1]) if fused else None
    roof = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s", "path_fused": fused,
            "algorithmic_equivalent_GBs": round(equiv, 1), "traffic": round(traffic) if traffic else None}
    if traffic:
        roof["achieved"] = round(traffic / step_s / 1e9, 1)
        roof["frac"] = round(traffic / step_s / 1e9 / HBM_PEAK_GBS, 4)
        roof["basis"] = "counted HBM bytes per step (FETCH_SIZE + WRITE_SIZE) over the mean step time"
    else:
        roof["achieved"] = None
        roof["frac"] = None
        roof["basis"] = "no counter summary for this kernel source: fraction not reported"
    return {"workload": tag, "Gcell_s": round(nc / step_s / 1e9, 3), "ms_per_step": round(step_s * 1e3, 4),
            "launches_per_step": round(launches / steps, 3), "roofline": roof}


def scan_leg(axf, torch, steps_scale, count=512, tune=True):
    """Batched parameter scan (512 runs: 1D 1k-64k cells, 2D 256^2-1024^2, step
    counts scaled by steps_scale) against the same runs launched one by one."""
    from paper_2406_16796_amd import workloads as W
    cfgs = W.scan_runs(count=count)
    steps = [max(1, int(round(c["steps"] * steps_scale))) for c in cfgs]
    work = sum(W.active_cells(c) * n for c, n in zip(cfgs, steps))
    # tile shapes: one tuning run per power-of-two size class of the 2D runs
    classes = {}
    for c in cfgs:
        if int(c["n"][1]) > 1:
            classes.setdefault(tuple(int(math.ceil(math.log2(int(v)))) for v in c["n"][:2]), c)
    tuned = {}
    if tune:
        for key, c in sorted(classes.items()):
            t = axf.tune(c, precision=axf.F32, steps=10)
            tuned["%dx%d" % (1 << key[0], 1 << key[1])] = [t["steps_per_pass"], t["chunk"], t["prefetch"],
                                                            t["frame_chunk"]]
    batch = axf.Batch(cfgs, precision=axf.F32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    probe = list(range(0, count, max(1, count // 8)))
    p_batch = {i: batch.runs[i].diag_now()["p_gen"] for i in probe}
    batch.close()
    del batch
    torch.cuda.empty_cache()
    # one run at a time, each with its own launches
    t_alone = 0.0
    p_alone = {}
    for i, (c, n) in enumerate(zip(cfgs, steps)):
        run = axf.Run(c, precision=axf.F32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.step(n)
        run.sync()
        t_alone += time.perf_counter() - t0
        if i in probe:
            p_alone[i] = run.diag_now()["p_gen"]
        run.close()
        del run
    torch.cuda.empty_cache()
    return {"runs": count, "steps_scale": steps_scale, "cell_updates": work,
            "batched": round(work / t_batch / 1e9, 3), "per_run": round(work / t_alone / 1e9, 3),
            "unit": "Gcell-updates/s", "speedup": round(t_alone / t_batch, 3),
            "batched_s": round(t_batch, 3), "per_run_s": round(t_alone, 3),
            "p_bitwise_equal": all(p_batch[i] == p_alone[i] for i in probe),
            "tuned_steps_chunk_prefetch_frame": tuned}


def percentile(v, q):
    v = sorted(v)
    if not v:
        return None
    k = min(len(v) - 1, max(0, int(round(q / 100.0 * (len(v) - 1)))))
    return v[k]


def serve_leg(axf, torch, rates, count, steps_scale, pool_gb, max_slots=64, macro=16, with_fifo=True):
    """Poisson arrivals of conversion requests (90% like the scan, 10% 3D
    128^3-256^3), served by the continuous-batching server and, for the same
    trace, one request at a time in arrival order (per-request launches).
    Latency = completion - arrival, reported for all requests and for the
    1D/2D ("small") and 3D requests apart."""
    from paper_2406_16796_amd import workloads as W

    def stats(lat, kinds, span, work):
        small = [v for v, k in zip(lat, kinds) if k < 3]
        r4 = lambda v: None if v is None else round(v, 4)
        out = {"Gcell_s": round(work / span / 1e9, 3), "req_s": round(len(lat) / span, 2),
               "p50_s": r4(percentile(lat, 50)), "p99_s": r4(percentile(lat, 99)),
               "small_p50_s": r4(percentile(small, 50)), "small_p99_s": r4(percentile(small, 99))}
        for d in (1, 2, 3):
            cls = [v for v, k in zip(lat, kinds) if k == d]
            out["%dd_p50_s" % d] = r4(percentile(cls, 50))
            out["%dd_p99_s" % d] = r4(percentile(cls, 99))
        return out

    last = [0.0]

    def progress(label, done, total, t0):
        t = time.perf_counter() - t0
        if done % 50 == 0 or done == total or t - last[0] > 15.0:
            last[0] = t
            print("serving %s: %d/%d done at %.1f s" % (label, done, total, t), file=sys.stderr, flush=True)

    out = []
    for rate in rates:
        trace = W.serving_requests(count=count, rate=rate)
        reqs = [(t, c, max(1, int(round(c["steps"] * steps_scale)))) for t, c in trace]
        ndim = [sum(1 for v in c["n"] if v > 1) for _, c, _ in reqs]
        work = sum(W.active_cells(c) * n for _, c, n in reqs)
        srv = axf.Server(int(pool_gb * (1 << 30)), max_slots=max_slots, macro_steps=macro)
        lat, kinds, ids = [], [], {}
        t0 = time.perf_counter()
        i = 0
        while len(lat) < len(reqs):
            now = time.perf_counter() - t0
            while i < len(reqs) and reqs[i][0] <= now:
                ids[srv.submit(reqs[i][1], reqs[i][2])] = i
                i += 1
            for r in srv.poll():
                if r["status"] != 0:
                    raise SystemExit("served request failed with status %d" % r["status"])
                lat.append(r["t_done"] - r["t_submit"])
                kinds.append(ndim[ids[r["id"]]])
                progress("server %g req/s" % rate, len(lat), len(reqs), t0)
            time.sleep(0.0005)
        span = time.perf_counter() - t0
        srv.close()
        del srv
        torch.cuda.empty_cache()
        point = {"offered_req_s": rate, "requests": len(reqs), "cell_updates": work,
                 "server": stats(lat, kinds, span, work)}
        print("serving %g req/s, server: %s" % (rate, json.dumps(point["server"])), file=sys.stderr, flush=True)
        if not with_fifo:
            out.append(point)
            continue
        # the same trace, one request at a time in arrival order
        fifo = []
        t0 = time.perf_counter()
        for t_arr, c, n in reqs:
            now = time.perf_counter() - t0
            if now < t_arr:
                time.sleep(t_arr - now)
            run = axf.Run(c, precision=axf.F32)
            run.step(n)
            run.diag_now()
            fifo.append(time.perf_counter() - t0 - t_arr)
            progress("per-request %g req/s" % rate, len(fifo), len(reqs), t0)
            run.close()
            del run
        fifo_span = time.perf_counter() - t0
        torch.cuda.empty_cache()
        point["fifo_per_request"] = stats(fifo, ndim, fifo_span, work)
        out.append(point)
    return {"steps_scale": steps_scale, "pool_GB": pool_gb, "max_slots": max_slots,
            "slice_cell_updates": macro * (1 << 20), "points": out}


def pmc_rows(path):
    """(kernel name, counter value) per dispatch from a rocprofv3 counter CSV."""
    out = []
    with open(path) as f:
        for row in csv.DictReader(f):
            out.append((row["Kernel_Name"], float(row["Counter_Value"])))
    return out


PROFILE_WARMUP = 4     # steps of the profile-only run before the timed ones (one four-step pass)


def pmc_summary(args):
    """Scale the FETCH_SIZE / WRITE_SIZE readings of the step kernels by the
    readings of the device copy of known size, write the summary file."""
    cfg = workload(args.workload)
    tag = workload_tag(cfg, args.precision)
    kernel, pats = WORKLOADS[args.workload][1], step_patterns(args.workload, args.precision)
    nsteps = args.steps + PROFILE_WARMUP
    res = {}
    for counter, path in (("FETCH_SIZE", args.pmc_summary[0]), ("WRITE_SIZE", args.pmc_summary[1])):
        rows = pmc_rows(path)
        copy = [v for k, v in rows if "neg" in k.lower()]
        if not copy:
            raise SystemExit("no copy dispatches in %s" % path)
        kib_copy = max(copy)
        factor = COPY_BYTES / (kib_copy * 1024.0)
        # every dispatch of a step kernel over the whole run, per step
        per = {}
        for pat in pats:
            vals = [v for k, v in rows if pat in k.replace(" ", "")]
            per[pat] = (len(vals), sum(vals))
        if not any(n for n, _ in per.values()):
            raise SystemExit("no step-kernel dispatches in %s" % path)
        kib_step = sum(t for _, t in per.values()) / nsteps
        res[counter] = (kib_copy, factor, kib_step, per, kib_step * 1024.0 * factor)
    ndim = sum(1 for v in cfg["n"] if v > 1)
    esize = 4 if args.precision == "f32" else 8
    nc = int(cfg["n"][0]) * int(cfg["n"][1]) * int(cfg["n"][2])
    algo = words_per_cell(ndim) * esize * nc
    traffic = res["FETCH_SIZE"][4] + res["WRITE_SIZE"][4]
    cmd = "python3 $REPO/bench.py --profile-only --workload %s --precision %s --steps %d" % (
        args.workload, args.precision, args.steps)
    disp = ", ".join("%s x%d" % (pattern_label(p), n) for p, (n, _) in res["FETCH_SIZE"][3].items() if n)
    lines = ["# HBM traffic of %s, workload %s" % (kernel, tag), "",
             "Two rocprofv3 counter passes over `%s` (the device copy of %d bytes read and %d written, then "
             "%d steps of the default path: %s):" % (cmd.replace("$REPO/", ""), COPY_BYTES, COPY_BYTES, nsteps, disp),
             "",
             "    cd /tmp && export TMPDIR=/tmp",
             "    timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -d $OUT/fetch -o fetch --output-format csv -- " + cmd,
             "    timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -d $OUT/write -o write --output-format csv -- " + cmd,
             "    python3 $REPO/bench.py --workload %s --precision %s --steps %d --pmc-summary "
             "<fetch counter_collection.csv> <write counter_collection.csv>"
             % (args.workload, args.precision, args.steps), "",
             "| counter | copy kernel KiB | scale (bytes per KiB read) | step kernels KiB per step (all dispatches / %d steps) | bytes per step |"
             % nsteps,
             "|---|---|---|---|---|"]
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        kc, fac, ks, _, b = res[counter]
        lines.append("| %s | %.0f | %.4f x 1024 | %.0f | %.4g |" % (counter, kc, fac, ks, b))
    lines += ["",
              "Algorithmic bytes per step: %d words x %d B x %d cells = %.4g B; measured / algorithmic = %.3f."
              % (words_per_cell(ndim), esize, nc, algo, traffic / algo), "",
              "- `traffic_bytes_per_launch = %.6g`" % traffic,
              "- `algorithmic_bytes_per_launch = %d`" % algo,
              "- `kernel_source_sha256 = %s`" % kernel_source_hash(args.workload), ""]
    path = traffic_file(tag, kernel)
    with open(path, "w") as f:
        f.write("\n".join(lines))
    print(path)


def trace_summary(args):
    """Per-kernel call count and mean duration from a rocprofv3 kernel_stats CSV."""
    cfg = workload(args.workload)
    tag = workload_tag(cfg, args.precision)
    kernel, pats = WORKLOADS[args.workload][1], step_patterns(args.workload, args.precision)
    rows = list(csv.DictReader(open(args.trace_summary)))
    cmd = ("python3 $REPO/bench.py --workload %s --precision %s --steps %d --warmup %d --plain-steps %d "
           % (args.workload, args.precision, args.steps, args.warmup, args.plain_steps)) + (
        "--profile-only" if args.workload in ("fps", "window") else
        "--no-cpu-baseline --no-scan --no-serve --no-2d --no-1d --no-fps --no-window --no-tune")
    lines = ["# Kernel trace of bench.py, workload %s" % tag, "",
             "    cd /tmp && export TMPDIR=/tmp",
             "    timeout -k 10 300 rocprofv3 --kernel-trace --stats -d $OUT/kt -o kt --output-format csv -- " + cmd,
             "    python3 $REPO/bench.py --workload %s --precision %s --steps %d --warmup %d --plain-steps %d "
             "--trace-summary $OUT/kt/kt_kernel_stats.csv"
             % (args.workload, args.precision, args.steps, args.warmup, args.plain_steps), "",
             ("The run steps the workload once: the fused 2D passes, broken at every move of the window "
              "(every 8 columns the light crosses).  A move is `k_win_xghosts<T>` (the x-face ghosts after "
              "the move, one thread per face point) and `k_win_rows<T, R>` (every array's rows shifted left "
              "in place, a row per workgroup of 256 threads through R registers each).  The copy kernel is "
              "the bandwidth calibration.  " if args.workload == "window" else
              "The run steps the workload once (the particle path: unfused field phases and the particle "
              "kernels), first to the late window (the pulse centre three quarters of the way across the "
              "grid, %d steps) and then the profiled steps; the table covers every call, the figures "
              "below it the last %d calls of each kernel (the late window).  The copy kernel is the "
              "bandwidth calibration.  " % (fps_late_start(cfg), args.steps) if args.workload == "fps" else
              "The run times the fused path twice (with and without diagnostics) and the unfused phase "
              "sequence once; the copy kernel is the bandwidth calibration.  ") + (
                 "In 3D one step is `k_march3d<T, NW, 0>` over the interior box (every workgroup clear "
                 "of the faces), `k_march3d<T, NW, 1>` over the columns at both x faces (one wavefront "
                 "per row holds both faces) and "
                 "`k_march3d<T, NW, 2>` over the rest of the boundary frame; the last two run beside "
                 "the first on a second stream, so their durations overlap and the step time is the "
                 "span of the three."
                 if args.workload == "3d" else
                 "With particles a step is the unfused field phases (`k_e0`, `k_c`, `k_e1`, `k_mur`, `k_b`, "
                 "`k_phi`), then `k_jzero<T>` clearing the current arrays and `k_push<T>` (one thread per "
                 "particle: the push, its first-order derivative, the atomic deposit of both currents)."
                 if args.workload == "fps" else
                 "In 2D a pass of NS steps is `k_wave2d_pass<T, PD, NS, MODE>` over the interior with NS "
                 "`k_wave2d` launches over the boundary frame beside it on a second stream.  A pass of three "
                 "or four steps splits its interior into a core launch (MODE 1) and a ring launch (MODE 2, on "
                 "a third stream, storing the intermediate steps the frame launches read); a two-step pass is "
                 "one launch (MODE 0)."), "",
             "| kernel | calls | mean us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"].replace("(anonymous namespace)::", "")
        short = name.split("(")[0].replace("void ", "")
        if len(short) > 70:
            short = short[:67] + "..."
        lines.append("| `%s` | %s | %.1f | %.1f | %.1f | %.2f |" % (
            short, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))
    lines.append("")
    modes = {"0": "", "1": " core", "2": " ring"}
    tpath = os.path.join(os.path.dirname(args.trace_summary),
                         os.path.basename(args.trace_summary).replace("kernel_stats", "kernel_trace"))
    late = {}
    if args.workload == "fps":
        # the last args.steps dispatches of each step kernel (the late window)
        disp = {pat: [] for pat in pats}
        for r in csv.DictReader(open(tpath)):
            name = r["Kernel_Name"].replace(" ", "")
            for pat in pats:
                if pat in name:
                    disp[pat].append((int(r["Correlation_Id"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
        for pat, d in disp.items():
            d = [ns for _, ns in sorted(d)[-args.steps:]]
            if d:
                late[pat] = (sum(d) / len(d), len(d))
    for pat in pats:
        dom = [r for r in rows if pat in r["Name"].replace(" ", "")]
        if pat in late:
            lines.append("- `%s_mean_us = %.2f` (the last %d calls)" % (pattern_label(pat), late[pat][0] / 1e3,
                                                                       late[pat][1]))
        elif dom:
            lines.append("- `%s_mean_us = %.2f`" % (pattern_label(pat), float(dom[0]["AverageNs"]) / 1e3))
        for r in dom:
            m = re.search(r"k_wave2d_pass<\w+,\d+,(\d+),(\d+)>", r["Name"].replace(" ", ""))
            if m:
                ns = int(m.group(1))
                lines.append("- `%s_mean_us_per_step = %.2f` (%s calls, a launch of the%s interior advances "
                             "%d steps)" % (pattern_label(pat), float(r["AverageNs"]) / 1e3 / ns, r["Calls"],
                                            modes.get(m.group(2), ""), ns))
    if args.workload == "window":
        dom = [r for r in rows if pats[0] in r["Name"].replace(" ", "")]
        if dom:
            nbytes = 2 * WINDOW_WORDS_2D * 4 * window_points(cfg)
            us = float(dom[0]["AverageNs"]) / 1e3
            lines.append("- `bytes_per_move = %d` (%d words of each of %d points, read and written)"
                         % (nbytes, WINDOW_WORDS_2D, window_points(cfg)))
            gbs = nbytes / us / 1e3
            lines.append("- `move_GBs = %.1f` = %.1f%% of %.0f GB/s" % (gbs, 100.0 * gbs / HBM_PEAK_GBS, HBM_PEAK_GBS))
    if args.workload == "3d":
        # the x-face and frame launches run beside the interior one, so their
        # durations overlap: a step is the span from the first start to the
        # last end of its three dispatches (consecutive correlation ids)
        if os.path.exists(tpath):
            disp = []
            for r in csv.DictReader(open(tpath)):
                name = r["Kernel_Name"].replace(" ", "")
                k = [i for i, pat in enumerate(pats) if pat in name]
                if k:
                    disp.append((int(r["Correlation_Id"]), k[0], int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
            disp.sort()
            spans, cur = [], []
            for d in disp:
                if d[1] == 0 and cur:
                    spans.append(max(e for *_, e in cur) - min(b for _, _, b, _ in cur))
                    cur = []
                cur.append(d)
            if cur:
                spans.append(max(e for *_, e in cur) - min(b for _, _, b, _ in cur))
            if spans:
                lines.append("- `step_span_mean_us = %.2f` over %d steps (first start to last end of the three "
                             "launches of a step; the sum of their mean durations exceeds it because they overlap)"
                             % (sum(spans) / len(spans) / 1e3, len(spans)))
    lines.append("- `kernel_source_sha256 = %s`" % kernel_source_hash(args.workload))
    path = os.path.join(ROOT, "profiles", "%s_%s_kernel_trace.md" % (kernel, tag))
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="3d", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--diag-every", type=int, default=100)
    ap.add_argument("--plain-steps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-only", action="store_true")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--trace-summary", metavar="KERNEL_STATS_CSV")
    ap.add_argument("--no-scan", action="store_true")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2D 4096^2 leg")
    ap.add_argument("--no-1d", action="store_true", help="skip the 1D 4096-cell leg")
    ap.add_argument("--no-fps", action="store_true", help="skip the weak-laser plasma (particles) leg")
    ap.add_argument("--no-window", action="store_true", help="skip the moving-window leg")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in launch shapes")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--steps-scale", type=float, default=0.1,
                    help="step counts of the scan and serving legs relative to the workload's 1000-5000")
    ap.add_argument("--serve-rates", default="8,32,128")
    ap.add_argument("--serve-requests", type=int, default=100)
    ap.add_argument("--serve-no-fifo", action="store_true",
                    help="serve only (no one-request-at-a-time pass over the same trace)")
    ap.add_argument("--serve-slice", type=int, default=256,
                    help="server work slice per run and round, in units of 2^20 cell-updates")
    args = ap.parse_args()
    if args.gpus != 1:
        print("the benchmark runs on one GPU only (--gpus %d requested): the step is a single-GPU kernel; "
              "slab sharding across GPUs is a design, not code" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.pmc_summary:
        pmc_summary(args)
        return
    if args.trace_summary:
        trace_summary(args)
        return

    import torch
    from paper_2406_16796_amd import axf
    torch.cuda.set_device(0)
    cfg = workload(args.workload)
    prec = axf.F32 if args.precision == "f32" else axf.F64
    esize = 4 if prec == axf.F32 else 8
    ndim = sum(1 for v in cfg["n"] if v > 1)
    nc = int(cfg["n"][0]) * int(cfg["n"][1]) * int(cfg["n"][2])
    tag = workload_tag(cfg, args.precision)
    kernel, pats = WORKLOADS[args.workload][1], step_patterns(args.workload, args.precision)

    copy_gbs = device_copy(torch)
    tuned = None
    if args.workload == "2d" and not args.no_tune and not args.profile_only:
        axf.tune_reset()
        tuned = axf.tune(cfg, precision=prec, steps=40)
    if args.profile_only:
        # the particle workload is profiled in its late window (see leg_fps)
        warm = fps_late_start(cfg) if args.workload == "fps" else PROFILE_WARMUP
        time_path(axf, torch, cfg, prec, axf.PATH_AUTO, args.steps, warm, 0)
        print(json.dumps({"profile_only": tag, "steps": args.steps}), flush=True)
        return

    # whole hot path: step + diagnostics at the configured cadence
    wall, _, _, rec, fused = time_path(axf, torch, cfg, prec, axf.PATH_AUTO, args.steps, args.warmup,
                                       args.diag_every)
    value = nc * args.steps / wall / 1e9
    # the step kernels alone (no diagnostics): HIP events on the run's stream
    # around the timed steps (in 3D one step is the interior launch followed by
    # the boundary-frame launch; in 2D a pass of several steps is the interior
    # launch with the frame launches beside it on a second stream)
    _, k_ms, k_launches, _, _ = time_path(axf, torch, cfg, prec, axf.PATH_AUTO, args.steps, 2, 0)
    per_step_s = k_ms / 1e3 / args.steps
    algo_bytes = words_per_cell(ndim) * esize * nc
    achieved = algo_bytes / per_step_s / 1e9
    # the counter summary was taken with the built-in launch shape
    default_shape = DEFAULT_WAVE_SHAPE[args.precision]
    same_shape = tuned is None or (tuned["steps_per_pass"], tuned["chunk"], tuned["prefetch"],
                                   tuned["frame_chunk"]) == default_shape
    traffic = read_traffic(args.workload, tag, kernel) if fused and same_shape else None
    # 3D FP64 runs step through the merged tile walks, not the march
    tiles = args.workload == "3d" and args.precision == "f64"
    # the unfused phase sequence for comparison
    p_wall, _, p_launches, _, _ = time_path(axf, torch, cfg, prec, axf.PATH_PLAIN, args.plain_steps, 2, 0)
    plain_value = nc * args.plain_steps / p_wall / 1e9

    line = {
        "metric": "Gcell-updates/s + % HBM roofline (fused vs plain); p50/p99 latency of served scans",
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
            "workload": tag, "ndim": ndim, "n": cfg["n"], "dx": cfg["dx"][0], "dt": cfg["dt"],
            "m": cfg["m"], "g": cfg["g"], "em_bc": "mur", "axion_bc": cfg["ax_bc"][0],
            "diag_every": args.diag_every, "path": "fused" if fused else "plain",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": round(traffic) if traffic is not None else None,
            "kernel": ("merged tile-walk launches (k3_tile<3,double,...>, k_mur<3,double>)" if tiles else
                       " + ".join(pattern_label(p) for p in pats)) if fused else "plain phase sequence",
            "unit_of_work": "one step of the whole grid (%s)" % (
                "the tile-walk launches" if tiles else
                "interior, x-face and frame launches" if args.workload == "3d" else "fused launches"),
            "bytes_per_step": algo_bytes, "launches_per_step": round(k_launches / args.steps, 3),
            "mean_step_ms": round(per_step_s * 1e3, 5), "steps_timed": args.steps,
            "traffic_over_algorithmic": round(traffic / algo_bytes, 3) if traffic is not None else None,
            "copy_kernel_GBs": round(copy_gbs, 1),
            "tuned": None if tuned is None else {"steps_per_pass": tuned["steps_per_pass"],
                                                 "chunk": tuned["chunk"], "prefetch": tuned["prefetch"],
                                                 "frame_chunk": tuned["frame_chunk"],
                                                 "candidates": tuned["candidates"],
                                                 "best_ms": round(tuned["ms_per_step"], 4),
                                                 "default_ms": round(tuned["default_ms_per_step"], 4)},
        },
        "plain": {"value": round(plain_value, 3), "unit": "Gcell-updates/s",
                  "ms_per_step": round(p_wall / args.plain_steps * 1e3, 4),
                  "launches_per_step": round(p_launches / max(args.plain_steps, 1), 2),
                  "fused_speedup": round(value / plain_value, 3) if plain_value > 0 else None},
        "diag": {"step": rec["step"], "p_gen": rec["p_gen"], "p_conv": rec["p_conv"], "finite": rec["finite"]},
    }
    if not args.no_2d:
        if args.workload == "2d":
            other = "f64" if args.precision == "f32" else "f32"
            line[other] = leg_2d(axf, torch, other)
        else:
            line["2d"] = {p: leg_2d(axf, torch, p) for p in ("f32", "f64")}
    if not args.no_1d and args.workload != "1d":
        line["1d"] = leg_1d(axf, torch)
    if not args.no_fps and args.workload != "fps":
        line["fps"] = leg_fps(axf, torch)
    if not args.no_window and args.workload != "window":
        line["window"] = leg_window(axf, torch)
    if not args.no_scan:
        line["scan"] = scan_leg(axf, torch, args.steps_scale, tune=not args.no_tune)
    if not args.no_serve:
        rates = [float(v) for v in args.serve_rates.split(",") if v]
        line["serving"] = serve_leg(axf, torch, rates, args.serve_requests, args.steps_scale, pool_gb=64,
                                    macro=args.serve_slice, with_fifo=not args.serve_no_fifo)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

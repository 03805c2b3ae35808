#!/usr/bin/env python3
"""Benchmark of the exact occlusion detector on one MI355X.

Headline workload (one "step"): one batched launch of 64 fp32 disparity maps
of mixed size (640x480, 1280x960, 1920x1080, 2048x1536; seed 3000), each
with the 8 peripheral views of a 3x3 camera array (axis views r = 1,
diagonal views r = sqrt(2)), c1 scene statistics (objects with disparity in
[0, 48], noise 0.1 px), per-frame L_v = ceil(max(D) * r_v) + 2, gamma = 1,
beta = 0.5, zeta = 1, N = 1: edges + candidates (Eqs. 1-2), scanlines, warp,
sort, occlusion test and mask (Eqs. 4-6) of every frame and view in one
graph launch.  D and M stay resident in HBM.

Prints ONE JSON line.  `value` is Mpixel-views/s of the whole batch;
`roofline` describes the dominant kernel (the batched scanline pass) timed
with HIP events on the library's stream; `cpu_baseline` is the CPU oracle on
the host cores over (frame, view) jobs of the same workload.  Secondary
sections: single 1280x960 frames with frames in flight (c1), one 3840x2160
frame with 15 views (c2), 1920x1080 frames (c4, exact and learned), quality,
fusion, thinning and the paper's Table 3 shape as context.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PREWARM_STEPS = 1000  # default untimed steps before the first timed region (see main)
METRIC = "Mpixel-views/s occlusion masks (exact vs CNN+fallback @IoU≥0.99), HBM GB/s"
HBM_PEAK_GBPS = 8000.0
# 32-bit VALU lane operations: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
ALU_PEAK_GOPS = 256 * 4 * 16 * 2.4
PAPER_GPU_MPVS = 1600 * 1200 * 8 / 0.026 / 1e6   # Table 3, RTX 3090, 1600x1200 x 8 directions
CSRC = "paper_2408_14050_amd/csrc/"


def kernel_source(kernel: str) -> str:
    if kernel.startswith(("k_conv", "k_pack", "k_bce", "k_adam", "k_wgrad", "k_dgrad", "k_reduce",
                          "k_transpose_w")):
        return CSRC + "k_cnn.hip"
    if kernel.startswith(("k_route", "k_stats", "k_confusion", "k_zbuf", "k_fill", "k_median",
                          "k_edges_out")):
        return CSRC + "k_util.hip"
    return CSRC + "k_exact.hip"


def kernel_hash(kernel: str = "k_scanlines") -> str:
    """First 16 hex digits of the SHA-256 of the kernel's source file."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, kernel_source(kernel)), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def scan_kernels(scan_len):
    """Names of the scanline-pass kernels a plain exact-path frame launches:
    one per register class of its views (K = 2, 4, 8, 16 samples per lane for
    n = 2h + 1 samples, K <= 2 sharing the first); the second template
    argument 0 is the form without the bilinear / routed-tile checks."""
    out = []
    for L in scan_len:
        n = 2 * (int(L) // 2) + 1
        K = 1
        while 64 * K < n:
            K *= 2
        name = f"k_scanlines<{max(K, 2)}, 0>"
        if name not in out:
            out.append(name)
    return out


def scanline_ops(n_cand, scan_len, neighbours=1):
    """Algorithmic work of Eqs. (4)-(6): per scanline of n samples a
    comparison sort (n * ceil(log2 n) key comparisons) and 2 * n_s * n
    neighbour tests."""
    ns = max(1, (neighbours + 1) // 2)
    tot = 0
    for c, L in zip(n_cand, scan_len):
        n = 2 * (int(L) // 2) + 1
        tot += int(c) * (n * max(1, math.ceil(math.log2(n))) + 2 * ns * n)
    return tot


def traffic_for(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(traffic_key(kernel, workload), {})
    if e.get("kernel_hash") != kernel_hash(kernel) or e.get("workload") != workload:
        return None
    return e.get("bytes_per_launch")


def traffic_key(kernel: str, workload: str) -> str:
    """Entry of profiles/traffic.json: one per kernel and workload."""
    return f"{kernel} @ {workload}"


def host_cpu():
    """nproc, the threads this process may use (the job's share of the host)
    and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable": usable, "model": model}


def cpu_baseline(frames, seconds: float, max_threads: int = 16):
    """The CPU oracle, unchanged and single-threaded per call, on the
    headline workload for a bounded time:
      all cores: independent (frame, view) jobs of the batch, dealt to a
        thread pool (ctypes releases the GIL) of the host's usable threads,
        capped at the job's share of 16;
      one core: whole frames, all views in one oracle call (Eq. (1) once per
        frame).
    Throughput is the pixel-views of the completed jobs over the elapsed
    time."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import occl_ref

    cpu = host_cpu()
    threads = max(1, min(max_threads, cpu["usable"]))
    jobs = [(f, v) for f in frames for v in range(f.n_views)]

    def one(job):
        f, v = job
        p = f.params
        occl_ref.detect(f.D, f.angles[v:v + 1], f.ratios[v:v + 1], f.scan_len[v:v + 1], p["edge_thr"],
                        p["disp_thr"], p["dist_thr"], p["neighbours"])
        return f.H * f.W

    t0 = time.perf_counter()
    pv1, n1 = 0, 0
    while time.perf_counter() - t0 < seconds / 3:
        f = frames[n1 % len(frames)]
        p = f.params
        occl_ref.detect(f.D, f.angles, f.ratios, f.scan_len, p["edge_thr"], p["disp_thr"],
                        p["dist_thr"], p["neighbours"])
        pv1 += f.pixel_views
        n1 += 1
    t1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    pvn, nj = 0, 0
    with ThreadPoolExecutor(threads) as ex:
        while time.perf_counter() - t0 < 2 * seconds / 3:
            chunk = [jobs[(nj + i) % len(jobs)] for i in range(4 * threads)]
            pvn += sum(ex.map(one, chunk))
            nj += len(chunk)
    tn = time.perf_counter() - t0
    return {
        "value": round(pvn / tn / 1e6, 3), "unit": "Mpixel-views/s", "cores": threads,
        "kind": "oracle",
        "sample": f"{nj} (frame, view) jobs of the 64-frame batch (seed 3000), one view per oracle "
                  f"call, on {threads} threads in {tn:.1f} s",
        "host": cpu,
        "single_thread": {"value": round(pv1 / t1 / 1e6, 3), "cores": 1,
                          "sample": f"{n1} whole frames of the batch (all 8 views per call) in {t1:.1f} s"},
    }


def bitonic_ops(n_cand, scan_len, neighbours=1):
    """Algorithmic ALU work of Eqs. (4)-(6), counted as a sorting network
    would do it: per scanline of n samples a bitonic sort of
    n' = 2^ceil(log2 n) keys,
    (n'/2) log2 n' (log2 n' + 1) / 2 compare-exchanges, plus 2 n_s n
    neighbour tests."""
    ns = max(1, (neighbours + 1) // 2)
    tot = 0
    for c, L in zip(n_cand, scan_len):
        n = 2 * (int(L) // 2) + 1
        lg = max(1, math.ceil(math.log2(n)))
        tot += int(c) * ((1 << lg) // 2 * lg * (lg + 1) // 2 + 2 * ns * n)
    return tot


# ---------------------------------------------------------------------------
# profiling helpers (run under rocprofv3 on the GPU, summarised here)
# ---------------------------------------------------------------------------
PROFILE_CMD = ("rocprofv3 {mode} -d gpurun_out/{out} -o run -- python3 bench.py --steps 20 "
               "--warmup 2 --prewarm-batched 0 --prewarm 0 --c1-steps 20 --streams 1 --no-c2 "
               "--no-cpu-baseline --no-context --no-check --no-learned --no-quality")
QUALITY_PROFILE_CMD = ("rocprofv3 {mode} -d gpurun_out/{out} -o run -- python3 bench.py "
                       "--quality-only")
THIN_PROFILE_CMD = "rocprofv3 {mode} -d gpurun_out/{out} -o run -- python3 bench.py --thin-only"
LEARNED_PROFILE_CMD = ("rocprofv3 {mode} -d gpurun_out/{out} -o run -- python3 bench.py --learned-only "
                       "--learned-steps 10 --learned-eval 1 --no-train-step")
TRAIN_PROFILE_CMD = ("rocprofv3 {mode} -d gpurun_out/{out} -o run -- python3 bench.py --train-only "
                     "--train-steps 10")
TRAIN_WORKLOAD = "training step 128 crops 256x256 x8 channels"
TRAIN_KERNELS = ("k_conv_fwd_p", "k_conv_last", "k_conv_wgrad", "k_conv_dgrad", "k_reduce_groups",
                 "k_reduce_chunks", "k_wgrad_last", "k_dgrad_last", "k_adam", "k_bce",
                 "k_transpose_w")
BATCH_WORKLOAD = "c3 64 mixed frames seed 3000"
C1_WORKLOAD = "c1 1280x960 x8 views seed 1002"
C2_WORKLOAD = "c2 3840x2160 x15 views seed 2000"
FUSED_KERNEL = "k_fused<16>"  # the fused pass at its tile height (rows per tile)
C2_PROFILE_CMD = "rocprofv3 {mode} -d gpurun_out/{out} -o run -- python3 bench.py --c2-only --c2-steps 5"
C2_KERNELS = ("k_edges", "k_scanlines<4, 0>", "k_scanlines<8, 0>")
QUALITY_WORKLOAD = "c1 1280x960 x8 views seeds 1000-1003"
LEARNED_WORKLOAD = "c4 1920x1080 x8 views seed 4100"
THIN_WORKLOAD = "c1 1280x960 x8 views seed 1002 thinned"
THIN_KERNELS = ("k_scanlines<2, 1>",)
LEARNED_KERNELS = ("k_pack", "k_conv", "k_route")
QUALITY_KERNELS = ("k_zbuf", "k_fill", "k_median", "k_confusion", "k_stats")
COPY_CMD = "rocprofv3 --pmc {ctr} -d gpurun_out/{out} -o run -- python3 bench.py --copy-probe 256"


def copy_probe(mib: int) -> int:
    """A plain device-to-device copy of `mib` MiB: calibrates the HBM byte
    counters (FETCH_SIZE / WRITE_SIZE) against a known amount of traffic."""
    import torch
    a = torch.ones(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_mib": mib}))
    return 0


def _pmc_per_kernel(db_path: str, counter: str):
    import re
    import sqlite3
    con = sqlite3.connect(db_path)
    rows = con.execute("select name, dispatch_id, sum(counter_value) from pmc_events "
                       "where counter_name = ? group by name, dispatch_id", (counter,)).fetchall()
    out = {}
    for name, _, val in rows:
        m = re.search(r"(k_[a-z_0-9]+(<[0-9, ]+>)?)", name)
        key = m.group(1) if m else name.split("(")[0][-40:]
        out.setdefault(key, []).append(val)
    return {k: sum(v) / len(v) for k, v in out.items()}


def _trace_per_kernel(db_path: str):
    import re
    import sqlite3
    con = sqlite3.connect(db_path)
    tabs = [r[0] for r in con.execute("select name from sqlite_master where type in ('table','view')")]
    tab = "kernels" if "kernels" in tabs else [t for t in tabs if t.startswith("rocpd_kernel_dispatch")][0]
    cols = [r[1] for r in con.execute(f"pragma table_info({tab})")]
    name_col = "name" if "name" in cols else "kernel_name"
    grid = "grid_x" if "grid_x" in cols else None
    rows = con.execute(f"select {name_col}, start, end, {grid or 0} from {tab}").fetchall()
    out, by_grid = {}, {}
    for name, st, en, gx in rows:
        m = re.search(r"(k_[a-z_0-9]+(<[0-9, ]+>)?)", name or "")
        key = m.group(1) if m else (name or "?").split("(")[0][-40:]
        out.setdefault(key, []).append((en - st) / 1e3)
        by_grid.setdefault(key, {}).setdefault(int(gx or 0), []).append((en - st) / 1e3)
    return {k: {"calls": len(v), "avg_us": sum(v) / len(v), "min_us": min(v), "max_us": max(v),
                "by_grid": {g: (len(d), sum(d) / len(d)) for g, d in sorted(by_grid[k].items())}}
            for k, v in out.items()}


def profiles_from(run_dir: str, workload: str) -> int:
    """Writes profiles/<kernel>__<workload>.txt and profiles/traffic.json from
    the rocprofv3 databases of the profiling runs: trace, FETCH_SIZE and
    WRITE_SIZE passes of the benchmark (prof, pmc_fetch, pmc_write), of its
    learned, quality, thinning, c2 and training sections (l-, q-, t-, c- and
    r-prefixed; optional)
    and of the copy probe (copy_fetch, copy_write)."""
    import glob
    def db(sub):
        g = glob.glob(os.path.join(run_dir, sub, "*.db"))
        return g[0] if g else None
    cf = _pmc_per_kernel(db("copy_fetch"), "FETCH_SIZE")
    cw = _pmc_per_kernel(db("copy_write"), "WRITE_SIZE")
    copy_kib = 256 * 1024
    f_read = max(cf.values()) / copy_kib if cf else None
    f_write = max(cw.values()) / copy_kib if cw else None
    traffic = {}
    try:  # entries of runs not present here are kept
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
            traffic = json.load(f)
    except (OSError, ValueError):
        pass
    traffic["copy_probe"] = {"mib": 256, "fetch_kib": max(cf.values()) if cf else None,
                              "write_kib": max(cw.values()) if cw else None,
                              "read_factor": f_read, "write_factor": f_write}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    runs = [("", PROFILE_CMD, lambda k: not k.startswith(LEARNED_KERNELS + QUALITY_KERNELS)),
            ("l", LEARNED_PROFILE_CMD, lambda k: k.startswith(LEARNED_KERNELS)),
            ("q", QUALITY_PROFILE_CMD, lambda k: k.startswith(QUALITY_KERNELS)),
            ("t", THIN_PROFILE_CMD, lambda k: k.startswith(THIN_KERNELS)),
            ("c", C2_PROFILE_CMD, lambda k: k.startswith(C2_KERNELS)),
            ("r", TRAIN_PROFILE_CMD, lambda k: k.startswith(TRAIN_KERNELS))]
    for pre, cmd, keep in runs:
        if not db(pre + "prof"):
            continue
        trace = _trace_per_kernel(db(pre + "prof"))
        fetch = _pmc_per_kernel(db(pre + "pmc_fetch"), "FETCH_SIZE")
        write = _pmc_per_kernel(db(pre + "pmc_write"), "WRITE_SIZE")
        for k in sorted(k for k in set(trace) & set(fetch) & set(write) if k.startswith("k_") and keep(k)):
            if pre == "l":
                wl = LEARNED_WORKLOAD
            elif pre == "q":
                wl = QUALITY_WORKLOAD
            elif pre == "t":
                wl = THIN_WORKLOAD
            elif pre == "c":
                wl = C2_WORKLOAD
            elif pre == "r":
                wl = TRAIN_WORKLOAD
            else:
                wl = BATCH_WORKLOAD if any(x in k for x in ("batched", "finish_frames", "k_fused",
                                                           "k_clear_masks")) else workload
            tag = wl.split(":")[0].replace(" ", "_").replace("x8_views", "v8")
            rd = fetch[k] * 1024 / (f_read or 1.0)
            wr = write[k] * 1024 / (f_write or 1.0)
            traffic[traffic_key(k, wl)] = {"kernel_hash": kernel_hash(k), "source": kernel_source(k), "workload": wl,
                          "fetch_kib": fetch[k], "write_kib": write[k], "bytes_per_launch": round(rd + wr),
                          "read_bytes": round(rd), "write_bytes": round(wr),
                          "avg_us": round(trace[k]["avg_us"], 3)}
            lines = [
                f"# {k} -- {wl}",
                "",
                "Commands (from the repository root):",
                "  " + cmd.format(mode="--kernel-trace --stats", out=pre + "prof"),
                "  " + cmd.format(mode="--pmc FETCH_SIZE", out=pre + "pmc_fetch"),
                "  " + cmd.format(mode="--pmc WRITE_SIZE", out=pre + "pmc_write"),
                "  " + COPY_CMD.format(ctr="FETCH_SIZE", out="copy_fetch"),
                "  " + COPY_CMD.format(ctr="WRITE_SIZE", out="copy_write"),
                "  python bench.py --profiles-from gpurun_out   (this summary)",
                "",
                f"kernel source: {kernel_source(k)} (sha256 prefix {kernel_hash(k)})",
                f"dispatches: {trace[k]['calls']}",
                f"duration avg/min/max (us): {trace[k]['avg_us']:.2f} / {trace[k]['min_us']:.2f} / "
                f"{trace[k]['max_us']:.2f}",
                "by grid size (work-items: dispatches, avg us; the autotuner's trial shapes included):",
            ] + [f"  {g}: {c}, {a:.2f}" for g, (c, a) in trace[k]["by_grid"].items()] + [
                f"FETCH_SIZE per dispatch (KiB): {fetch[k]:.1f}",
                f"WRITE_SIZE per dispatch (KiB): {write[k]:.1f}",
                f"copy probe 256 MiB: FETCH_SIZE {traffic['copy_probe']['fetch_kib']} KiB, "
                f"WRITE_SIZE {traffic['copy_probe']['write_kib']} KiB "
                f"(read factor {f_read}, write factor {f_write})",
                f"HBM bytes per dispatch (counters / copy factor): read {rd:.0f}, write {wr:.0f}",
            ]
            name = k.replace("<", "_").replace(">", "").replace(", ", "_").replace(",", "_")
            with open(os.path.join(ROOT, "profiles", f"{name}__{tag}.txt"), "w") as f:
                f.write("\n".join(lines) + "\n")
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
        json.dump(traffic, f, indent=1)
    write_profile_index()
    print(json.dumps(traffic, indent=1))
    return 0


def write_profile_index() -> int:
    """profiles/INDEX.md: one line per summary of profiles/traffic.json
    (workload, kernel, average duration, HBM bytes per dispatch, file), and
    the other summaries in profiles/."""
    import glob
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        traffic = json.load(f)
    rows, listed = [], set()
    for key, e in traffic.items():
        if not isinstance(e, dict) or "workload" not in e:
            continue
        k = key.split(" @ ")[0]
        tag = e["workload"].split(":")[0].replace(" ", "_").replace("x8_views", "v8")
        name = k.replace("<", "_").replace(">", "").replace(", ", "_").replace(",", "_") + f"__{tag}.txt"
        if not os.path.exists(os.path.join(ROOT, "profiles", name)):
            continue
        listed.add(name)
        rows.append((e["workload"], k, e["avg_us"], e["read_bytes"] / 1e6, e["write_bytes"] / 1e6, name))
    lines = ["# rocprofv3 summaries", "",
             "One file per kernel and workload, written by `python bench.py --profiles-from gpurun_out` from the",
             "trace and counter runs whose commands each file lists. Durations are the trace's average per dispatch;",
             "HBM bytes are the FETCH_SIZE and WRITE_SIZE counters per dispatch, scaled by what the same counters",
             "read for a plain copy of known size (`traffic.json` holds the figures and the source hash of each).", "",
             "| workload | kernel | avg µs | HBM read MB | HBM write MB | file |", "|---|---|---|---|---|---|"]
    for wl, k, us, rd, wr, name in sorted(rows):
        lines.append(f"| {wl} | `{k}` | {us:.1f} | {rd:.1f} | {wr:.1f} | [{name}]({name}) |")
    other = sorted(os.path.basename(x) for x in glob.glob(os.path.join(ROOT, "profiles", "*.txt"))
                   if os.path.basename(x) not in listed)
    if other:
        lines += ["", "Other summaries:", ""] + [f"- [{x}]({x})" for x in other]
    with open(os.path.join(ROOT, "profiles", "INDEX.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    return 0


def tune_in_flight(ctxs, run, reps: int = 200):
    """Launch shape for frames in flight, chosen by measured throughput (not
    timed).  The autotuner picks the shape that finishes one frame soonest;
    with several frames in flight a scanline grid that leaves a wavefront
    slot per SIMD to the next frame's edge pass, or another edge-pass block
    height, can move more frames.  Tries the autotuned blocks per CU and a few
    below it, then edge-pass heights around the autotuned one, on every
    context; keeps the fastest and returns it."""
    import tempfile
    import torch
    path = os.path.join(tempfile.gettempdir(), f"occl_tune_{os.getpid()}.txt")
    ctxs[0].occl_tune_save(path)
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    if not rows:
        return None

    def timed(er, bpc):
        with open(path, "w") as f:
            for key, _, _ in rows:
                f.write(f"{key} {er} {bpc}\n")
        for c in ctxs:
            c.occl_tune_load(path)
        run(50)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(reps)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e6

    er0, bpc0 = int(rows[0][1]), int(rows[0][2])
    best = min(((timed(er0, b), er0, b) for b in sorted({bpc0, max(1, bpc0 - 1), max(1, bpc0 - 2),
                                                         2 * bpc0})), key=lambda t: t[0])
    for er in sorted({max(1, er0 // 2), min(16, er0 * 2)} - {er0}):
        t = (timed(er, best[2]), er, best[2])
        best = min(best, t, key=lambda t: t[0])
    timed(best[1], best[2])  # leave the winner loaded
    os.remove(path)
    return {"edge_rows": best[1], "scan_blocks_per_cu": best[2]}


def bench_c3(ctx, args):
    """The headline: 64 frames of mixed size (640x480 .. 2048x1536, c1
    statistics, 8 views, per-frame L) in one graph launch per step."""
    import numpy as np
    import torch
    from paper_2408_14050_amd import occl, scenes
    frames = scenes.make_batch(seed=3000, n_frames=64)
    Ds = [torch.from_numpy(f.D).cuda() for f in frames]
    Ms = [torch.empty((f.n_views, f.H, f.W), dtype=torch.uint8, device="cuda") for f in frames]
    batch = [(D, M, f.scan_len) for D, M, f in zip(Ds, Ms, frames)]
    prm = occl.params(**frames[0].params)
    angles, ratios = frames[0].angles, frames[0].ratios
    shape = None
    if not args.no_tune:  # launch shape chosen by the autotuner (not timed)
        shape = ctx.occl_autotune_batched(batch, angles, ratios, prm, reps=3)
    # untimed pre-warm (the HIP runtime's one-off stall some thousand
    # launches into a process stays out of the timed region)
    for _ in range(max(args.warmup, args.prewarm_batched)):
        ctx.occl_detect_batched(batch, angles, ratios, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.occl_detect_batched(batch, angles, ratios, prm)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dt = elapsed / args.steps
    pv = sum(f.pixel_views for f in frames)
    alg = sum((4 + f.n_views) * f.H * f.W for f in frames)
    # the dominant kernel alone: the batch's stages re-run outside the graph
    # between HIP events on the context's stream
    stages = ctx.occl_time_batched(max(3, min(args.steps, 20)))
    out = {"value": pv * args.steps / elapsed / 1e6, "ms_per_step": dt * 1e3, "pixel_views": pv,
           "alg_bytes": alg, "frames": frames, "masks": Ms, "launch_shape": shape, "stages_ms": stages}
    if stages.get("form") == "fused":
        kern, k_ms, launches = FUSED_KERNEL, stages["fused"], 1
        note = ("algorithmic bytes of the batch (D read once, every mask byte written once) over the "
                "fused pass's time per batch (Eqs. (1)-(6) in one launch; it and the mask fill before "
                "it re-run outside the graph between HIP events)")
    else:
        kern, k_ms, launches = "k_scanlines_batched<2, 0>", stages["scanlines"], ctx_branches()
        note = ("algorithmic bytes of the batch (D read once, every mask byte written once) over "
                "the batched scanline pass's time per batch (its launches re-run outside the "
                "graph, branch after branch, between HIP events)")
    roof = {"kernel": kern, "bound": "hbm",
            "achieved": round(alg / (k_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(alg / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "traffic": None, "avg_ms": round(k_ms, 5), "launches_per_step": launches,
            "bytes_per_step": alg, "note": note}
    t = traffic_for(kern, BATCH_WORKLOAD)
    if t is not None:
        roof["traffic"] = t * launches
    out["roofline"] = roof
    if not args.no_check:
        from concurrent.futures import ThreadPoolExecutor
        from oracle import occl_ref
        with ThreadPoolExecutor(max(1, min(16, host_cpu()["usable"]))) as ex:
            refs = list(ex.map(lambda f: occl_ref.detect_scene(f), frames))
        bad = 0
        n_cand = []
        for (M_ref, _, nc), M in zip(refs, Ms):
            bad += int((M.cpu().numpy() != M_ref).sum())
            n_cand.append(nc)
        out["parity"] = {"frames": len(frames), "mismatches": bad}
        ops = sum(bitonic_ops(nc, f.scan_len) for nc, f in zip(n_cand, frames))
        out["alu"] = {"kernel": kern, "ops_per_step": ops,
                      "count": "bitonic compare-exchanges of 2^ceil(log2 n) keys + 2 n neighbour tests "
                               "per scanline",
                      "achieved_gops": round(ops / (k_ms * 1e-3) / 1e9, 1), "peak_gops": ALU_PEAK_GOPS,
                      "frac": round(ops / (k_ms * 1e-3) / 1e9 / ALU_PEAK_GOPS, 4),
                      "scanlines": int(sum(int(np.sum(nc)) for nc in n_cand))}
    return out


def ctx_branches():
    """Graph branches of a batched launch (the library's default split)."""
    return 2


def bench_c1(args):
    """Single 1280x960 frames (c1, seed args.seed) one at a time and with
    frames in flight on separate streams."""
    import numpy as np
    import torch
    from paper_2408_14050_amd import occl, scenes
    sc = scenes.make_scene("c1", args.seed)
    H, W, V = sc.H, sc.W, sc.n_views
    D = torch.from_numpy(sc.D).cuda()
    M = torch.empty((V, H, W), dtype=torch.uint8, device="cuda")
    ctx = occl.Context(0, max_pixels_hint=H * W, max_views_hint=V)
    prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len)
    steps = args.c1_steps
    tune = None
    if not args.no_tune:
        tune = ctx.occl_autotune(D, sc.angles, sc.ratios, prm, M, reps=20)
    det = ctx.occl_detect_prepared(sc.angles, sc.ratios, prm)
    for _ in range(args.prewarm):
        det(D, M)
    torch.cuda.synchronize()

    def median_ms(fn, n, windows=5):
        """Median over windows of n steps: a one-off host or runtime stall
        (the HIP runtime pauses once some thousand launches into a process)
        must not set the figure."""
        per = []
        for _ in range(windows):
            t0 = time.perf_counter()
            fn(n)
            torch.cuda.synchronize()
            per.append((time.perf_counter() - t0) * 1e3 / n)
        return sorted(per)[len(per) // 2], per

    def single(n):
        for _ in range(n):
            det(D, M)

    single_ms, single_w = median_ms(single, max(1, steps // 5))
    # frames in flight: one context (workspace) and one output per HIP stream
    S = max(1, args.streams)
    fl_streams = [torch.cuda.Stream() for _ in range(S)]
    fl_ctxs = [occl.Context(0, stream=st, max_pixels_hint=H * W, max_views_hint=V) for st in fl_streams]
    fl_Ms = [torch.empty((V, H, W), dtype=torch.uint8, device="cuda") for _ in range(S)]
    fl_Ds = [D.clone() for _ in range(S)]
    torch.cuda.synchronize()
    if not args.no_tune:
        for c, m in zip(fl_ctxs, fl_Ms):
            c.occl_autotune(D, sc.angles, sc.ratios, prm, m, reps=20)
    fl_det = [c.occl_detect_prepared(sc.angles, sc.ratios, prm) for c in fl_ctxs]

    def run(n):
        for i in range(n):
            k = i % S
            fl_det[k](fl_Ds[k], fl_Ms[k])

    fl_shape = None
    if not args.no_tune and S > 1:
        fl_shape = tune_in_flight(fl_ctxs, run)
    run(args.prewarm)
    torch.cuda.synchronize()
    ms_fl, fl_w = median_ms(run, max(1, steps // 5))
    fl_bad = sum(int((m != M).sum().item()) for m in fl_Ms)
    for c in fl_ctxs:
        c.occl_release()
    ctx.occl_profile_enable(True)
    for _ in range(min(steps, 200)):
        ctx.occl_detect(D, sc.angles, sc.ratios, prm, M=M)
    prof = ctx.occl_profile_read()
    ctx.occl_profile_enable(False)
    n_cand = ctx.occl_last_candidate_counts(V)
    scan_rep = ctx.occl_time_scanlines(200)
    alg = (4 + V) * H * W
    out = {"workload": C1_WORKLOAD, "frames_in_flight": S, "in_flight_launch_shape": fl_shape,
           "ms_per_frame": round(ms_fl, 5), "value": round(H * W * V / (ms_fl * 1e-3) / 1e6, 1),
           "windows_ms": [round(x, 5) for x in fl_w],
           "hbm_frac": round(alg / (ms_fl * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
           "single_stream": {"ms_per_frame": round(single_ms, 5),
                             "value": round(H * W * V / (single_ms * 1e-3) / 1e6, 1),
                             "windows_ms": [round(x, 5) for x in single_w]},
           "stages_ms": {k: round(prof[k][0] / max(1, prof[k][1]), 5) for k in ("edges", "scanlines")},
           "scanline_pass_ms": round(scan_rep, 5), "launch_shape": tune,
           "scanline_hbm_frac": round(alg / (scan_rep * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
           "scanline_alu_frac": round(bitonic_ops(n_cand, sc.scan_len) / (scan_rep * 1e-3) / 1e9
                                      / ALU_PEAK_GOPS, 4),
           "candidates_per_view": [int(x) for x in n_cand]}
    if not args.no_check:
        from oracle import occl_ref
        M_ref, _, nc_ref = occl_ref.detect_scene(sc)
        out["parity"] = {"mismatches": int((M.cpu().numpy() != M_ref).sum()),
                         "candidates_equal": bool(np.array_equal(n_cand, nc_ref)),
                         "frames_in_flight_disagreeing_bytes": fl_bad}
    ctx.occl_release()
    return out


def bench_c2(ctx, steps: int, tune: bool = True):
    """One 3840x2160 frame with 15 views of a 4x4 array (L up to 366)."""
    import torch
    from paper_2408_14050_amd import occl, scenes
    sc = scenes.make_scene("c2", 2000)
    H, W, V = sc.H, sc.W, sc.n_views
    D = torch.from_numpy(sc.D).cuda()
    M = torch.empty((V, H, W), dtype=torch.uint8, device="cuda")
    prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len)
    shape = ctx.occl_autotune(D, sc.angles, sc.ratios, prm, M, reps=3) if tune else None
    for _ in range(3):
        ctx.occl_detect(D, sc.angles, sc.ratios, prm, M=M)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.occl_detect(D, sc.angles, sc.ratios, prm, M=M)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ctx.occl_profile_enable(True)
    for _ in range(steps):
        ctx.occl_detect(D, sc.angles, sc.ratios, prm, M=M)
    prof = ctx.occl_profile_read()
    ctx.occl_profile_enable(False)
    n_cand = ctx.occl_last_candidate_counts(V)
    scan_rep = ctx.occl_time_scanlines(steps)
    alg = (4 + V) * H * W
    ops = bitonic_ops(n_cand, sc.scan_len)
    return {"workload": C2_WORKLOAD, "ms": round(ms, 4), "value": round(H * W * V / (ms * 1e-3) / 1e6, 1),
            "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "stages_ms": {k: round(prof[k][0] / max(1, prof[k][1]), 4) for k in ("edges", "scanlines")},
            "scanline_pass_ms": round(scan_rep, 4), "scan_kernels": scan_kernels(sc.scan_len),
            "alu": {"ops": ops, "achieved_gops": round(ops / (scan_rep * 1e-3) / 1e9, 1),
                    "peak_gops": ALU_PEAK_GOPS,
                    "frac": round(ops / (scan_rep * 1e-3) / 1e9 / ALU_PEAK_GOPS, 4)},
            "scan_len": [int(x) for x in sc.scan_len], "candidates": int(sum(n_cand)),
            "launch_shape": shape}


def bench_quality(ctx, n_frames: int = 4):
    """Eq. (7) of the exact method against forward-warping ground truth
    (occl_zbuffer) on c1 frames: configs' L and Eq. (3)'s L."""
    import torch
    from paper_2408_14050_amd import occl, scenes
    out = {"workload": f"c1 1280x960 x8 views seeds 1000..{1000 + n_frames - 1}",
           "reference": "forward-warping z-buffer (nearest target pixel, beta 0.5)"}
    for name, mode, extra in (("scan_len_config", 0, 0), ("scan_len_eq3", -1, 0),
                              ("scan_len_eq3_bilinear", -1, occl.FLAG_BILINEAR),
                              ("scan_len_config_thin", 0, occl.FLAG_THIN),
                              ("scan_len_eq3_thin", -1, occl.FLAG_THIN)):
        acc = [0, 0, 0, 0]
        per_frame = []
        for k in range(n_frames):
            sc = scenes.make_scene("c1", 1000 + k)
            D = torch.from_numpy(sc.D).cuda()
            if mode == 0:
                prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len, flags=extra)
            else:
                prm = occl.params(**sc.params, scan_len=-1, flags=extra)
            M = ctx.occl_detect(D, sc.angles, sc.ratios, prm)
            Z = ctx.occl_zbuffer(D, sc.angles, sc.ratios, sc.params["disp_thr"])
            q = ctx.occl_quality(M, Z)
            per_frame.append(q["f1"])
            for i, key in enumerate(("tp", "fp", "fn", "tn")):
                acc[i] += q[key]
        tp, fp, fn = acc[0], acc[1], acc[2]
        P, R = tp / max(1, tp + fp), tp / max(1, tp + fn)
        out[name] = {"precision": round(P, 4), "recall": round(R, 4), "f1": round(2 * P * R / (P + R), 4),
                     "f1_per_frame_mean": round(sum(per_frame) / len(per_frame), 4),
                     "iou": round(tp / max(1, tp + fp + fn), 4)}
    # the limitation cases of Sec. 5: what the method (on the GPU) misses
    # against a ground truth of every painted surface
    from oracle import layered_gt
    lim = {}
    for kind in scenes.LIMITATION_CASES:
        sl, layers = scenes.limitation_scene(kind)
        Dl = torch.from_numpy(sl.D).cuda()
        Ml = ctx.occl_detect(Dl, sl.angles, sl.ratios,
                             occl.params(**sl.params, scan_len_per_view=sl.scan_len)).cpu().numpy()
        Zt = layered_gt.zbuffer_layers(sl.D, layers, sl.angles, sl.ratios, sl.params["disp_thr"])
        tp = int((Ml.astype(bool) & Zt.astype(bool)).sum())
        lim[kind] = {"true_occluded": int(Zt.sum()), "found": tp,
                     "missed": int((Zt.astype(bool) & ~Ml.astype(bool)).sum()),
                     "false": int((Ml.astype(bool) & ~Zt.astype(bool)).sum()),
                     "recall": round(tp / max(1, int(Zt.sum())), 4)}
    out["limitations_sec5"] = lim
    sc = scenes.make_scene("c1", 1000)
    D = torch.from_numpy(sc.D).cuda()
    Z = ctx.occl_zbuffer(D, sc.angles, sc.ratios, 0.5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        ctx.occl_zbuffer(D, sc.angles, sc.ratios, 0.5, M=Z)
    torch.cuda.synchronize()
    out["zbuffer_ms"] = round((time.perf_counter() - t0) / 20 * 1e3, 4)
    return out


def bench_thin(ctx, seed: int, steps: int = 500, prewarm: int = 300):
    """Candidate thinning (OCCL_FLAG_THIN, a variant) on one c1 frame at a
    time: ms per frame beside the exact path on the same context and stream,
    the scanline pass alone, and how far the mask moves from the exact one."""
    import torch
    from paper_2408_14050_amd import occl, scenes
    sc = scenes.make_scene("c1", seed)
    D = torch.from_numpy(sc.D).cuda()
    out = {"workload": f"c1 1280x960 x8 views seed {seed}, configured L, one frame at a time"}
    masks = {}
    for name, fl in (("exact", 0), ("thin", occl.FLAG_THIN)):
        prm = occl.params(**sc.params, scan_len_per_view=sc.scan_len, flags=fl)
        f = ctx.occl_detect_prepared(sc.angles, sc.ratios, prm)
        M = torch.empty((len(sc.angles),) + sc.D.shape, dtype=torch.uint8, device="cuda")
        for _ in range(prewarm):
            f(D, M)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            f(D, M)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        out[name] = {"ms": round(ms, 4), "scanline_pass_ms": round(ctx.occl_time_scanlines(200), 4)}
        masks[name] = M.clone()
    c = ctx.occl_confusion(masks["thin"], masks["exact"])
    out["vs_exact"] = {"differing_bytes": int(c["fp"] + c["fn"]),
                       "iou": round(c["tp"] / max(1, c["tp"] + c["fp"] + c["fn"]), 5)}
    out["speedup_vs_exact"] = round(out["exact"]["ms"] / out["thin"]["ms"], 3)
    return out


def bench_fusion(ctx, steps: int = 50):
    """Median fusion of 8 noisy per-view maps into D at 1280x960 (HBM-bound:
    (K + 1) * 4 bytes per pixel)."""
    import torch
    from paper_2408_14050_amd import scenes
    sc = scenes.make_scene("c1", 1002)
    K = 8
    maps = torch.from_numpy(scenes.fusion_maps(1, sc.D, K=K)).cuda()
    D = ctx.occl_median_fuse(maps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.occl_median_fuse(maps, D=D)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    alg = (K + 1) * 4 * sc.H * sc.W
    return {"workload": f"8 maps 1280x960 (c1 seed 1002 + noise 0.3, 5 % outliers, 3 % holes)",
            "ms": round(dt * 1e3, 4), "alg_bytes": alg, "alg_gbps": round(alg / dt / 1e9, 1),
            "hbm_frac": round(alg / dt / 1e9 / HBM_PEAK_GBPS, 4)}


def cnn_flops(H: int, W: int) -> int:
    """Multiply-adds x 2 of the tile network's convolutions on one H x W view."""
    layers = [(8, 32, 2), (32, 32, 2), (32, 32, 2), (32, 32, 2), (32, 32, 1), (32, 1, 1)]
    tot = 0
    for ci, co, st in layers:
        H, W = (H + st - 1) // st, (W + st - 1) // st
        tot += 2 * H * W * co * 9 * ci
    return tot


def cnn_train_flops(H: int, W: int) -> int:
    """Multiply-adds x 2 of one training step of the tile network on one
    H x W input: the forward, the weight gradient of every layer and the
    input gradient of every layer but the first."""
    layers = [(8, 32, 2), (32, 32, 2), (32, 32, 2), (32, 32, 2), (32, 32, 1), (32, 1, 1)]
    tot = 0
    for li, (ci, co, st) in enumerate(layers):
        H, W = (H + st - 1) // st, (W + st - 1) // st
        f = 2 * H * W * co * 9 * ci
        tot += f * (3 if li > 0 else 2)
    return tot


def bench_train(steps: int, crops: int = 128, crop: int = 256):
    """One Adam step of the tile network on `crops` random crops of crop x
    crop x 8 input channels (the training batch of the shipped weights), on a
    context of its own: ms per step, crops/s and the convolutions' TFLOP/s."""
    import numpy as np
    import torch
    from paper_2408_14050_amd import occl
    tctx = occl.Context(0)
    tctx.occl_cnn_init(1)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(size=(crops, crop, crop, 8), dtype=np.float32)
    x[..., 7] = 0.0
    X = torch.from_numpy((x.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)).cuda()
    del x
    T = torch.from_numpy(rng.uniform(size=(crops, crop // 16, crop // 16)).astype(np.float32)).cuda()
    for _ in range(3):
        tctx.occl_cnn_train_step(X, T, 1e-3, want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tctx.occl_cnn_train_step(X, T, 1e-3, want_loss=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    tctx.occl_release()
    fl = cnn_train_flops(crop, crop) * crops
    return {"workload": f"{crops} random crops of {crop}x{crop} x 8 channels, one Adam step each",
            "steps": steps, "ms_per_step": round(dt * 1e3, 4), "crops_per_s": round(crops / dt, 1),
            "gflop_per_step": round(fl / 1e9, 2), "tflops": round(fl / dt / 1e12, 2)}


def bench_learned(ctx, steps: int, n_eval: int, train: bool = True):
    """Learned tile proposal + exact fallback against the exact path on
    1920x1080 frames x 8 views (c1 statistics, held-out seeds 4100...)."""
    import torch
    from paper_2408_14050_amd import occl, scenes
    from paper_2408_14050_amd.train_tile_cnn import DEFAULT_WEIGHTS, EVAL_SEED0, load_state
    meta = load_state(ctx, DEFAULT_WEIGHTS)
    angles, ratios = scenes.views_3x3()
    frames = [scenes.make_c1_like(EVAL_SEED0 + k, W=1920, H=1080) for k in range(max(1, n_eval))]
    bands = [(0.05, 0.95), (0.02, 0.98)]
    qual = {b: [0, 0, 0, 0, 0] for b in bands}   # tp, fp, fn, exact tiles, tiles
    for sc in frames:
        D = torch.from_numpy(sc.D).cuda()
        M = ctx.occl_detect(D, angles, ratios, occl.params(scan_len_per_view=sc.scan_len))
        Z = ctx.occl_cnn_propose(D, angles, ratios, sc.scan_len)
        st = torch.empty(Z.shape, dtype=torch.uint8, device="cuda")
        for b in bands:
            prm = occl.params(scan_len_per_view=sc.scan_len, cnn_lo=b[0], cnn_hi=b[1],
                              flags=occl.FLAG_USE_CNN)
            Mc = ctx.occl_detect(D, angles, ratios, prm)
            ctx.occl_detect_routed(D, angles, ratios, prm, Z, tile_state=st)
            c = ctx.occl_confusion(Mc, M)
            q = qual[b]
            q[0] += c["tp"]; q[1] += c["fp"]; q[2] += c["fn"]
            q[3] += int((st == 2).sum().item()); q[4] += st.numel()
    sc = frames[0]
    D = torch.from_numpy(sc.D).cuda()
    M = torch.empty((8, sc.H, sc.W), dtype=torch.uint8, device="cuda")
    pv = sc.H * sc.W * 8

    def timed(prm):
        for _ in range(5):
            ctx.occl_detect(D, angles, ratios, prm, M=M)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.occl_detect(D, angles, ratios, prm, M=M)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        ctx.occl_profile_enable(True)
        for _ in range(steps):
            ctx.occl_detect(D, angles, ratios, prm, M=M)
        pr = ctx.occl_profile_read()
        ctx.occl_profile_enable(False)
        stages = {k: round(v[0] / max(1, v[1]), 5) for k, v in pr.items() if v[1]}
        return dt, stages

    dt_exact, st_exact = timed(occl.params(scan_len_per_view=sc.scan_len))
    out = {"workload": "c4: 1920x1080 x8 views, c1 statistics, held-out seeds "
                       f"{EVAL_SEED0}..{EVAL_SEED0 + len(frames) - 1} (timing on the first)",
           "weights": os.path.relpath(DEFAULT_WEIGHTS, ROOT), "training": meta,
           "train_step": bench_train(max(5, steps // 2)) if train else None,
           "exact": {"ms": round(dt_exact * 1e3, 4), "mpixel_views_per_s": round(pv / dt_exact / 1e6, 1),
                     "stages_ms": st_exact}}
    fl = cnn_flops(sc.H, sc.W) * 8
    for b in bands:
        prm = occl.params(scan_len_per_view=sc.scan_len, cnn_lo=b[0], cnn_hi=b[1], flags=occl.FLAG_USE_CNN)
        dt, stages = timed(prm)
        tp, fp, fn, ex, nt = qual[b]
        cnn_ms = stages.get("cnn", float("nan"))
        out[f"cnn_band_{b[0]}_{b[1]}"] = {
            "ms": round(dt * 1e3, 4), "mpixel_views_per_s": round(pv / dt / 1e6, 1),
            "vs_exact": round(dt_exact / dt, 4), "iou": round(tp / max(1, tp + fp + fn), 5),
            "precision": round(tp / max(1, tp + fp), 5), "recall": round(tp / max(1, tp + fn), 5),
            "exact_tile_share": round(ex / max(1, nt), 5), "stages_ms": stages,
            "cnn_tflops": round(fl / (cnn_ms * 1e-3) / 1e12, 2) if cnn_ms == cnn_ms else None,
            "cnn_gflop_per_frame": round(fl / 1e9, 2)}
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed batched launches (headline)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prewarm-batched", type=int, default=300,
                    help="untimed batched launches before the timed region")
    ap.add_argument("--seed", type=int, default=1002, help="c1 frame of the single-frame section")
    ap.add_argument("--c1-steps", type=int, default=1000)
    ap.add_argument("--c2-steps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-context", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-c1", action="store_true")
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--c2-only", action="store_true", help="only the 3840x2160 x15 section")
    ap.add_argument("--profiles-from", default=None, metavar="DIR")
    ap.add_argument("--profiles-index", action="store_true", help="only rewrite profiles/INDEX.md")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-only", action="store_true", help="only the learned-path section")
    ap.add_argument("--train-only", action="store_true", help="only the network's training step")
    ap.add_argument("--train-steps", type=int, default=20)
    ap.add_argument("--no-train-step", action="store_true", help="learned section without the training step")
    ap.add_argument("--no-quality", action="store_true")
    ap.add_argument("--quality-only", action="store_true", help="only the quality and fusion sections")
    ap.add_argument("--thin-only", action="store_true", help="only the candidate-thinning section")
    ap.add_argument("--streams", type=int, default=3,
                    help="c1 section: frames in flight on separate HIP streams")
    ap.add_argument("--prewarm", type=int, default=PREWARM_STEPS,
                    help="c1 section: untimed steps before each timed region")
    ap.add_argument("--learned-steps", type=int, default=50)
    ap.add_argument("--learned-eval", type=int, default=4, help="c4 frames for IoU / P / R")
    args = ap.parse_args()
    if args.copy_probe:
        return copy_probe(args.copy_probe)
    if args.profiles_from:
        return profiles_from(args.profiles_from, C1_WORKLOAD)
    if args.profiles_index:
        return write_profile_index()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the detector's "
              "sharding across GPUs is not built", file=sys.stderr)
        return 2

    import torch
    from paper_2408_14050_amd import occl, scenes

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 3
    if args.train_only:
        print(json.dumps({"train_step": bench_train(args.train_steps)}), flush=True)
        return 0
    if args.learned_only:
        ctx = occl.Context(0)
        print(json.dumps(bench_learned(ctx, args.learned_steps, args.learned_eval, not args.no_train_step)),
              flush=True)
        ctx.occl_release()
        return 0
    if args.thin_only:
        ctx = occl.Context(0)
        print(json.dumps({"thinning": bench_thin(ctx, args.seed)}), flush=True)
        ctx.occl_release()
        return 0
    if args.quality_only:
        ctx = occl.Context(0)
        print(json.dumps({"quality_vs_zbuffer": bench_quality(ctx), "median_fusion": bench_fusion(ctx),
                          "thinning": bench_thin(ctx, args.seed)}), flush=True)
        ctx.occl_release()
        return 0
    if args.c2_only:
        ctx = occl.Context(0)
        print(json.dumps({"c2": bench_c2(ctx, args.c2_steps, not args.no_tune)}), flush=True)
        ctx.occl_release()
        return 0

    ctx = occl.Context(0)
    c3 = bench_c3(ctx, args)
    frames = c3.pop("frames")
    c3.pop("masks")
    sizes = sorted({(f.W, f.H) for f in frames})
    out = {
        "metric": METRIC, "value": round(c3["value"], 1), "unit": "Mpixel-views/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(c3["ms_per_step"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c3: 64 frames of mixed size, 8 views each, seed 3000, one batched "
                               "graph launch per step",
                   "frames": len(frames), "frame_sizes": [f"{w}x{h}" for w, h in sizes],
                   "views": 8, "pixel_views_per_step": c3["pixel_views"], "path": "exact",
                   "parallelism": "single GPU", "launch_shape": c3["launch_shape"]},
        "prewarm_steps": max(args.warmup, args.prewarm_batched),
        "frames_per_s": round(len(frames) / (c3["ms_per_step"] * 1e-3), 1),
        "roofline": c3["roofline"],
        "hbm": {"alg_bytes_per_step": c3["alg_bytes"],
                "path_gbps": round(c3["alg_bytes"] / (c3["ms_per_step"] * 1e-3) / 1e9, 1),
                "path_frac": round(c3["alg_bytes"] / (c3["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)},
        "stages_ms": {k: (round(v, 5) if isinstance(v, float) else v) for k, v in c3["stages_ms"].items()},
    }
    for k in ("parity", "alu"):
        if k in c3:
            out[k] = c3[k]

    if not args.no_c1:
        out["c1"] = bench_c1(args)

    if not args.no_c2:
        out["c2"] = bench_c2(ctx, args.c2_steps, not args.no_tune)

    if not args.no_context:
        # the shape of the paper's runtime experiment (Table 3), as context only
        scp = scenes.make_scene("paper", 1)
        Dp = torch.from_numpy(scp.D).cuda()
        Mp = torch.empty((scp.n_views, scp.H, scp.W), dtype=torch.uint8, device="cuda")
        pp = occl.params(**scp.params, scan_len_per_view=scp.scan_len)
        detp = ctx.occl_detect_prepared(scp.angles, scp.ratios, pp)
        for _ in range(50):
            detp(Dp, Mp)
        torch.cuda.synchronize()
        windows = []  # median of 5 windows: a one-off host stall must not set the figure
        for _ in range(5):
            t0 = time.perf_counter()
            for _ in range(50):
                detp(Dp, Mp)
            torch.cuda.synchronize()
            windows.append((time.perf_counter() - t0) / 50)
        tp = sorted(windows)[2]
        out["context_paper_shape"] = {
            "workload": "1600x1200 x8 views, c1 statistics", "ms": round(tp * 1e3, 4),
            "windows_ms": [round(w * 1e3, 4) for w in windows],
            "value": round(scp.pixel_views / tp / 1e6, 1),
            "paper_gpu_ms": 26.0, "paper_gpu_value": round(PAPER_GPU_MPVS, 1),
            "paper_hw": "NVIDIA GeForce RTX 3090 (paper's own scene, not this one)"}

    if not args.no_learned:
        out["learned"] = bench_learned(ctx, args.learned_steps, args.learned_eval, not args.no_train_step)
        ex = out["learned"]["exact"]
        pv4 = 1920 * 1080 * 8
        out["c4_exact"] = {"workload": "c4 1920x1080 x8 views, c1 statistics, seed 4100",
                           "ms": ex["ms"], "value": ex["mpixel_views_per_s"],
                           "hbm_frac": round((4 + 8) * pv4 / 8 / (ex["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                           "stages_ms": ex["stages_ms"]}

    if not args.no_quality:
        out["quality_vs_zbuffer"] = bench_quality(ctx)
        out["median_fusion"] = bench_fusion(ctx)
        out["thinning"] = bench_thin(ctx, args.seed)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(frames, args.cpu_seconds)

    ctx.occl_release()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

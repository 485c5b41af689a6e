#!/usr/bin/env python3
"""Throughput of the w-stacking imager on one MI355X.

One step = one dirty image of the workload: rick_reset + rick_grid
(bin-and-sort + LDS-tiled gridding) + rick_fft_planes + rick_wstack_image,
with inputs already resident in HBM and the plan built beforehand.

Prints ONE JSON line (metric Mvis/s through grid + iFFT + w-stack), with a
roofline entry for the kernel that takes the most device time and the float64
oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CU_COUNT = 256
CLOCK_HZ = 2.4e9
METRIC = "Mvis/s through grid+iFFT+w-stack at fixed image RMS vs FP64 DFT oracle"


def algorithmic_bytes(name, ds, info):
    """Bytes the method must move per launch of kernel `name`.  The gridder's
    unit figures are the method's: a 16-byte record {int32 X, int32 Y,
    complex64 W V} read per gridded visibility (this library packs it into
    12 bytes; the difference is its own gain, not counted) and 8 bytes
    written per cell that holds gridded values.  Only tiles that received
    visibilities (or their neighbours' margins) hold gridded values: the
    gridder writes those tiles, the row pass reads them and (fused) writes
    the rows of tile rows holding any, which the fused column pass reads.
    The binning kernels are counted with the records this library writes
    (level-1 records of rec1_bytes, 12-byte gridding records)."""
    nvis, nrow = ds.nvis, ds.nrow
    n2 = ds.grid_n * ds.grid_n
    cells = ds.n_wplanes * n2
    T = info["tile"]
    set_cells = info["tiles_set"] * T * T                  # cells of tiles holding gridded values
    row_cells = info["tile_rows_set"] * T * ds.grid_n      # cells of rows in tile rows holding any
    fused = bool(info.get("row_mesh_ptr"))
    wbytes = 4 * nvis if ds.weight is not None else 0
    r1 = info.get("rec1_bytes") or 16                     # bytes per level-1 record (position + W V)
    p1 = r1 - (16 if r1 == 24 else 8)                      # bytes of its position
    table = {
        "bin_count": 24 * nrow + wbytes,                # uvw (and weights): V is not read
        "bin_scatter": 24 * nrow + 8 * nvis + wbytes + r1 * nvis,   # writes the level-1 records
        "fine_count": p1 * nvis,                                    # reads their positions
        "fine_scatter": r1 * nvis + 12 * nvis,                      # reads them, writes 12-byte records
        "grid": 16 * nvis + 8 * set_cells,                         # 16 B {X, Y, W V} per visibility
        "fft_rows": 8 * set_cells + 8 * (row_cells if fused else cells),
        "fft_cols": 16 * cells,
        "wscreen": 8 * cells + 4 * n2,
        "fft_cols_screen": 8 * row_cells + 4 * n2,
    }
    return table.get(name)


def host_threads():
    """Threads the host share of this process offers: the CPU affinity set,
    capped by OMP_NUM_THREADS when that is set."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_model():
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ds, vis_host, threads, n_rows_sample=1_048_576, n_grid_target=8_000_000, n_planes_fft=4):
    """The float64 oracle, as it stands, timed stage by stage on a bounded
    sample of the same workload and scaled to the whole job:
      T = t_bin / n_binned * N_vis + t_grid / n_gridded * N_kept + N_w * t_plane / n_planes.
    `threads` workers run the oracle's own functions on independent pieces
    (row blocks for binning, w-planes for gridding, FFT and screen), the
    method's natural parallelism; numpy releases the interpreter lock inside
    its array loops, so the pieces overlap."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import wstack as ow
    kw = ds.plan_kwargs()
    geo = {k: kw[k] for k in ("grid_n", "n_wplanes", "support", "oversample", "fov", "w_min", "w_max")}
    rows = min(n_rows_sample, ds.nrow)
    step = max(1, ds.nrow // rows)
    sel = np.arange(0, ds.nrow, step)[:rows]
    uvw_s = ds.uvw[sel]
    vis_s = vis_host[sel]
    wt_s = None if ds.weight is None else ds.weight[sel]
    n_s = uvw_s.shape[0] * ds.nchan
    blocks = np.array_split(np.arange(uvw_s.shape[0]), max(1, threads))
    table = ow.tap_table(ds.support, ds.oversample, ds.kernel, ds.kernel_param)
    corr = ow.grid_correction(table, ds.grid_n)
    wk = ow.plane_centres(ds.w_min, ds.w_max, ds.n_wplanes)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        t0 = time.perf_counter()
        parts = list(ex.map(lambda ix: ow.bin_visibilities(uvw_s[ix], ds.freq, vis_s[ix],
                                                           None if wt_s is None else wt_s[ix], **geo), blocks))
        t_bin = time.perf_counter() - t0
        # gridding: the fullest planes of the first row block's binning, one task per plane
        b = parts[0]
        keep = np.nonzero(b.keep)[0]
        kk = b.k[keep]
        todo, n_grid = [], 0
        for k in np.argsort(-np.bincount(kk, minlength=ds.n_wplanes)):
            if n_grid >= n_grid_target // max(1, len(blocks)) or len(todo) >= max(threads, 2):
                break
            idx = keep[kk == k]
            todo.append(idx)
            n_grid += idx.size

        def grid_one(idx):
            G = np.zeros((ds.grid_n, ds.grid_n), np.complex128)
            ow.grid_plane(G, b, idx, table)
            return G

        t0 = time.perf_counter()
        planes = list(ex.map(grid_one, todo))
        t_grid = time.perf_counter() - t0
        src = [planes[j % len(planes)] for j in range(n_planes_fft)]

        def plane_one(j):
            F = ow.ifft_planes(src[j][None])
            S = ow.screen_sum(F, wk[j:j + 1], ds.fov)
            return ow.normalise(S, corr, 1.0, ds.fov)

        t0 = time.perf_counter()
        list(ex.map(plane_one, range(n_planes_fft)))
        t_plane = time.perf_counter() - t0
        del planes, src
    kept_frac = float(np.mean([p.keep.mean() for p in parts])) if n_s else 0.0
    total = (t_bin / n_s * ds.nvis + (t_grid / n_grid if n_grid else 0.0) * kept_frac * ds.nvis +
             ds.n_wplanes * t_plane / n_planes_fft)
    spent = t_bin + t_grid + t_plane
    sample = (f"oracle stages on {threads} thread(s): {n_s:,} visibilities binned ({uvw_s.shape[0]:,} rows x "
              f"{ds.nchan} channels, every {step}th row), {n_grid:,} of them gridded onto {len(todo)} plane(s), "
              f"{n_planes_fft} {ds.grid_n}^2 planes transformed, screened and normalised ({spent:.1f} s); "
              f"per-visibility and per-plane costs scaled to {ds.nvis:,} visibilities and {ds.n_wplanes} planes "
              f"(est. {total:.0f} s per image)")
    return {"value": ds.nvis / total / 1e6, "unit": "Mvis/s", "cores": threads, "kind": "oracle",
            "sample": sample, "sample_seconds": round(spent, 2), "est_seconds_per_image": round(total, 1)}


def check_pixels(ds, n_patch=8, n_sources=8):
    """Pixels the benchmark checks: an n_patch x n_patch patch at the phase
    centre and the n_sources brightest sources."""
    N = ds.grid_n
    half = n_patch // 2
    qq, pp = np.meshgrid(np.arange(N // 2 - half, N // 2 - half + n_patch),
                         np.arange(N // 2 - half, N // 2 - half + n_patch), indexing="ij")
    pp, qq = pp.ravel(), qq.ravel()
    src = ds.sources
    order = np.argsort(-np.asarray(src["flux"]))[:n_sources]
    dl = ds.fov / N
    sp = np.rint(np.asarray(src["l"])[order] / dl).astype(np.int64) + N // 2
    sq = np.rint(np.asarray(src["m"])[order] / dl).astype(np.int64) + N // 2
    return np.r_[pp, sp], np.r_[qq, sq]


# image tolerances of the benchmark's check (the parity bar of the tests):
# float32 modes within 1e-5 of the float64 oracle (apparent image), and the
# distance to the direct Fourier sum equal to the oracle's own within 1 %
TOL_ORACLE = 1e-5
TOL_DFT = 0.01


def oracle_leg(ds, vis_host, img_pix, pp, qq, corr):
    """The float64 oracle (per-pixel w-stacking over every visibility) and
    the direct Fourier sum at the checked pixels, against the GPU image
    values img_pix there."""
    import oracle.dft
    import oracle.pixels
    t0 = time.perf_counter()
    orc, _, kept, sw = oracle.pixels.wstack_pixels(ds.uvw, ds.freq, vis_host, ds.weight, pp, qq,
                                                   **ds.plan_kwargs())
    t_orc = time.perf_counter() - t0
    cp = corr[pp] * corr[qq]

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    out = {"pixels": int(len(pp)), "oracle_kept": int(kept),
           "gpu_vs_oracle": {"apparent_rel_rms": rel(img_pix * cp, orc * cp), "image_rel_rms": rel(img_pix, orc)},
           "oracle_seconds": round(t_orc, 1)}
    if kept == ds.nvis and ds.freq is not None:
        t0 = time.perf_counter()
        dft = oracle.dft.dft_pixels_rows(ds.uvw, ds.freq, vis_host, ds.weight, pp, qq, grid_n=ds.grid_n,
                                         fov=ds.fov, sum_w=sw)
        out["dft_seconds"] = round(time.perf_counter() - t0, 1)
        out["gpu_vs_dft"] = rel(img_pix, dft)
        out["oracle_vs_dft"] = rel(orc, dft)
        out["dft_gate"] = abs(out["gpu_vs_dft"] / out["oracle_vs_dft"] - 1.0)
    return out


# ---------------------------------------------------------------------------
# rocprofv3 runs and their text summaries.  `--profile OUT` runs each pass as a
# child process (in /tmp, TMPDIR=/tmp, the program after `--`), each under its
# own time limit, stops at the first pass that fails, and writes the summaries
# into OUT/summary; those are the files kept under profiles/.
# ---------------------------------------------------------------------------
PROFILE_BENCH = ["--steps", "3", "--warmup", "1", "--no-cpu-baseline", "--no-check"]
COPY_MIB = 1024
SQ_COUNTERS = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_WAIT_INST_LDS",
               "SQ_LDS_BANK_CONFLICT", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES"]
# library kernel -> the plan timer that brackets it
KERNEL_TIMER = {"k_zero_stats": "reset", "k_set_scales": "(scales upload)", "k_l1_count": "bin_count",
                "k_flat_partials": "bin_scan", "k_flat_top": "bin_scan", "k_flat_apply": "bin_scan",
                "k_l2_chunks": "bin_scan", "k_l1_scatter": "bin_scatter", "k_l2_count": "fine_count",
                "k_l2_totals": "fine_scan", "k_scan_partials": "fine_scan", "k_scan_top": "fine_scan",
                "k_scan_apply": "fine_scan", "k_l2_bases": "fine_scan", "k_l2_scatter": "fine_scatter",
                "k_zero_heavy": "zero_heavy",
                "k_grid": "grid", "k_zero_mesh": "zero_mesh", "k_fft_rows": "fft_rows", "k_fft_rows_panel": "fft_rows", "k_fft_cols": "fft_cols",
                "k_fft_cols_screen": "fft_cols_screen", "k_wscreen": "wscreen", "k_merge_margins": "merge_margins", "k_row_bits": "merge_margins",
                "k_clear_bits": "reset", "k_bin_vmax": "fine_scatter", "k_orient": "(orientation)"}


# Sources whose kernels the imaging step never launches (prediction): they do
# not change what the imaging counters describe.
NOT_IN_IMAGING_STEP = ("degrid.hip",)


def kernel_sources_digest():
    """sha256 over the sources of the kernels the imaging step launches and of
    the plan: counters taken on other sources do not describe the kernels that
    run now."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2504_00959_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".cpp", ".h")) and f not in NOT_IN_IMAGING_STEP:
            h.update(f.encode())
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    with open(os.path.join(ROOT, "include", "rick.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, timer):
    """HBM bytes per launch of the kernel behind `timer`, from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None when there is none or the
    kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")
    if not os.path.exists(path):
        return None, "no counter summary for this workload"
    digest, rows = None, {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("# source_sha256:"):
                digest = line.split(":", 1)[1].strip()
            elif line.startswith("timer "):
                name, val = line[len("timer "):].rsplit(None, 1)
                rows[name.strip()] = float(val)
    if digest != kernel_sources_digest():
        return None, "kernel sources changed since the counters were taken"
    if timer not in rows:
        return None, f"no counters for {timer}"
    return int(rows[timer]), f"FETCH_SIZE + WRITE_SIZE, copy-calibrated ({os.path.basename(path)})"


def measured_valu(workload, timer):
    """VALU wave instructions per launch of the kernels behind `timer`, from
    the committed SQ counter summary, or None when there is none or the
    kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"sq_counters_{workload}.txt")
    if not os.path.exists(path):
        return None
    digest, total = None, 0.0
    nc = len(SQ_COUNTERS)
    with open(path) as fh:
        for line in fh:
            if line.startswith("# source_sha256:"):
                digest = line.split(":", 1)[1].strip()
            elif line.strip() and not line.startswith(("#", "kernel")):
                # kernel name (spaces inside its template arguments), then one column per counter
                parts = line.split()
                name = " ".join(parts[:-nc])
                if KERNEL_TIMER.get(name.split("<")[0]) == timer:
                    total += float(parts[-nc:][SQ_COUNTERS.index("SQ_INSTS_VALU")])
    if digest != kernel_sources_digest() or total == 0.0:
        return None
    return total


def short_kernel(name):
    import re
    m = re.search(r"::(k_[a-z0-9_]+)(<[^()]*>)?\(", name)
    return (m.group(1), m.group(1) + (m.group(2) or "")) if m else (None, name[:60])


def read_counters(path):
    """{kernel (short name with template args): [values per dispatch]} for one counter run."""
    import csv
    out = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            base, full = short_kernel(r["Kernel_Name"])
            key = full if base else r["Kernel_Name"]
            out.setdefault((key, r["Counter_Name"]), {}).setdefault(r["Dispatch_Id"], 0.0)
            out[(key, r["Counter_Name"])][r["Dispatch_Id"]] += float(r["Counter_Value"])
    return out


def profile_commands(out, workload):
    py, me = sys.executable, os.path.abspath(__file__)
    bench = [py, me, "--workload", workload] + PROFILE_BENCH
    copy = [py, me, "--copy-calibration", str(COPY_MIB)]

    def pmc(name, regex, counters, prog, limit):
        return (name, ["rocprofv3", "--kernel-include-regex", regex, "--pmc"] + counters +
                ["-f", "csv", "-d", os.path.join(out, name), "-o", "run", "--"] + prog, limit)
    return [
        ("trace", ["rocprofv3", "--kernel-trace", "--stats", "-f", "csv", "-d", os.path.join(out, "trace"), "-o",
                   "run", "--"] + bench, 600),
        pmc("fetch", "rick", ["FETCH_SIZE"], bench, 300),
        pmc("write", "rick", ["WRITE_SIZE"], bench, 300),
        pmc("copy_fetch", "copyBuffer", ["FETCH_SIZE"], copy, 120),
        pmc("copy_write", "copyBuffer", ["WRITE_SIZE"], copy, 120),
        pmc("sq", "rick", SQ_COUNTERS, bench, 300),
    ]


def run_profiles(out, workload):
    import signal
    import subprocess
    os.makedirs(out, exist_ok=True)
    env = dict(os.environ, TMPDIR="/tmp")
    for name, cmd, limit in profile_commands(out, workload):
        print(f"[profile] {name}: {' '.join(cmd)}", file=sys.stderr, flush=True)
        with open(os.path.join(out, f"{name}.log"), "w") as log:
            p = subprocess.Popen(cmd, cwd="/tmp", env=env, stdout=log, stderr=subprocess.STDOUT,
                                 start_new_session=True)
            try:
                rc = p.wait(timeout=limit)
            except subprocess.TimeoutExpired:
                os.killpg(p.pid, signal.SIGKILL)
                p.wait()
                raise SystemExit(f"[profile] {name} exceeded {limit} s; later passes not started")
        results = [f for f in os.listdir(os.path.join(out, name))] if os.path.isdir(os.path.join(out, name)) else []
        print(f"[profile] {name}: rc={rc}, files {sorted(results)}", file=sys.stderr, flush=True)
        if rc != 0:
            # any nonzero exit fails the pass, also after a complete-looking run:
            # a fault at teardown (the library's or the profiler's) is not told
            # apart here, so the pass's rc and the end of its log are kept
            with open(os.path.join(out, f"{name}.log")) as fh:
                tail = fh.readlines()[-15:]
            with open(os.path.join(out, f"{name}.failed.txt"), "w") as fh:
                fh.write(f"rc={rc}\n" + "".join(tail))
            raise SystemExit(f"[profile] {name} failed (rc={rc}); later passes not started; "
                             f"log tail in {name}.failed.txt")
    summarize_profiles(out, workload)


def summarize_profiles(out, workload):
    import csv
    summ = os.path.join(out, "summary")
    os.makedirs(summ, exist_ok=True)
    cmds = {name: " ".join(cmd).replace(sys.executable, "python").replace(ROOT, "<repo>")
            for name, cmd, _ in profile_commands(out, workload)}
    prelude = "cd /tmp && export TMPDIR=/tmp   # <repo> = the repository root (absolute path)\n"
    bench_json = None
    with open(os.path.join(out, "trace.log")) as fh:
        for line in fh:
            if line.startswith('{"'):
                bench_json = json.loads(line)
    # 1. kernel trace
    rows = []
    with open(os.path.join(out, "trace", "run_kernel_stats.csv")) as fh:
        for r in csv.DictReader(fh):
            base, full = short_kernel(r["Name"])
            if base is None or "rick" not in r["Name"]:
                continue
            rows.append((full, KERNEL_TIMER.get(base, "?"), int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                         float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6))
    rows.sort(key=lambda t: -t[6])
    steps = int(PROFILE_BENCH[1]) + int(PROFILE_BENCH[3])
    lines = [f"# rocprofv3 kernel trace, {workload}: {bench_json['config']['workload'] if bench_json else ''}",
             "# command:", "#   " + prelude.strip(), "#   " + cmds["trace"],
             f"# {steps} steps traced (warmup included); library kernels only (the workload generator's "
             "torch kernels are left out)",
             f"# bench line of the same run: {bench_json['value']} Mvis/s, {bench_json['ms_per_step']} ms/step"
             if bench_json else "#",
             f"{'kernel':48s} {'plan timer':16s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} "
             f"{'total_ms':>10s}"]
    for full, timer, calls, avg, mn, mx, tot in rows:
        lines.append(f"{full:48s} {timer:16s} {calls:6d} {avg:10.1f} {mn:10.1f} {mx:10.1f} {tot:10.2f}")
    if bench_json:
        lines.append("# plan timers (HIP events in the bench's timed region), ms per call:")
        for k, v in bench_json["kernels"].items():
            lines.append(f"#   {k:16s} {v['ms']:.4f}")
    with open(os.path.join(summ, f"kernel_trace_{workload}.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")

    # 2. HBM traffic, copy-calibrated
    def mean_per_dispatch(path, counter):
        res = {}
        for (k, c), per in read_counters(path).items():
            if c == counter:
                res[k] = sum(per.values()) / len(per)
        return res
    cf = mean_per_dispatch(os.path.join(out, "copy_fetch", "run_counter_collection.csv"), "FETCH_SIZE")
    cw = mean_per_dispatch(os.path.join(out, "copy_write", "run_counter_collection.csv"), "WRITE_SIZE")
    copy_bytes = COPY_MIB << 20
    f_fetch = copy_bytes / (1024.0 * max(cf.values()))
    f_write = copy_bytes / (1024.0 * max(cw.values()))
    fetch = mean_per_dispatch(os.path.join(out, "fetch", "run_counter_collection.csv"), "FETCH_SIZE")
    write = mean_per_dispatch(os.path.join(out, "write", "run_counter_collection.csv"), "WRITE_SIZE")
    by_timer = {}
    lines = [f"# HBM traffic per dispatch, {workload}", "# commands:", "#   " + prelude.strip()]
    lines += ["#   " + cmds[n] for n in ("fetch", "write", "copy_fetch", "copy_write")]
    lines += [f"# calibration: a plain {COPY_MIB} MiB device copy reads FETCH_SIZE {max(cf.values()):.0f} KiB and "
              f"WRITE_SIZE {max(cw.values()):.0f} KiB per launch; scale factors {f_fetch:.4f} (fetch) and "
              f"{f_write:.4f} (write)",
              f"# source_sha256: {kernel_sources_digest()}",
              f"{'kernel':48s} {'fetch_KiB':>14s} {'write_KiB':>14s} {'traffic_bytes':>16s} {'algorithmic':>16s} "
              f"{'ratio':>7s}"]
    for k in sorted(set(fetch) | set(write), key=lambda k: -(fetch.get(k, 0) + write.get(k, 0))):
        base = k.split("<")[0]
        t = fetch.get(k, 0.0) * 1024 * f_fetch + write.get(k, 0.0) * 1024 * f_write
        timer = KERNEL_TIMER.get(base)
        alg = bench_json["kernels"].get(timer, {}).get("bytes") if bench_json and timer else None
        ratio = f"{t / alg:7.3f}" if alg else "      -"
        lines.append(f"{k:48s} {fetch.get(k, 0):14.0f} {write.get(k, 0):14.0f} {t:16.0f} "
                     f"{alg if alg else '-':>16} {ratio}")
        if timer:
            by_timer[timer] = by_timer.get(timer, 0.0) + t
    for timer, t in by_timer.items():
        lines.append(f"timer {timer} {t:.0f}")
    with open(os.path.join(summ, f"hbm_traffic_{workload}.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")

    # 3. SQ instruction counters
    sq_path = os.path.join(out, "sq", "run_counter_collection.csv")
    if os.path.exists(sq_path):
        sq = read_counters(sq_path)
        kernels = sorted({k for k, _ in sq})
        lines = [f"# SQ counters per dispatch (summed over the chip), {workload}", "# command:",
                 "#   " + prelude.strip(), "#   " + cmds["sq"],
                 f"# source_sha256: {kernel_sources_digest()}",
                 f"{'kernel':48s} " + " ".join(f"{c[3:]:>16s}" for c in SQ_COUNTERS)]
        for k in kernels:
            vals = []
            for c in SQ_COUNTERS:
                per = sq.get((k, c), {})
                vals.append(sum(per.values()) / len(per) if per else float("nan"))
            lines.append(f"{k:48s} " + " ".join(f"{v:16.4g}" for v in vals))
        with open(os.path.join(summ, f"sq_counters_{workload}.txt"), "w") as fh:
            fh.write("\n".join(lines) + "\n")
    print(f"[profile] summaries in {summ}", file=sys.stderr, flush=True)


def make_workload(name, device):
    import synth
    if name == "ska_low_share":
        return synth.ska_low_share(device=device)
    if name == "ska_low_precision":
        return synth.ska_low_precision(device=device)
    if name == "tiny":
        return synth.tiny(device=device)
    if name == "ska_low_small":
        return synth.ska_low_small(device=device)
    raise SystemExit(f"unknown workload {name}")


def precision_report(args):
    """Image error of each precision mode on one workload: every mode's image
    against the all-float64 GPU image (whole image), against the float64
    oracle at sampled pixels, and against the direct Fourier sum at the same
    pixels beside the oracle's own distance to it; plus each mode's step
    time.  Prints one JSON line."""
    import torch
    from paper_2504_00959_amd import rick
    import oracle.dft
    import oracle.pixels
    from oracle import wstack as ow

    dev = "cuda:0"
    t0 = time.time()
    ds = make_workload(args.workload, dev)
    print(f"[report] generated {describe(ds)} in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    N = ds.grid_n
    uvw = torch.as_tensor(ds.uvw, dtype=torch.float64).to(dev)
    vis_host = ds.vis.cpu().numpy()
    corr = ow.grid_correction(ow.tap_table(ds.support, ds.oversample, ds.kernel, ds.kernel_param), N)
    stream = torch.cuda.current_stream()
    images, runs = {}, {}
    for prec in ("fp32", "fp32_kahan", "fp64"):
        # float64 runs unfused: its fused form would need a second mesh-sized buffer
        fused = prec != "fp64"
        vis = ds.vis if prec != "fp64" else ds.vis.to(torch.complex128)
        plan = rick.Plan.for_dataset(ds, precision=prec, fused=fused)
        img = torch.empty((N, N), dtype=plan.real_dtype, device=dev)

        def step():
            plan.reset(stream)
            plan.grid(uvw, vis, None, ds.freq, stream)
            plan.fft(stream)
            plan.image(img, stream)

        step()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            step()
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        info = plan.info()
        runs[prec] = {"ms_per_step": round(ms, 3), "mvis_per_s": round(ds.nvis / (ms * 1e-3) / 1e6, 1),
                      "fused_screen": fused, "n_gridded": info["n_gridded"]}
        images[prec] = img.double().cpu().numpy()
        print(f"[report] {prec}: {ms:.2f} ms/step", file=sys.stderr, flush=True)
        plan.close()
        del vis, img, plan
        torch.cuda.empty_cache()

    # whole-image comparisons against the float64 GPU image
    c2 = np.outer(corr, corr)
    ref = images["fp64"]
    central = c2 >= 0.1
    for prec in ("fp32", "fp32_kahan"):
        d = images[prec] - ref
        runs[prec]["vs_fp64_gpu"] = {
            "apparent_rel_rms": float(np.linalg.norm(d * c2) / np.linalg.norm(ref * c2)),
            "central_rel_rms": float(np.linalg.norm(d[central]) / np.linalg.norm(ref[central])),
            "image_rel_rms": float(np.linalg.norm(d) / np.linalg.norm(ref)),
        }

    # sampled pixels: a patch at the phase centre and the brightest sources
    half = args.patch // 2
    qq, pp = np.meshgrid(np.arange(N // 2 - half, N // 2 - half + args.patch),
                         np.arange(N // 2 - half, N // 2 - half + args.patch), indexing="ij")
    pp, qq = pp.ravel(), qq.ravel()
    src = ds.sources
    order = np.argsort(-np.asarray(src["flux"]))[:8]
    dl = ds.fov / N
    sp = np.rint(np.asarray(src["l"])[order] / dl).astype(np.int64) + N // 2
    sq = np.rint(np.asarray(src["m"])[order] / dl).astype(np.int64) + N // 2
    pp, qq = np.r_[pp, sp], np.r_[qq, sq]
    t0 = time.time()
    orc, _, kept, sw = oracle.pixels.wstack_pixels(ds.uvw, ds.freq, vis_host, ds.weight, pp, qq,
                                                   **ds.plan_kwargs())
    t_orc = time.time() - t0
    cp = corr[pp] * corr[qq]
    dft = None
    t0 = time.time()
    if kept == ds.nvis:
        sc = np.asarray(ds.freq) / 299_792_458.0
        u = (ds.uvw[:, 0:1] * sc[None, :]).ravel()
        v = (ds.uvw[:, 1:2] * sc[None, :]).ravel()
        w = (ds.uvw[:, 2:3] * sc[None, :]).ravel()
        lm = ow.pixel_lm(N, ds.fov)
        L, M = lm[pp], lm[qq]
        nm1 = ow.nm1_of(L, M)
        D = oracle.dft.dft_sum(u, v, w, vis_host.reshape(-1), L, M, nm1)
        dft = (1.0 + nm1) * D.real / float(ds.nvis)
        del u, v, w
    t_dft = time.time() - t0

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    for prec in runs:
        got = images[prec][qq, pp]
        runs[prec]["vs_oracle_pixels"] = {"apparent_rel_rms": rel(got * cp, orc * cp),
                                          "image_rel_rms": rel(got, orc)}
        if dft is not None:
            runs[prec]["vs_dft_pixels"] = rel(got, dft)
    out = {"report": "precision", "workload": describe(ds), "n_vis": ds.nvis, "steps": args.steps,
           "pixels": {"patch": f"{args.patch}x{args.patch} at the phase centre", "sources": int(len(sp)),
                      "count": int(len(pp))},
           "oracle_vs_dft_pixels": rel(orc, dft) if dft is not None else None,
           "oracle_seconds": round(t_orc, 1), "dft_seconds": round(t_dft, 1), "runs": runs}
    print(json.dumps(out), flush=True)


def batch_report(args):
    """The batched form: many independent jobs of uneven size (grid, planes,
    visibility count, field) recorded once into a graph and replayed.  Plans
    per (grid, planes) shape (--replicas of them, the shape's jobs dealt to
    them in turn), tile and chunk picked by the autotuner on the shape's
    largest job, retargeted to each job's field.  Reports jobs/s, per-job
    latency percentiles (device timestamps between the jobs), the same jobs
    run eagerly, and the graph images against the eager ones; with --streams
    above 1 also the jobs spread over several streams inside the recording.
    Prints one JSON line."""
    import torch
    import synth
    from paper_2504_00959_amd import rick

    dev = "cuda:0"
    t0 = time.time()
    sizes = tuple(int(x) for x in args.grid_sizes.split(","))
    jobs = synth.batched_jobs(n_jobs=args.jobs, grid_sizes=sizes, device=dev)
    n = len(jobs)
    nvis = sum(ds.nvis for ds in jobs)
    print(f"[batch] generated {n} jobs, {nvis:,} visibilities in {time.time() - t0:.1f} s", file=sys.stderr,
          flush=True)
    uvw = [ds.uvw.contiguous() for ds in jobs]
    vis = [ds.vis.contiguous() for ds in jobs]
    shapes = {}
    for i, ds in enumerate(jobs):
        shapes.setdefault((ds.grid_n, ds.n_wplanes), []).append(i)
    stream = torch.cuda.Stream()
    tuned, plans, slot_of = {}, {}, {}
    t0 = time.time()
    for key, idx in sorted(shapes.items()):
        big = max(idx, key=lambda i: jobs[i].nvis)
        tile, chunk, ms = rick.autotune(jobs[big], uvw[big], vis[big], fused=True, stream=stream,
                                        orient=not args.no_orient)
        tuned[key] = (tile, chunk, ms)
        reps = max(1, min(args.replicas, len(idx)))
        for r in range(reps):
            mine = idx[r::reps]
            plans[(key, r)] = rick.Plan.for_dataset(jobs[big], max_vis=max(jobs[i].nvis for i in mine), tile=tile,
                                                    chunk=chunk, fused=True, orient=not args.no_orient)
            for i in mine:
                slot_of[i] = (key, r)
    print(f"[batch] autotuned {len(shapes)} shapes in {time.time() - t0:.1f} s; {len(plans)} plans",
          file=sys.stderr, flush=True)
    imgs = [torch.empty((ds.grid_n, ds.grid_n), dtype=torch.float32, device=dev) for ds in jobs]

    def issue(i, s):
        ds = jobs[i]
        p = plans[slot_of[i]]
        p.retarget(ds.fov, ds.w_min, ds.w_max)
        p.reset(s)
        p.grid(uvw[i], vis[i], None, ds.freq, s)
        p.fft(s)
        p.image(imgs[i], s)

    stamps = rick.Stamps(n + 1)
    # eager runs: reference images and timing
    eager_ms = []
    for rep in range(max(1, args.warmup)):
        stamps.stamp(0, stream)
        for i in range(n):
            issue(i, stream)
            stamps.stamp(i + 1, stream)
        eager_ms.append(stamps.elapsed(0, n))
    eager = [im.clone() for im in imgs]
    with rick.Graph.record(stream) as graph:
        stamps.stamp(0, stream)
        for i in range(n):
            issue(i, stream)
            stamps.stamp(i + 1, stream)
    totals, lat = [], []
    for rep in range(args.steps):
        for im in imgs:
            im.fill_(0.0)
        torch.cuda.synchronize()
        graph.launch(stream)
        totals.append(stamps.elapsed(0, n))
        lat = [stamps.elapsed(i, i + 1) for i in range(n)]
    seq_imgs = [im.clone() for im in imgs]
    # the same jobs on several streams: each plan stays on one stream, so its
    # jobs keep their order; plans are spread over the streams by the total
    # visibility count of their jobs, and the streams fork from and join the
    # first one
    S = max(1, min(args.streams, len(plans)))
    conc = None
    if S > 1:
        streams = [stream] + [torch.cuda.Stream() for _ in range(S - 1)]
        load, plan_stream = [0] * S, {}
        plan_jobs = {k: [i for i in range(n) if slot_of[i] == k] for k in plans}
        for key in sorted(plans, key=lambda k: -sum(jobs[i].nvis for i in plan_jobs[k])):
            j = min(range(S), key=lambda x: load[x])
            plan_stream[key] = j
            load[j] += sum(jobs[i].nvis for i in plan_jobs[key])
        per_stream = [[i for i in range(n) if plan_stream[slot_of[i]] == j] for j in range(S)]
        order = [lst[r] for r in range(max(len(x) for x in per_stream)) for lst in per_stream if r < len(lst)]
        cstamps = rick.Stamps(2 * n + 2)

        def issue_concurrent():
            cstamps.stamp(0, streams[0])
            ev = torch.cuda.Event()
            ev.record(streams[0])
            for st in streams[1:]:
                st.wait_event(ev)
            for i in order:
                st = streams[plan_stream[slot_of[i]]]
                cstamps.stamp(2 + 2 * i, st)
                issue(i, st)
                cstamps.stamp(3 + 2 * i, st)
            for st in streams[1:]:
                e = torch.cuda.Event()
                e.record(st)
                streams[0].wait_event(e)
            cstamps.stamp(1, streams[0])

        ceager = []
        for rep in range(max(1, args.warmup)):
            issue_concurrent()
            ceager.append(cstamps.elapsed(0, 1))
        with rick.Graph.record(stream) as cgraph:
            issue_concurrent()
        ctot, clat = [], []
        for rep in range(args.steps):
            for im in imgs:
                im.fill_(0.0)
            torch.cuda.synchronize()
            cgraph.launch(stream)
            ctot.append(cstamps.elapsed(0, 1))
            clat = [cstamps.elapsed(2 + 2 * i, 3 + 2 * i) for i in range(n)]
        torch.cuda.synchronize()
        conc_imgs = [im.clone() for im in imgs]
        cmed = float(np.median(ctot))
        cl = np.sort(np.asarray(clat))
        conc = {"streams": S, "plans": len(plans), "jobs_per_s": round(n / (cmed * 1e-3), 2),
                "batch_ms": round(cmed, 3),
                "mvis_per_s": round(nvis / (cmed * 1e-3) / 1e6, 1),
                "eager_batch_ms": round(float(np.median(ceager)), 3),
                "latency_ms": {"p50": round(float(np.percentile(cl, 50)), 3),
                               "p99": round(float(np.percentile(cl, 99)), 3), "max": round(float(cl[-1]), 3)}}
        cgraph.close()
        cstamps.close()
        for i in range(n):
            imgs[i].copy_(seq_imgs[i])
    # the jobs in rounds on one stream, each round's gridding ONE persistent
    # launch over the work items of all its jobs (rick_grid_jobs; one launch
    # per tile edge among them) and the fused column passes of its small grids
    # one launch per grid size (rick_wstack_image_jobs): round r holds the
    # r-th job of every plan
    plan_jobs = {k: [i for i in range(n) if slot_of[i] == k] for k in plans}
    rounds = [[lst[r] for lst in plan_jobs.values() if r < len(lst)]
              for r in range(max(len(x) for x in plan_jobs.values()))]
    jstamps = rick.Stamps(len(rounds) + 1)

    def issue_joint(s):
        jstamps.stamp(0, s)
        for ri, rd in enumerate(rounds):
            for i in rd:
                p = plans[slot_of[i]]
                p.retarget(jobs[i].fov, jobs[i].w_min, jobs[i].w_max)
                p.reset(s)
            rick.grid_jobs([(plans[slot_of[i]], uvw[i], vis[i], None, jobs[i].freq) for i in rd], s)
            for i in rd:
                plans[slot_of[i]].fft(s)
            rick.wstack_image_jobs([(plans[slot_of[i]], imgs[i]) for i in rd], s)
            jstamps.stamp(ri + 1, s)

    jeager = []
    for rep in range(max(1, args.warmup)):
        issue_joint(stream)
        jeager.append(jstamps.elapsed(0, len(rounds)))
    with rick.Graph.record(stream) as jgraph:
        issue_joint(stream)
    jtot, jround = [], []
    for rep in range(args.steps):
        for im in imgs:
            im.fill_(0.0)
        torch.cuda.synchronize()
        jgraph.launch(stream)
        jtot.append(jstamps.elapsed(0, len(rounds)))
        jround = [jstamps.elapsed(r, r + 1) for r in range(len(rounds))]
    torch.cuda.synchronize()
    joint_imgs = [im.clone() for im in imgs]
    jgraph.close()
    jstamps.close()
    for i in range(n):
        imgs[i].copy_(seq_imgs[i])
    jmed = float(np.median(jtot))
    # a job's latency is its round's (the round's jobs complete together)
    jl = np.sort(np.asarray([jround[r] for r, rd in enumerate(rounds) for _ in rd]))
    joint = {"rounds": len(rounds), "streams": 1, "jobs_per_s": round(n / (jmed * 1e-3), 2),
             "latency_ms": {"p50": round(float(np.percentile(jl, 50)), 3),
                            "p99": round(float(np.percentile(jl, 99)), 3), "max": round(float(jl[-1]), 3)},
             "batch_ms": round(jmed, 3), "mvis_per_s": round(nvis / (jmed * 1e-3) / 1e6, 1),
             "eager_batch_ms": [round(x, 3) for x in jeager],
             "round_ms": [round(x, 3) for x in jround]}
    # graph against eager in the apparent image (both multiplied by C_p C_q): the
    # shared-tile float atomics add in no fixed order, and dividing by the taper
    # magnifies that rounding in the outermost pixels of the corrected image
    import oracle.pixels
    from oracle import wstack as ow
    def apparent_rel(ds, a, b):
        c = torch.as_tensor(ow.grid_correction(ow.tap_table(ds.support, ds.oversample, ds.kernel,
                                                            ds.kernel_param), ds.grid_n), device=dev)
        c2 = c[:, None] * c[None, :]
        return float(torch.linalg.vector_norm((a - b).double() * c2) /
                     max(float(torch.linalg.vector_norm(b.double() * c2)), 1e-300))

    diffs = [apparent_rel(ds, a, b) for ds, a, b in zip(jobs, imgs, eager)]
    worst = max(diffs)
    if conc is not None:
        conc["vs_one_stream_max_apparent_rel_rms"] = max(
            apparent_rel(ds, a, b) for ds, a, b in zip(jobs, conc_imgs, seq_imgs))
    joint["vs_one_stream_max_apparent_rel_rms"] = max(
        apparent_rel(ds, a, b) for ds, a, b in zip(jobs, joint_imgs, seq_imgs))
    # the smallest job against the oracle at sampled pixels
    small = min(range(n), key=lambda i: jobs[i].nvis)
    ds = jobs[small]
    rng = np.random.default_rng(0)
    N = ds.grid_n
    pp = np.r_[N // 2, rng.integers(N // 4, 3 * N // 4, 5)]
    qq = np.r_[N // 2, rng.integers(N // 4, 3 * N // 4, 5)]
    dsh = synth.Dataset(uvw=ds.uvw.cpu().numpy(), freq=ds.freq, vis=ds.vis.cpu().numpy(), weight=None,
                        grid_n=ds.grid_n, n_wplanes=ds.n_wplanes, support=ds.support, oversample=ds.oversample,
                        fov=ds.fov, w_min=ds.w_min, w_max=ds.w_max)
    ref, _, kept, _ = oracle.pixels.wstack_pixels(dsh.uvw, dsh.freq, dsh.vis, None, pp, qq, **dsh.plan_kwargs())
    got = imgs[small].double().cpu().numpy()[qq, pp]
    corr = ow.grid_correction(ow.tap_table(ds.support, ds.oversample, ds.kernel, ds.kernel_param), N)
    c2 = corr[pp] * corr[qq]
    ocheck = float(np.linalg.norm((got - ref) * c2) / np.linalg.norm(ref * c2))
    med = float(np.median(totals))
    lat_sorted = np.sort(np.asarray(lat))
    out = {"report": "batch", "jobs": n, "grid_sizes": list(sizes), "n_vis": nvis, "steps": args.steps,
           "jobs_per_s": round(n / (med * 1e-3), 2), "batch_ms": round(med, 3),
           "mvis_per_s": round(nvis / (med * 1e-3) / 1e6, 1),
           "latency_ms": {"p50": round(float(np.percentile(lat_sorted, 50)), 3),
                          "p99": round(float(np.percentile(lat_sorted, 99)), 3),
                          "max": round(float(lat_sorted[-1]), 3)},
           "eager_batch_ms": round(float(np.median(eager_ms)), 3),
           "graph_vs_eager_max_apparent_rel_rms": worst,
           "graph_vs_eager_apparent_rel_rms": [float("%.3g" % d) for d in diffs],
           "job_shapes": [f"{ds.grid_n}x{ds.n_wplanes}:{ds.nvis}" for ds in jobs],
           "oracle_check": {"job": small, "pixels": int(len(pp)), "apparent_rel_rms": ocheck},
           "concurrent": conc,
           "joint_gridding": joint,
           "shapes": {f"{k[0]}x{k[1]}": {"jobs": len(shapes[k]), "tile": v[0], "chunk": v[1],
                                         "tuned_ms": round(v[2], 3)} for k, v in sorted(tuned.items())}}
    print(json.dumps(out), flush=True)
    graph.close()
    stamps.close()
    for p in plans.values():
        p.close()


def predict_report(args):
    """Prediction (degridding): the workload's visibility positions predicted
    from a model image holding its point sources on pixels.  One step is
    rick_predict_planes (screened model planes, centred FFT) plus rick_degrid
    over every visibility, inputs resident on the device.  Reports Mvis/s,
    per-kernel times and rates, and sampled visibilities against the oracle's
    sparse-model prediction.  Prints one JSON line."""
    import torch
    import synth
    from paper_2504_00959_amd import rick

    dev = "cuda:0"
    ds = make_workload(args.workload, dev) if args.workload != "ska_low_share" else \
        synth.ska_low_share(device=dev, with_vis=False)
    print(f"[predict] {describe(ds)}", file=sys.stderr, flush=True)
    N = ds.grid_n
    dl = ds.fov / N
    pp = np.rint(np.asarray(ds.sources["l"]) / dl).astype(np.int64) + N // 2
    qq = np.rint(np.asarray(ds.sources["m"]) / dl).astype(np.int64) + N // 2
    fl = np.asarray(ds.sources["flux"], dtype=np.float64)
    uvw = torch.as_tensor(ds.uvw, dtype=torch.float64).to(dev).contiguous()
    nrow = uvw.shape[0]
    nchan = 1 if ds.freq is None else len(ds.freq)
    nvis = nrow * nchan
    with rick.Plan.for_dataset(ds, precision=args.precision, fused=not args.unfused, timing=True,
                               max_vis=1) as p:
        M = torch.zeros((N, N), dtype=p.real_dtype, device=dev)
        M.index_put_((torch.as_tensor(qq, device=dev), torch.as_tensor(pp, device=dev)),
                     torch.as_tensor(fl, dtype=p.real_dtype, device=dev), accumulate=True)
        out = torch.empty((nrow, nchan), dtype=p.complex_dtype, device=dev)

        def timed(step):
            for _ in range(args.warmup):
                step()
            torch.cuda.synchronize()
            p.info()                      # restart the kernel timers
            t0 = time.perf_counter()
            for _ in range(args.steps):
                step()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) * 1e3 / args.steps, p.info()["timers"]

        def step_direct():
            p.predict_planes(M)
            p.degrid(uvw, ds.freq, out)

        ms_direct, timers_direct = timed(step_direct)
        rng = np.random.default_rng(62)
        rows = np.sort(rng.choice(nrow, min(40, nrow), replace=False))
        got = out[torch.as_tensor(rows, device=dev)].cpu().numpy().astype(np.complex128).reshape(-1)
        uvw_s = uvw[torch.as_tensor(rows, device=dev)].cpu().numpy()
        # the same positions quantised and sorted once (repeated prediction)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        order = p.degrid_order(uvw, ds.freq)
        order_ms = (time.perf_counter() - t0) * 1e3
        out2 = torch.empty_like(out)

        def step_sorted():
            p.predict_planes(M)
            p.degrid_sorted(order, out2)

        ms, timers = timed(step_sorted)
        sorted_vs_direct = float((out2 - out).abs().max() / out.abs().max())
        got = out2[torch.as_tensor(rows, device=dev)].cpu().numpy().astype(np.complex128).reshape(-1)
        order.close()
    import oracle.predict
    t1 = time.time()
    ref = oracle.predict.wstack_predict_sparse(pp, qq, fl, uvw_s, ds.freq, **ds.plan_kwargs())
    chk = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    rb = 8 if args.precision == "fp64" else 4
    mesh_b = 2 * rb * ds.n_wplanes * N * N
    kern = {}
    for name, (kms, calls) in list(timers.items()) + [("degrid_direct", timers_direct["degrid"])]:
        e = {"ms": round(kms, 4), "calls": calls}
        byt = {"predict_screen": mesh_b + rb * N * N,
               "predict_fft": 4 * mesh_b,
               "degrid": 16 * nvis + 2 * rb * nvis,
               "degrid_direct": 24 * nrow + 2 * rb * nvis}.get(name)
        if byt:
            e["bytes"] = int(byt)
            e["GBps"] = round(byt / (kms * 1e-3) / 1e9, 1)
        if name.startswith("degrid"):
            e["tap_bytes_gathered"] = int(2 * rb * ds.support ** 2 * nvis)
        kern[name] = e
    out_line = {"report": "predict", "workload": describe(ds), "n_vis": nvis, "steps": args.steps,
                "ms_per_step": round(ms, 4), "mvis_per_s": round(nvis / (ms * 1e-3) / 1e6, 1),
                "order": "sorted once (rick_degrid_order_create), interpolation in sorted order",
                "order_create_ms": round(order_ms, 2),
                "direct_ms_per_step": round(ms_direct, 4),
                "direct_mvis_per_s": round(nvis / (ms_direct * 1e-3) / 1e6, 1),
                "sorted_vs_direct_max_rel": sorted_vs_direct,
                "precision": args.precision, "model": f"{len(fl)} point sources on pixels",
                "kernels": kern,
                "check": {"rows": int(len(rows)), "visibilities": int(got.size), "rel_rms_vs_oracle": chk,
                          "oracle_seconds": round(time.time() - t1, 1)}}
    print(json.dumps(out_line), flush=True)


def learned_report(args):
    """The learned-kernel form: train the MLP kernel on generated scenes
    against the direct Fourier sum (256^2 grids, 16 planes, support 7,
    oversample 64), then image the SKA-LOW-like 209.3M-visibility workload
    with the Gaussian, Kaiser-Bessel and learned kernels at equal support and
    report each one's distance to the direct sum on two 128^2 patches and its
    Mvis/s.  Prints one JSON line."""
    import torch
    import synth
    from paper_2504_00959_amd import rick
    from paper_2504_00959_amd.learned import LearnedKernel

    dev = "cuda:0"
    n_train, n_eval = args.scenes, args.eval_scenes
    t0 = time.time()
    s0 = synth.learned_scene(0, nvis=args.scene_vis)
    lk = LearnedKernel(grid_n=s0.grid_n, n_wplanes=s0.n_wplanes, support=s0.support, oversample=s0.oversample,
                       fov=s0.fov, w_min=s0.w_min, w_max=s0.w_max, max_vis=args.scene_vis, n_wbins=args.wbins,
                       seed=args.seed)
    data = []
    for i in range(n_train + n_eval):
        ds = synth.learned_scene(i, nvis=args.scene_vis, device=dev)
        uvw = torch.as_tensor(ds.uvw, dtype=torch.float64, device=dev)
        data.append((uvw, ds.vis, lk.target(uvw, ds.vis)))
        if i % 50 == 0:
            print(f"[learned] scene {i}: {len(ds.sources['l'])} sources ({time.time() - t0:.1f} s)", file=sys.stderr,
                  flush=True)
    torch.cuda.synchronize()
    t_data = time.time() - t0
    geo = lk.geo
    kb = rick.Plan(**geo, max_vis=args.scene_vis, kernel="kb")

    def held_out(plan):
        sums = torch.zeros((n_eval, 2), dtype=torch.float64, device=dev)
        for j in range(n_eval):
            uvw, vis, D = data[n_train + j]
            lk.loss(plan, uvw, vis, D, sums[j])
        s = sums.cpu().numpy()
        return float(np.mean(s[:, 0] / s[:, 1]))

    res = {"gaussian": held_out(lk.gauss), "kaiser_bessel": held_out(kb)}
    t0 = time.time()
    fit = lk.fit_table(lk.gaussian_table(), steps=args.fit_steps, lr=3e-3)
    lk.install()
    res["learned_start"] = held_out(lk.plan)
    print(f"[learned] start from the Gaussian table: fit mse {fit:.3e}, held-out loss {res['learned_start']:.4e} "
          f"(Gaussian {res['gaussian']:.4e}, KB {res['kaiser_bessel']:.4e})", file=sys.stderr, flush=True)
    rng = np.random.default_rng(args.seed)
    curve = []
    # the parameters kept are those of the epoch with the lowest held-out loss
    # (the start, fitted to the Gaussian table, included)
    best, best_loss, best_epoch = lk.snapshot(), res["learned_start"], 0
    t1 = time.time()
    for ep in range(args.epochs):
        sums = torch.zeros((n_train, 2), dtype=torch.float64, device=dev)
        for i in rng.permutation(n_train):
            uvw, vis, D = data[i]
            lk.step(uvw, vis, D, sums[i], args.lr)
        s = sums.cpu().numpy()
        lk.install()
        curve.append({"epoch": ep + 1, "train_loss": float(np.mean(s[:, 0] / s[:, 1])),
                      "held_out_loss": held_out(lk.plan)})
        if curve[-1]["held_out_loss"] < best_loss:
            best, best_loss, best_epoch = lk.snapshot(), curve[-1]["held_out_loss"], ep + 1
        print(f"[learned] epoch {ep + 1}: {curve[-1]}", file=sys.stderr, flush=True)
    t_train = time.time() - t1
    steps = args.epochs * n_train
    lk.restore(best)
    lk.install()
    res["learned"] = best_loss
    res["learned_epoch"] = best_epoch
    table = lk.table.clone()
    kb.close()

    # evaluation at the SKA-LOW-like shape
    ds = synth.ska_low_share(device=dev)
    uvw = torch.as_tensor(ds.uvw, dtype=torch.float64).to(dev)
    N = ds.grid_n
    off = int(round(0.3 * N))
    patches = {"centre": (N // 2 - 64, N // 2 - 64), "offset": (N // 2 - 64 + off, N // 2 - 64 + off)}
    t0 = time.time()
    with rick.Plan.for_dataset(ds) as pg:
        dft = {k: pg.dft_image(uvw, ds.vis, None, ds.freq, q0=q0, p0=p0, nq=128, np_=128).cpu().numpy()
               for k, (q0, p0) in patches.items()}
    t_dft = time.time() - t0
    evals = {}
    for name, kw in (("gaussian", {}), ("kaiser_bessel", {"kernel": "kb"}),
                     ("learned", {"kernel": "user_lut", "lut_wbins": args.wbins})):
        plan = rick.Plan.for_dataset(ds, fused=True, **kw)
        if name == "learned":
            plan.set_lut(table)
        img = torch.empty((N, N), dtype=torch.float32, device=dev)
        stream = torch.cuda.current_stream()

        def one():
            plan.reset(stream)
            plan.grid(uvw, ds.vis, None, ds.freq, stream)
            plan.fft(stream)
            plan.image(img, stream)

        one()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            one()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        im = img.double().cpu().numpy()
        ev = {"ms_per_step": round(ms, 3), "mvis_per_s": round(ds.nvis / (ms * 1e-3) / 1e6, 1)}
        for k, (q0, p0) in patches.items():
            d = dft[k]
            ev[f"vs_dft_{k}"] = float(np.linalg.norm(im[q0:q0 + 128, p0:p0 + 128] - d) / np.linalg.norm(d))
        evals[name] = ev
        print(f"[learned] {name} at {N}^2 x {ds.n_wplanes}: {ev}", file=sys.stderr, flush=True)
        plan.close()
        del img, plan
        torch.cuda.empty_cache()
    out = {"report": "learned_kernel",
           "training": {"scenes": n_train, "held_out_scenes": n_eval, "vis_per_scene": args.scene_vis,
                        "grid": f"{geo['grid_n']}^2 x {geo['n_wplanes']} planes", "support": geo["support"],
                        "oversample": geo["oversample"], "w_fraction_bins": args.wbins, "epochs": args.epochs,
                        "steps": steps, "lr": args.lr, "start": "MLP fitted to the Gaussian table",
                        "fit_steps": args.fit_steps, "fit_mse": fit, "seconds": round(t_train, 1),
                        "ms_per_step": round(1e3 * t_train / max(1, steps), 2),
                        "data_and_targets_seconds": round(t_data, 1)},
           "held_out_loss": res, "curve": curve,
           "evaluation": {"workload": describe(ds), "patches": {k: [q0, p0, 128, 128] for k, (q0, p0) in
                                                                 patches.items()},
                          "dft_seconds": round(t_dft, 1), "kernels": evals}}
    lk.close()
    print(json.dumps(out), flush=True)


def describe(ds):
    return (f"{ds.name}: {ds.nrow:,} rows x {ds.nchan} channels = {ds.nvis:,} visibilities, "
            f"{ds.grid_n}^2 x {ds.n_wplanes} w-planes, support {ds.support}, oversample {ds.oversample}, "
            f"{ds.kernel} kernel")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ska_low_precision",
                    help="ska_low_precision (418.6M visibilities, 8192^2 x 128 planes; the default) or "
                         "ska_low_share (209.3M, 4096^2 x 64), tiny, ska_low_small")
    ap.add_argument("--precision", default=None, choices=["fp32", "fp32_kahan", "fp64"],
                    help="default: fp32_kahan for ska_low_precision, fp32 otherwise")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--unfused", action="store_true",
                    help="column FFT and w-screen as separate kernels (F_k written to HBM)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the image check (oracle and direct sum at sampled pixels, float64 GPU image)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (scale for HBM byte counters)")
    ap.add_argument("--profile", metavar="OUT",
                    help="run the rocprofv3 passes (kernel trace, HBM byte counters with copy calibration, SQ "
                         "counters) on this workload as child processes and summarise them in OUT/summary")
    ap.add_argument("--summarize", metavar="OUT", help="only rewrite the summaries of an earlier --profile OUT")
    ap.add_argument("--precision-report", action="store_true",
                    help="run fp32, fp32_kahan and fp64 on the workload and report each image's error against the "
                         "float64 GPU image, the oracle and the direct Fourier sum at sampled pixels")
    ap.add_argument("--patch", type=int, default=8, help="edge of the centre pixel patch of --precision-report")
    ap.add_argument("--batch", action="store_true",
                    help="the batched form: many uneven jobs recorded into a graph and replayed (jobs/s, latency)")
    ap.add_argument("--jobs", type=int, default=64, help="number of jobs of --batch")
    ap.add_argument("--grid-sizes", default="512,1024,2048,4096",
                    help="--batch: grid sizes the jobs are drawn from (comma-separated)")
    ap.add_argument("--replicas", type=int, default=2,
                    help="--batch: plans per (grid, planes) shape, the shape's jobs dealt to them in turn")
    ap.add_argument("--no-orient", action="store_true",
                    help="--batch: keep every plane in its own orientation (no transposed planes)")
    ap.add_argument("--streams", type=int, default=4,
                    help="streams of the concurrent run of --batch (1 = only the one-stream run)")
    ap.add_argument("--learned", action="store_true",
                    help="the learned-kernel form: train on generated scenes against the direct sum, then compare "
                         "with the Gaussian and Kaiser-Bessel kernels on the SKA-LOW-like workload")
    ap.add_argument("--scenes", type=int, default=200, help="training scenes of --learned")
    ap.add_argument("--eval-scenes", type=int, default=16, help="held-out scenes of --learned")
    ap.add_argument("--scene-vis", type=int, default=1_000_000, help="visibilities per scene of --learned")
    ap.add_argument("--epochs", type=int, default=10, help="passes over the training scenes of --learned")
    ap.add_argument("--lr", type=float, default=2e-4, help="Adam step of --learned")
    ap.add_argument("--fit-steps", type=int, default=1500, help="steps fitting the MLP to the Gaussian table")
    ap.add_argument("--wbins", type=int, default=4, help="w-fraction bins of the learned table")
    ap.add_argument("--seed", type=int, default=0, help="initial MLP parameters of --learned")
    ap.add_argument("--predict", action="store_true",
                    help="prediction (degridding) of the workload's visibilities from a point-source model image")
    args = ap.parse_args()
    if args.precision is None:
        args.precision = "fp32_kahan" if args.workload == "ska_low_precision" else "fp32"
    if args.profile:
        run_profiles(os.path.abspath(args.profile), args.workload)
        return
    if args.summarize:
        summarize_profiles(os.path.abspath(args.summarize), args.workload)
        return
    if args.precision_report:
        precision_report(args)
        return
    if args.batch:
        batch_report(args)
        return
    if args.predict:
        predict_report(args)
        return
    if args.learned:
        learned_report(args)
        return
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: the imager runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding the planes over several GPUs is designed, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_00959_amd import rick

    dev = "cuda:0"
    t0 = time.time()
    ds = make_workload(args.workload, dev)
    print(f"[bench] generated {describe(ds)} in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    uvw = torch.as_tensor(ds.uvw, dtype=torch.float64).to(dev)
    cd = torch.complex128 if args.precision == "fp64" else torch.complex64
    vis = ds.vis.to(dtype=cd).contiguous()
    wt = None
    plan = rick.Plan.for_dataset(ds, precision=args.precision, timing=True, tile=args.tile, chunk=args.chunk,
                                 fused=not args.unfused)
    stream = torch.cuda.current_stream()
    img = torch.empty((ds.grid_n, ds.grid_n), dtype=plan.real_dtype, device=dev)

    def step():
        plan.reset(stream)
        plan.grid(uvw, vis, wt, ds.freq, stream)
        plan.fft(stream)
        plan.image(img, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.info()                                  # clears the per-kernel timers
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    info = plan.info()
    ms_step = ms_total / args.steps
    value = ds.nvis / (ms_step * 1e-3) / 1e6
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step", file=sys.stderr, flush=True)

    kernels = {}
    for name, (ms, calls) in info["timers"].items():
        kernels[name] = {"ms": round(ms, 4), "calls": calls}
    dominant = max((k for k in kernels if algorithmic_bytes(k, ds, info) is not None),
                   key=lambda k: kernels[k]["ms"])
    dbytes = algorithmic_bytes(dominant, ds, info)
    achieved = dbytes / (kernels[dominant]["ms"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "algorithmic_bytes": int(dbytes), "launch_ms": kernels[dominant]["ms"]}
    for k, v in kernels.items():
        ab = algorithmic_bytes(k, ds, info)
        if ab is not None:
            v["bytes"] = int(ab)
            v["GBps"] = round(ab / (v["ms"] * 1e-3) / 1e9, 1)
    roofline["traffic"], roofline["traffic_note"] = measured_traffic(args.workload, dominant)
    valu = measured_valu(args.workload, dominant)
    if valu is not None:
        # the FFT and gridding kernels are bound by instruction issue rather
        # than HBM: one VALU wave instruction per clock per CU (no packed math)
        cap = kernels[dominant]["ms"] * 1e-3 * CU_COUNT * CLOCK_HZ
        roofline["valu_issue"] = {"insts_per_launch": valu, "issue_slots": round(cap),
                                  "frac": round(valu / cap, 3), "source": "SQ_INSTS_VALU, committed SQ summary"}
    if roofline["traffic"] is not None:
        roofline["traffic_over_algorithmic"] = round(roofline["traffic"] / dbytes, 3)

    img_host = img.double().cpu().numpy()
    plan.close()
    del plan, img, vis
    torch.cuda.empty_cache()

    # ---- checks and the CPU baseline (after the timed region) ----
    from oracle import wstack as ow
    N = ds.grid_n
    corr = ow.grid_correction(ow.tap_table(ds.support, ds.oversample, ds.kernel, ds.kernel_param), N)
    check = None
    vis_host = None
    if not args.no_check or not args.no_cpu_baseline:
        vis_host = ds.vis.cpu().numpy()
    if not args.no_check:
        check = {"n_gridded": info["n_gridded"]}
        if args.precision != "fp64":
            # the same image in the all-float64 mode of the library (unfused: its
            # fused form needs a second mesh-sized buffer), whole-image errors
            t0 = time.time()
            p64 = rick.Plan.for_dataset(ds, precision="fp64", fused=False)
            i64 = torch.empty((N, N), dtype=torch.float64, device=dev)
            v64 = ds.vis.to(torch.complex128)
            p64.reset(stream)
            p64.grid(uvw, v64, wt, ds.freq, stream)
            p64.fft(stream)
            p64.image(i64, stream)
            torch.cuda.synchronize()
            ref = i64.cpu().numpy()
            p64.close()
            del p64, i64, v64
            torch.cuda.empty_cache()
            c2 = np.outer(corr, corr)
            d = img_host - ref
            central = c2 >= 0.1
            check["vs_fp64_gpu"] = {
                "apparent_rel_rms": float(np.linalg.norm(d * c2) / np.linalg.norm(ref * c2)),
                "central_rel_rms": float(np.linalg.norm(d[central]) / np.linalg.norm(ref[central])),
                "image_rel_rms": float(np.linalg.norm(d) / np.linalg.norm(ref)),
                "seconds": round(time.time() - t0, 1)}
            del ref, d, c2
            print(f"[bench] vs float64 GPU image: {check['vs_fp64_gpu']}", file=sys.stderr, flush=True)
        pp, qq = check_pixels(ds)
        check.update(oracle_leg(ds, vis_host, img_host[qq, pp], pp, qq, corr))
        check["tolerances"] = {"gpu_vs_oracle_apparent": TOL_ORACLE, "dft_gate": TOL_DFT,
                               "vs_fp64_gpu_apparent": TOL_ORACLE}
        ok = check["gpu_vs_oracle"]["apparent_rel_rms"] <= TOL_ORACLE
        if "dft_gate" in check:
            ok = ok and check["dft_gate"] <= TOL_DFT
        if "vs_fp64_gpu" in check:
            ok = ok and check["vs_fp64_gpu"]["apparent_rel_rms"] <= TOL_ORACLE
        check["pass"] = bool(ok)
        print(f"[bench] check: gpu vs oracle {check['gpu_vs_oracle']}, gpu vs dft {check.get('gpu_vs_dft')}, "
              f"oracle vs dft {check.get('oracle_vs_dft')}, pass={ok}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        nthr = host_threads()
        t0 = time.time()
        one = cpu_baseline(ds, vis_host, 1)
        print(f"[bench] cpu baseline, 1 thread: {one['value']:.3f} Mvis/s ({time.time() - t0:.1f} s)",
              file=sys.stderr, flush=True)
        cpu = one
        if nthr > 1:
            t0 = time.time()
            cpu = cpu_baseline(ds, vis_host, nthr)
            print(f"[bench] cpu baseline, {nthr} threads: {cpu['value']:.3f} Mvis/s ({time.time() - t0:.1f} s)",
                  file=sys.stderr, flush=True)
            cpu["single_thread"] = {k: one[k] for k in ("value", "sample_seconds", "est_seconds_per_image")}
        cpu["cpu_model"] = cpu_model()

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mvis/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": describe(ds), "n_vis": ds.nvis, "grid_n": ds.grid_n, "n_wplanes": ds.n_wplanes,
                   "support": ds.support, "oversample": ds.oversample, "precision": args.precision,
                   "tile": info["tile"], "chunk": info["chunk"], "fused_screen": not args.unfused,
                   "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "check": check,
    }
    print(json.dumps(out), flush=True)
    if check is not None and not check["pass"]:
        print("[bench] image check failed: the throughput above is not valid", file=sys.stderr, flush=True)
        sys.exit(3)


if __name__ == "__main__":
    main()

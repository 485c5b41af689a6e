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
METRIC = "Mvis/s through grid+iFFT+w-stack at fixed image RMS vs FP64 DFT oracle"


def algorithmic_bytes(name, ds, info):
    """Bytes the method must move per launch of kernel `name` (records are
    12 B: packed position + complex64 W V; replicas of tile-straddling
    records are not counted)."""
    nvis, nrow = ds.nvis, ds.nrow
    cells = ds.n_wplanes * ds.grid_n * ds.grid_n
    wbytes = 4 * nvis if ds.weight is not None else 0
    table = {
        "bin_count": 24 * nrow + wbytes,
        "bin_scatter": 24 * nrow + 8 * nvis + wbytes + 12 * nvis,
        "grid": 12 * nvis + 8 * cells,
        "fft_rows": 16 * cells,
        "fft_cols": 16 * cells,
        "wscreen": 8 * cells + 4 * ds.grid_n * ds.grid_n,
        "fft_cols_screen": 8 * cells + 4 * ds.grid_n * ds.grid_n,
    }
    return table.get(name)


def cpu_baseline(ds, vis_host, n_rows_sample=262_144, n_planes_sample=2):
    """The float64 oracle, as it stands, timed stage by stage on a bounded sample
    of the same workload and scaled to the whole job:
      T = (t_bin + t_grid) / n_sample_vis * N_vis + N_w * (t_fft_plane + t_screen_plane)."""
    import oracle
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
    t0 = time.perf_counter()
    b = ow.bin_visibilities(uvw_s, ds.freq, vis_s, wt_s, **geo)
    t_bin = time.perf_counter() - t0
    table = ow.tap_table(ds.support, ds.oversample, ds.kernel, ds.kernel_param)
    keep = np.nonzero(b.keep)[0]
    kk = b.k[keep]
    planes = np.argsort(-np.bincount(kk, minlength=ds.n_wplanes))[:n_planes_sample]
    G = np.zeros((1, ds.grid_n, ds.grid_n), np.complex128)
    t_grid, n_grid = 0.0, 0
    for k in planes:
        idx = keep[kk == k]
        G[0] = 0
        t0 = time.perf_counter()
        ow.grid_plane(G[0], b, idx, table)
        t_grid += time.perf_counter() - t0
        n_grid += idx.size
    t0 = time.perf_counter()
    F = ow.ifft_planes(G)
    t_fft = time.perf_counter() - t0
    t0 = time.perf_counter()
    S = ow.screen_sum(F, ow.plane_centres(ds.w_min, ds.w_max, ds.n_wplanes)[:1], ds.fov)
    corr = ow.grid_correction(table, ds.grid_n)
    ow.normalise(S, corr, 1.0, ds.fov)
    t_screen = time.perf_counter() - t0
    per_vis = t_bin / n_s + (t_grid / n_grid if n_grid else 0.0)
    total = per_vis * ds.nvis + ds.n_wplanes * (t_fft + t_screen)
    sample = (f"oracle stages timed on {n_s:,} visibilities ({uvw_s.shape[0]:,} rows x {ds.nchan} channels, "
              f"binned), {n_grid:,} of them gridded onto {len(planes)} plane(s), one {ds.grid_n}^2 plane "
              f"transformed and screened; per-visibility and per-plane costs scaled to {ds.nvis:,} "
              f"visibilities and {ds.n_wplanes} planes (est. {total:.1f} s per image)")
    return {"value": ds.nvis / total / 1e6, "unit": "Mvis/s", "cores": 1, "kind": "oracle", "sample": sample,
            "sample_seconds": round(t_bin + t_grid + t_fft + t_screen, 2)}


def make_workload(name, device):
    import synth
    if name == "ska_low_share":
        return synth.ska_low_share(device=device)
    if name == "tiny":
        return synth.tiny(device=device)
    if name == "ska_low_small":
        return synth.ska_low_small(device=device)
    raise SystemExit(f"unknown workload {name}")


def describe(ds):
    return (f"{ds.name}: {ds.nrow:,} rows x {ds.nchan} channels = {ds.nvis:,} visibilities, "
            f"{ds.grid_n}^2 x {ds.n_wplanes} w-planes, support {ds.support}, oversample {ds.oversample}, "
            f"{ds.kernel} kernel")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ska_low_share")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp32_kahan", "fp64"])
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--unfused", action="store_true",
                    help="column FFT and w-screen as separate kernels (F_k written to HBM)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check-pixels", type=int, default=6,
                    help="pixels of the timed image checked against the float64 oracle (0 = skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (scale for HBM byte counters)")
    args = ap.parse_args()
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
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the plane-sharded multi-GPU path is a design, not code)", file=sys.stderr)
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
            v["GBps"] = round(ab / (v["ms"] * 1e-3) / 1e9, 1)

    check = None
    vis_host = None
    if args.check_pixels > 0 or not args.no_cpu_baseline:
        vis_host = ds.vis.cpu().numpy()
    if args.check_pixels > 0:
        import oracle.pixels
        rng = np.random.default_rng(0)
        N = ds.grid_n
        pp = np.r_[N // 2, rng.integers(N // 4, 3 * N // 4, args.check_pixels - 1)]
        qq = np.r_[N // 2, rng.integers(N // 4, 3 * N // 4, args.check_pixels - 1)]
        t0 = time.time()
        ref, _, kept, sw = oracle.pixels.wstack_pixels(ds.uvw, ds.freq, vis_host, ds.weight, pp, qq,
                                                       **ds.plan_kwargs())
        got = img.double().cpu().numpy()[qq, pp]
        from oracle import wstack as ow
        corr = ow.grid_correction(ow.tap_table(ds.support, ds.oversample, ds.kernel, ds.kernel_param), N)
        c2 = corr[pp] * corr[qq]
        err = float(np.linalg.norm((got - ref) * c2) / np.linalg.norm(ref * c2))
        check = {"pixels": int(len(pp)), "apparent_rel_rms": err, "n_gridded": info["n_gridded"],
                 "oracle_kept": kept, "seconds": round(time.time() - t0, 1)}
        print(f"[bench] sampled-pixel check: apparent-image rel-RMS = {err:.2e} ({time.time() - t0:.1f} s)",
              file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.time()
        cpu = cpu_baseline(ds, vis_host)
        print(f"[bench] cpu baseline {cpu['value']:.3f} Mvis/s ({time.time() - t0:.1f} s)", file=sys.stderr,
              flush=True)

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
    plan.close()


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark: images searched per second on one MI355X.

A step is one full search of a synthetic segment at survey shape: 351
baselines (27-antenna Y array), 2048 integrations of 10 ms, 256 channels over
1-2 GHz, 2 polarisations, 128 DM trials over 0-1000 pc cm^-3, boxcar widths
{1, 2, 4, 8}, 1024 x 1024 images: 491,520 images per segment, with five
injected S/N 20 dispersed pulses.  The visibilities are resident in HBM before
the timed region; a step ends with the sorted candidate list on the host.

    python bench.py [--steps K] [--warmup W] [--storage cf32|cf16]

Prints one JSON line (rank 0).  Also reports the real-time factor (segment
duration / wall time per step), per-entry-point kernel timings measured with
HIP events on the launch stream, the roofline of the dominant kernel, and the
CPU oracle's rate on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, published
FP32_PEAK_TFLOPS = 157.3    # MI355X fp32 vector, published


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(p, vis, n_images_target, procs):
    """The CPU oracle, as it stands, on a bounded sample of the workload's
    images (DM indices spread over the grid x every width x integrations
    spread over the segment), run in a process pool."""
    import multiprocessing as mp
    import numpy as np
    import oracle
    du, dv = p.cell()
    plan = oracle.Plan(p.freq(), p.uvw(), p.tint_s, p.dms, p.widths, p.npix, du, dv,
                       kdm=p.kdm, threshold=p.threshold, nint=p.nint)
    ndm = len(p.dms)
    per = max(1, n_images_target // (4 * len(p.widths)))
    sample = []
    for i in np.linspace(0, ndm - 1, 4).astype(int):
        for j, w in enumerate(p.widths):
            K = p.nint // w
            for k in np.linspace(0, K - 1, per).astype(int):
                sample.append((int(i), j, int(k)))
    global _CPU_CTX
    _CPU_CTX = (vis, plan)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        res = pool.map(_cpu_one, sample, chunksize=1)
    dt = time.perf_counter() - t0
    return len(sample), dt, res


_CPU_CTX = None


def _cpu_one(key):
    import oracle
    vis, plan = _CPU_CTX
    i, j, k = key
    img = oracle.image_at(vis, plan, i, j, k)
    return key, oracle.image_stats(img)


def event_time(fn, reps, stream):
    import torch
    fn()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / reps * 1e-3  # seconds per call


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--storage", choices=["cf32", "cf16"], default="cf32")
    ap.add_argument("--workload", choices=["survey", "tiny"], default="survey")
    ap.add_argument("--cpu-images", type=int, default=96)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-leg", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: segments are independent, so N GPUs would each "
              "search their own segments with no exchange (run N=1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import rfgen

    p = rfgen.survey() if args.workload == "survey" else rfgen.tiny()
    t = time.perf_counter()
    vis = p.make_vis()
    log(f"generated {p.name} segment {vis.shape} {vis.nbytes / 1e9:.2f} GB in {time.perf_counter() - t:.1f}s")

    cpu = None
    if not args.no_cpu_baseline:
        procs = max(1, min(16, os.cpu_count() or 1))
        n, dt, _ = cpu_baseline(p, vis, args.cpu_images, procs)
        cpu = {"value": n / dt, "unit": "images/s", "cores": procs, "kind": "oracle",
               "sample": f"{n} images of the {p.name} workload (4 DM trials spread over the grid x "
                         f"{len(p.widths)} widths x integrations spread over the segment), float64 numpy, "
                         f"{procs} processes, {dt:.1f} s wall"}
        log(f"cpu oracle: {n} images in {dt:.1f}s on {procs} processes = {n / dt:.1f} img/s")

    import torch
    import paper_1802_03084_amd as rf

    dtype = rf.RF_CF32 if args.storage == "cf32" else rf.RF_CF16
    du, dv = p.cell()
    dev = torch.device("cuda:0")
    if dtype == rf.RF_CF32:
        dvis = torch.from_numpy(vis).to(dev)
    else:
        dvis = torch.from_numpy(rfgen.to_cf16(vis)).to(dev)
    plan = rf.Plan(p.freq(), p.uvw(), p.tint_s, p.dms, p.widths, p.npix, du, dv, nint=p.nint,
                   npol=p.npol, vis_dtype=dtype, kdm=p.kdm, threshold=p.threshold)
    ws = plan.workspace(rf.RF_OP_SEGMENT)
    stream = torch.cuda.current_stream()
    log(f"plan: {plan.n_images} images, W={plan.W}, cells={plan.info['n_cells']}, "
        f"rows={plan.info['n_rows']}, workspace {ws.numel() / 1e9:.2f} GB")

    cap = 65536
    for w in range(args.warmup):
        t = time.perf_counter()
        rows, n, _ = plan.search_segment(dvis, cap=cap, ws=ws)
        log(f"warmup {w}: {time.perf_counter() - t:.2f}s, {n} candidates")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        rows, n, _ = plan.search_segment(dvis, cap=cap, ws=ws)
        log(f"step {k} done at {time.perf_counter() - t0:.2f}s, {n} candidates")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_s = wall / args.steps
    img_s = plan.n_images / step_s
    seg_s = p.nint * p.tint_s
    keys = {(int(r["dm_idx"]), int(r["width_idx"]), int(r["t_int"]), int(r["x"]), int(r["y"])) for r in rows}
    found = sum((q.dm_idx, q.width_idx, q.t0, q.x, q.y) in keys for q in p.pulses)
    log(f"{img_s:.0f} images/s, {step_s * 1e3:.1f} ms/step, RTF {seg_s / step_s:.2f}, "
        f"pulses recovered {found}/{len(p.pulses)}, candidates {n}")

    kernels = {}
    roof = None
    if not args.no_kernel_leg:
        N = p.npix
        nb = 64
        per_int = p.nbl * p.nchan * p.npol
        dd = plan.empty_vis()
        rs = torch.empty((p.nint, p.nbl, p.nchan, p.npol), dtype=torch.complex64, device=dev)
        grid = torch.empty((nb, N, N), dtype=torch.complex64, device=dev)
        img = torch.empty((nb, N, N), dtype=torch.float32, device=dev)
        iws = plan.workspace(rf.RF_OP_IMAGE, nb)
        tags = torch.zeros((nb, 3), dtype=torch.int32, device=dev)
        cand = torch.empty((cap, 8), dtype=torch.int32, device=dev)
        ncand = torch.zeros(1, dtype=torch.int32, device=dev)
        L = rf.load_library()
        h = plan.handle
        sp = rf._stream(stream)
        P = rf._ptr
        plan.dedisperse(dvis, len(p.dms) - 1, out=dd)
        plan.resample(dd, 1, out=rs)
        plan.grid(rs[:nb], out=grid)
        plan.image(grid, out=img, ws=iws)
        reps = 20
        kernels["rf_dedisperse"] = event_time(lambda: L.rf_dedisperse(h, len(p.dms) - 1, P(dvis), P(dd), sp), reps, stream)
        kernels["rf_resample_w1"] = event_time(lambda: L.rf_resample(h, 1, P(dd), p.nint, P(rs), sp), reps, stream)
        kernels["rf_grid_64"] = event_time(lambda: L.rf_grid(h, P(rs), nb, P(grid), sp), reps, stream)
        kernels["rf_image_64"] = event_time(lambda: L.rf_image(h, P(grid), nb, P(img), P(iws), iws.numel(), sp), reps, stream)
        kernels["rf_search_64"] = event_time(lambda: L.rf_search(h, P(img), nb, P(tags), None, P(cand), cap, P(ncand), None, 0, sp), reps, stream)
        nw = len(p.widths)
        calls = {"rf_dedisperse": len(p.dms), "rf_resample_w1": len(p.dms) * nw,
                 "rf_grid_64": plan.n_images / nb, "rf_image_64": plan.n_images / nb,
                 "rf_search_64": plan.n_images / nb}
        share = {k: kernels[k] * calls[k] for k in kernels}
        log("entry-point seconds per step (event-timed x calls): " +
            ", ".join(f"{k}={v:.3f}" for k, v in share.items()))
        # rf_search launches exactly one kernel (k_search); its algorithmic
        # traffic is one read of each image: N^2 float32.
        dur = kernels["rf_search_64"]
        alg = nb * N * N * 4
        ach = alg / dur / 1e9
        roof = {"bound": "hbm", "kernel": "k_search", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_launch_us": round(dur * 1e6, 2), "alg_bytes_per_launch": alg}
        kernels = {k: round(v * 1e6, 2) for k, v in kernels.items()}

    out = {
        "metric": "images searched/sec",
        "value": round(img_s, 1),
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dtype == rf.RF_CF32 else "f32 (f16 storage)",
        "data": "synthetic",
        "config": {"workload": f"{p.name}: {p.nbl} baselines, {p.nint} x {p.tint_s * 1e3:g} ms, "
                               f"{p.nchan} chans {p.f_lo_ghz}-{p.f_hi_ghz} GHz, {p.npol} pols "
                               f"{args.storage}, {len(p.dms)} DMs 0-{p.dms[-1]:g}, widths {p.widths}, "
                               f"{p.npix}^2 images",
                   "images_per_step": plan.n_images, "path": "rf_search_segment"},
        "rtf": round(seg_s / step_s, 3),
        "pulses_recovered": f"{found}/{len(p.pulses)}",
        "candidates": n,
        "kernel_us": kernels,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

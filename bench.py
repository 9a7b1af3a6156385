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

# HBM bytes per dispatch of the fused search's kernels (survey workload,
# 1024^2 images, 16 image pairs per batch), from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of `bench.py --dms 2
# --profile-only`, each scaled by what the counter reads for a 1 GiB device
# copy (FETCH_SIZE reads 524,301 KiB for 1 GiB read: x2; WRITE_SIZE 1,048,576
# KiB for 1 GiB written: x1).  Valid only for the kernel sources with this
# digest (the device code of k_fused.hip, fft.h, rf_internal.h); null once
# they change.
FUSED_TRAFFIC = {"digest": "3f02c7c880b3bece", "fetch_scale": 2.0, "write_scale": 1.0,
                 "kib_per_dispatch": {"drs": (1439393.6, 2696128.1), "grid": (13128.5, 7362.9),
                                      "rows": (6346.9, 113502.1), "cols": (56770.0, 1610.1),
                                      "select": (2357.2, 0.0)}}


def fused_kernel_digest():
    """Digest of the fused kernels' device code: k_fused.hip up to its host
    side, fft.h and rf_internal.h, without comments and blank space (host
    scheduling and comment changes keep it)."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_1802_03084_amd", "csrc")
    h = hashlib.sha256()
    for f in ("k_fused.hip", "fft.h", "rf_internal.h"):
        text = open(os.path.join(csrc, f), "rb").read()
        if f == "k_fused.hip":
            cut = text.find(b"// ------------------------------------------------------------------ host side")
            assert cut > 0, "k_fused.hip: host side marker"
            text = text[:cut]
        text = re.sub(rb"//[^\n]*", b"", text)
        h.update(b" ".join(text.split()))
    return h.hexdigest()[:16]


def traffic_per_dispatch(kind):
    """Measured HBM bytes of one dispatch of `kind`, or None."""
    t = FUSED_TRAFFIC
    if t["digest"] is None or t["digest"] != fused_kernel_digest() or kind not in t["kib_per_dispatch"]:
        return None
    fetch, write = t["kib_per_dispatch"][kind]
    return 1024 * (fetch * t["fetch_scale"] + write * t["write_scale"])


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def serving_leg(speedup, nseg, nslots, storage, burst_nseg=0):
    """The serving workload: three subarrays (A 10 antennas 5 ms, B 19
    antennas 10 ms, C 27 antennas 5 ms; 10.24 s segments, 256 channels over
    1.272-1.528 GHz, 64 DMs, widths {1,2,4,8}, 512^2 images) streamed to an
    rf_server from pinned host memory.  Paced run: each subarray releases a
    segment every 10.24 / speedup s (phases offset by a third of a period);
    latency = candidates on the host - release.  Burst run: every segment
    released at once; sustained rate = data seconds / wall seconds."""
    import threading
    import numpy as np
    import torch
    import rfgen
    import paper_1802_03084_amd as rf

    dtype = rf.RF_CF16 if storage == "cf16" else rf.RF_CF32
    subs = []
    for name in "ABC":
        p = rfgen.serving(name)
        du, dv = p.cell()
        plan = rf.Plan(p.freq(), p.uvw(), p.tint_s, p.dms, p.widths, p.npix, du, dv, nint=p.nint,
                       npol=p.npol, vis_dtype=dtype, kdm=p.kdm, threshold=p.threshold)
        vis = p.make_vis()
        arr = rfgen.to_cf16(vis) if dtype == rf.RF_CF16 else np.ascontiguousarray(vis)
        host = torch.from_numpy(arr).pin_memory()
        del vis, arr
        subs.append((name, p, plan, host))
        log(f"serving subarray {name}: {p.nbl} baselines, {p.nint} x {p.tint_s * 1e3:g} ms, "
            f"{plan.n_images} images per segment")
    need = [rf.Server.request_bytes(pl, 4096) for _, _, pl, _ in subs]
    budget = 2 * sum(need)
    arena = torch.empty(budget, dtype=torch.uint8, device="cuda")
    srv = rf.Server(arena, nslots=nslots)
    seg_s = subs[0][1].nint * subs[0][1].tint_s

    def run(schedule):
        tickets, t0 = [], time.perf_counter()

        def submitter():
            for t, i in schedule:
                dt = t0 + t - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                tickets.append((i, srv.submit(subs[i][2], subs[i][3], cap=4096)))

        th = threading.Thread(target=submitter)
        th.start()
        out, k = [], 0
        while k < len(schedule):
            if k >= len(tickets):
                time.sleep(0.001)
                continue
            i, tk = tickets[k]
            rows, n, tm = srv.wait(tk)
            out.append((i, rows, n, tm))
            k += 1
            if k % 30 == 0:
                log(f"serving: {k}/{len(schedule)} segments done, last latency "
                    f"{tm['latency_s'] * 1e3:.0f} ms")
        th.join()
        return out, time.perf_counter() - t0

    for i in range(3):  # first use of each plan, outside the measurement
        srv.wait(srv.submit(subs[i][2], subs[i][3], cap=4096))
    period = seg_s / speedup
    paced = sorted((j * period + i * period / 3, i) for i in range(3) for j in range(nseg))
    res, wall_p = run(paced)
    lat = np.array([tm["latency_s"] for _, _, _, tm in res])
    found = 0
    for i, rows, n, _ in res:
        q = subs[i][1].pulses[0]
        keys = {(int(r["dm_idx"]), int(r["width_idx"]), int(r["t_int"]), int(r["x"]), int(r["y"])) for r in rows}
        found += (q.dm_idx, q.width_idx, q.t0, q.x, q.y) in keys
    burst = [(0.0, i) for j in range(burst_nseg or nseg) for i in range(3)]
    resb, wall_b = run(burst)

    def overlap(res):
        """Largest number of requests on the device at once (admitted, not
        yet done), from the server's own admission and completion times."""
        ev = sorted([(tm["started_s"], 1) for _, _, _, tm in res] +
                    [(tm["done_s"], -1) for _, _, _, tm in res], key=lambda e: (e[0], e[1]))
        cur = best = 0
        for _, d in ev:
            cur += d
            best = max(best, cur)
        return best
    srv.close()
    imgs = sum(subs[i][2].n_images for i, _, _, _ in resb)
    out = {
        "workload": "3 subarrays (10, 19, 27 antennas; 5/10/5 ms; 10.24 s segments), 256 chans "
                    "1.272-1.528 GHz, 64 DMs, widths [1,2,4,8], 512^2 images, "
                    f"{storage} storage, pinned host -> device per segment",
        "slots": nslots, "arena_bytes": budget,
        "paced": {"speedup_vs_real_time": speedup, "segments": len(res),
                  "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
                  "latency_p99_s": round(float(np.percentile(lat, 99)), 4),
                  "latency_max_s": round(float(lat.max()), 4),
                  "per_subarray_p99_s": {subs[i][0]: round(float(np.percentile(
                      [tm["latency_s"] for j, _, _, tm in res if j == i], 99)), 4) for i in range(3)},
                  "pulses_recovered": f"{found}/{len(res)}",
                  "max_requests_on_device": overlap(res),
                  "wall_s": round(wall_p, 1)},
        "burst": {"segments": len(resb), "wall_s": round(wall_b, 3), "images_per_s": round(imgs / wall_b, 1),
                  "rtf": round(len(resb) / 3 * seg_s / wall_b, 2),
                  "max_requests_on_device": overlap(resb)},
    }
    log(f"serving paced x{speedup}: p50 {out['paced']['latency_p50_s'] * 1e3:.0f} ms, "
        f"p99 {out['paced']['latency_p99_s'] * 1e3:.0f} ms over {len(res)} segments; burst "
        f"{out['burst']['images_per_s']:.0f} images/s, RTF {out['burst']['rtf']} (3 streams)")
    return out


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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


def copy_rate(torch, nbytes, reps=5):
    """Read + write GB/s of a plain device-to-device copy of nbytes."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    t1.synchronize()
    dt = t0.elapsed_time(t1) / reps * 1e-3
    del src, dst
    return 2 * nbytes / dt / 1e9


def large_leg(ndm, steps):
    """The large workload (351 baselines, 8192 x 1 ms, 1024 channels over
    2-4 GHz, widths 1..32, 2048^2 images) over ndm of its 400 DM trials spread
    evenly over the grid plus the five pulses' trials (every DM trial costs
    the same), generated on the device with the pulses,
    in CF16 and CF32 storage.  Reports images/s and the projected time and
    real-time factor of the full 400-trial segment."""
    import numpy as np
    import torch
    import rfgen
    import paper_1802_03084_amd as rf
    from paper_1802_03084_amd import mock
    p = rfgen.large()
    full_ndm = len(p.dms)
    keep = sorted(set(np.linspace(0, full_ndm - 1, ndm).round().astype(int).tolist())
                  | {q.dm_idx for q in p.pulses})
    mocks = p.mocks()
    pulses = [(keep.index(q.dm_idx), q.width_idx, q.t0, q.x, q.y) for q in p.pulses if q.dm_idx in keep]
    du, dv = p.cell()
    seg_s = p.nint * p.tint_s
    out = {"workload": f"large: {p.nbl} baselines, {p.nint} x {p.tint_s * 1e3:g} ms, {p.nchan} chans "
                       f"{p.f_lo_ghz}-{p.f_hi_ghz} GHz, widths {p.widths}, {p.npix}^2; {len(keep)} of "
                       f"{full_ndm} DM trials"}
    for name, dt in (("cf16", rf.RF_CF16), ("cf32", rf.RF_CF32)):
        plan = rf.Plan(p.freq(), p.uvw(), p.tint_s, p.dms[keep], p.widths, p.npix, du, dv,
                       nint=p.nint, npol=p.npol, vis_dtype=dt, kdm=p.kdm, threshold=p.threshold)
        t = time.perf_counter()
        vis = mock.synthesize(plan, p.seed, mocks)
        torch.cuda.synchronize()
        gen_s = time.perf_counter() - t
        ws = plan.workspace(rf.RF_OP_SEGMENT)
        rows, n, _ = plan.search_segment(vis, ws=ws)  # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            rows, n, _ = plan.search_segment(vis, ws=ws)
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t) / steps
        keys = {tuple(int(r[f]) for f in ("dm_idx", "width_idx", "t_int", "x", "y")) for r in rows}
        per_dm = dt_s / len(keep)
        out[name] = {"images_per_step": plan.n_images, "ms_per_step": round(dt_s * 1e3, 1),
                     "images_per_s": round(plan.n_images / dt_s, 1),
                     "ms_per_dm_trial": round(per_dm * 1e3, 2),
                     "full_segment_s": round(per_dm * full_ndm, 2),
                     "full_segment_rtf": round(seg_s / (per_dm * full_ndm), 3),
                     "pulses_recovered": f"{sum(k in keys for k in pulses)}/{len(pulses)}",
                     "generate_s": round(gen_s, 2)}
        log(f"large {name}: {plan.n_images / dt_s:.0f} images/s, {per_dm * 1e3:.1f} ms per DM trial, "
            f"full segment {per_dm * full_ndm:.1f} s (RTF {seg_s / (per_dm * full_ndm):.3f})")
        del vis, ws, plan
        torch.cuda.empty_cache()
    return out


def batching_leg(dms_per_segment):
    """The batching workload: 64 segments of uneven shape (nint 256-4096,
    128-512 channels, 512^2 to 2048^2 images, 64-254 DM trials each),
    FP16-stored visibilities generated on the device, all resident in HBM and
    searched as one batch (rf_batch_run).  Each segment keeps
    `dms_per_segment` of its DM trials spread over its grid plus the pulse's
    trial (every DM trial of a segment costs the same), so the run takes
    seconds; images/s is measured over the batch and the full workload's time
    projected from the per-segment DM fractions."""
    import numpy as np
    import torch
    import rfgen
    import paper_1802_03084_amd as rf
    from paper_1802_03084_amd import mock
    plans, segs, meta = [], [], []
    t = time.perf_counter()
    for s in range(rfgen.BATCHING_SEGMENTS):
        ndm = rfgen.batching_dm_count(s)
        keep = sorted(set(np.linspace(0, ndm - 1, dms_per_segment).round().astype(int).tolist())
                      | {ndm // 3})
        p = rfgen.batching(s, keep_dms=keep)
        du, dv = p.cell()
        plan = rf.Plan(p.freq(), p.uvw(), p.tint_s, p.dms, p.widths, p.npix, du, dv, nint=p.nint,
                       npol=p.npol, vis_dtype=rf.RF_CF16, kdm=p.kdm, threshold=p.threshold)
        segs.append(mock.synthesize(plan, p.seed, p.mocks()))
        plans.append(plan)
        meta.append((p, ndm, len(keep)))
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    seg_bytes = sum(v.numel() * v.element_size() for v in segs)
    b = rf.Batch(plans, segs, cap=65536)
    log(f"batching: {len(plans)} segments, {seg_bytes / 1e9:.1f} GB FP16 resident, workspace "
        f"{b.ws.numel() / 1e9:.1f} GB, generated in {gen_s:.1f} s")
    b.run()  # warm (first use of every shape)
    torch.cuda.synchronize()
    t = time.perf_counter()
    res = b.run()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    imgs = sum(pl.n_images for pl in plans)
    found = total = 0
    full_s = 0.0
    per_n = {}
    for (p, ndm, kept), pl, (rows, n, _) in zip(meta, plans, res):
        keys = {(int(r["dm_idx"]), int(r["width_idx"]), int(r["t_int"]), int(r["x"]), int(r["y"])) for r in rows}
        for q in p.pulses:
            total += 1
            found += (q.dm_idx, q.width_idx, q.t0, q.x, q.y) in keys
        per_n[p.npix] = per_n.get(p.npix, 0) + pl.n_images
    # projected full workload: each segment's share of the wall time scales
    # with its full DM count over the kept ones
    full_imgs = sum(p.n_images() // kept * ndm for (p, ndm, kept) in meta)
    out = {"workload": "batching: 64 segments, nint 256-4096, 128-512 chans, 351 baselines, 5 ms, "
                       "1-2 GHz, widths [1,2,4,8], 512^2-2048^2 images, FP16 storage, generated on "
                       f"the device; {dms_per_segment} spread DM trials per segment + the pulse's",
           "segments": len(plans), "images_per_run": imgs, "images_by_npix": per_n,
           "ms_per_run": round(wall * 1e3, 1), "images_per_s": round(imgs / wall, 1),
           "resident_GB": round(seg_bytes / 1e9, 2), "pulses_recovered": f"{found}/{total}",
           "full_workload_images": full_imgs,
           "full_workload_projected_s": round(full_imgs / (imgs / wall), 1),
           "path": "rf_batch_run (eager: graph capture is switched off)"}
    log(f"batching: {imgs / wall:.0f} images/s over {imgs} images in {wall:.2f} s, pulses {found}/{total}")
    del b, segs, plans
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--storage", choices=["cf32", "cf16"], default="cf32")
    ap.add_argument("--workload", choices=["survey", "tiny"], default="survey")
    ap.add_argument("--cpu-images", type=int, default=768)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain step-chain comparison")
    ap.add_argument("--dms", type=int, default=0,
                    help="search only the first K DM trials (short runs for hardware counters)")
    ap.add_argument("--profile-only", action="store_true",
                    help="run only the event-timed kernel pass (for counter collection)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--serving-speedup", type=float, default=8.0,
                    help="release rate of the paced serving run, in multiples of real time")
    ap.add_argument("--serving-segments", type=int, default=12, help="segments per subarray")
    ap.add_argument("--serving-slots", type=int, default=3)
    ap.add_argument("--serving-only", action="store_true", help="run only the serving legs")
    ap.add_argument("--serving-burst-segments", type=int, default=0,
                    help="segments per subarray of the burst run (default: as the paced run)")
    ap.add_argument("--no-periodic", action="store_true", help="skip the periodicity-search leg")
    ap.add_argument("--large", type=int, default=0, metavar="NDM",
                    help="only time the large workload (8192 x 1 ms, 1024 chans, 2048^2) over NDM "
                         "of its 400 DM trials, generated on the device, in both storages")
    ap.add_argument("--fp16-steps", type=int, default=3,
                    help="timed steps of the same search with FP16-stored visibilities (0: skip)")
    ap.add_argument("--large-dms-default", type=int, default=4, metavar="NDM",
                    help="the large-workload leg of the default run over NDM spread DM trials "
                         "plus the pulses' trials (0: skip)")
    ap.add_argument("--batching-dms", type=int, default=3, metavar="NDM",
                    help="the batching leg: NDM spread DM trials per segment plus the pulse's (0: skip)")
    ap.add_argument("--batching-only", action="store_true", help="run only the batching leg")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device (a plain copy kernel of known size, "
                         "to scale the HBM byte counters) and report its bandwidth")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: segments are independent, so N GPUs would each "
              "search their own segments with no exchange (run N=1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import rfgen

    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda")
        src.fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        dst.copy_(src)
        t0.record()
        reps = 5
        for _ in range(reps):
            dst.copy_(src)
        t1.record()
        t1.synchronize()
        dt = t0.elapsed_time(t1) / reps * 1e-3
        print(json.dumps({"copy_bytes": n, "read_plus_write_GBps": round(2 * n / dt / 1e9, 1),
                          "avg_us": round(dt * 1e6, 1)}), flush=True)
        return

    if args.large:
        print(json.dumps({"large": large_leg(args.large, args.steps)}), flush=True)
        return

    if args.batching_only:
        print(json.dumps({"batching": batching_leg(args.batching_dms or 3)}), flush=True)
        return

    if args.serving_only:
        print(json.dumps({"serving": serving_leg(args.serving_speedup, args.serving_segments,
                                                 args.serving_slots, "cf16",
                                                 args.serving_burst_segments)}), flush=True)
        return

    p = rfgen.survey() if args.workload == "survey" else rfgen.tiny()
    if args.dms > 0:
        p.dms = p.dms[: args.dms]
        p.pulses = [q for q in p.pulses if q.dm_idx < args.dms]
    t = time.perf_counter()
    vis = p.make_vis()
    log(f"generated {p.name} segment {vis.shape} {vis.nbytes / 1e9:.2f} GB in {time.perf_counter() - t:.1f}s")

    cpu = None
    if not args.no_cpu_baseline:
        # every core this process may run on, up to the 16 host cores that
        # go with one GPU on the machines this runs on
        avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        procs = max(1, min(16, avail))
        n, dt, _ = cpu_baseline(p, vis, args.cpu_images, procs)
        model = cpu_model()
        cpu = {"value": round(n / dt, 1), "unit": "images/s", "cores": procs, "kind": "oracle",
               "per_core": round(n / dt / procs, 2), "cpu": model, "cores_available": avail,
               "sample": f"{n} images of the {p.name} workload (4 DM trials spread over the grid x "
                         f"{len(p.widths)} widths x integrations spread over the segment), float64 numpy, "
                         f"{procs} processes ({avail} cores available), {dt:.1f} s wall"}
        log(f"cpu oracle: {n} images in {dt:.1f}s on {procs} processes ({model}) = {n / dt:.1f} img/s, "
            f"{n / dt / procs:.2f} per core")

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
    if args.profile_only:  # every launch in order on one stream: durations do not overlap
        times, _, n = plan.profile_segment(dvis, cap=cap, ws=ws)
        log("serial profile pass: " + ", ".join(f"{k}={v[0]:.1f} ms/{v[1]} ({1e3 * v[0] / v[1]:.2f} us)"
                                                 for k, v in times.items() if v[1]))
        return
    for w in range(args.warmup):
        t = time.perf_counter()
        rows, n, _ = plan.search_segment(dvis, cap=cap, ws=ws)
        log(f"warmup {w}: {time.perf_counter() - t:.2f}s, {n} candidates")

    # The timed steps: the fused search alone, in its own schedule (two lane
    # streams).  No events are recorded in them: an event on a launch (a
    # marker, or one attached to the dispatch) changes how the lanes overlap,
    # and with events on every launch a step takes about a fifth longer.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        rows, n, _ = plan.search_segment(dvis, cap=cap, ws=ws)
        log(f"step {k} done at {time.perf_counter() - t0:.2f}s, {n} candidates")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_s = wall / args.steps
    img_s = plan.n_images / step_s
    keys = {(int(r["dm_idx"]), int(r["width_idx"]), int(r["t_int"]), int(r["x"]), int(r["y"])) for r in rows}
    seg_s = p.nint * p.tint_s
    found = sum((q.dm_idx, q.width_idx, q.t0, q.x, q.y) in keys for q in p.pulses)
    log(f"{img_s:.0f} images/s, {step_s * 1e3:.1f} ms/step, RTF {seg_s / step_s:.2f}, "
        f"pulses recovered {found}/{len(p.pulses)}, candidates {n}")

    # The same search with FP16-stored visibilities (float32 arithmetic): the
    # precision form set against the plain float32 step chain below.
    fp16 = None
    if dtype == rf.RF_CF32 and args.fp16_steps > 0:
        dvis16 = torch.from_numpy(rfgen.to_cf16(vis)).to(dev)
        plan16 = rf.Plan(p.freq(), p.uvw(), p.tint_s, p.dms, p.widths, p.npix, du, dv, nint=p.nint,
                         npol=p.npol, vis_dtype=rf.RF_CF16, kdm=p.kdm, threshold=p.threshold)
        assert plan16.workspace_bytes(rf.RF_OP_SEGMENT) <= ws.numel()
        plan16.search_segment(dvis16, cap=cap, ws=ws)  # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.fp16_steps):
            rows16, n16, _ = plan16.search_segment(dvis16, cap=cap, ws=ws)
        torch.cuda.synchronize()
        t16 = (time.perf_counter() - t) / args.fp16_steps
        keys16 = {(int(r["dm_idx"]), int(r["width_idx"]), int(r["t_int"]), int(r["x"]), int(r["y"]))
                  for r in rows16}
        fp16 = {"path": "rf_search_segment (fused), cf16 storage, f32 arithmetic",
                "steps": args.fp16_steps, "ms_per_step": round(t16 * 1e3, 1),
                "images_per_s": round(plan16.n_images / t16, 1), "rtf": round(seg_s / t16, 3),
                "candidates": n16, "candidates_shared_with_cf32": len(keys16 & keys),
                "pulses_recovered": f"{sum((q.dm_idx, q.width_idx, q.t0, q.x, q.y) in keys16 for q in p.pulses)}"
                                    f"/{len(p.pulses)}"}
        log(f"fp16 storage: {plan16.n_images / t16:.0f} images/s, {t16 * 1e3:.1f} ms/step, "
            f"{n16} candidates ({len(keys16 & keys)} shared with cf32)")
        del dvis16, plan16

    N = p.npix
    nw = len(p.widths)
    n_rows = plan.info["n_rows"]
    pairs = len(p.dms) * sum((p.nint // w + 1) // 2 for w in p.widths)
    log2n = int(np.log2(N))
    in_bytes = dvis.numel() * dvis.element_size()
    vi_bytes = sum(p.nint // w for w in p.widths) * p.nbl * p.nchan * 8
    # algorithmic work per step: (bytes that must cross HBM, flops)
    algo = {
        "drs": (len(p.dms) * (in_bytes + vi_bytes), 0),
        "grid": (plan.n_images * (p.nbl * p.nchan + plan.info["n_cells"]) * 8, 0),
        "rows": (pairs * (2 * plan.info["n_cells"] + n_rows * N) * 8, pairs * n_rows * 5 * N * log2n),
        "cols": (pairs * n_rows * N * 8, pairs * N * 5 * N * log2n),
    }
    # Kernel durations: one more search with every launch in order on one
    # stream, an event pair attached to each dispatch (the launches do not
    # overlap, so the events change no overlap): each kernel's standalone rate,
    # the basis of its roofline.  Sharing the device, the two lanes' kernels
    # each take longer (the rocprofv3 trace of the timed steps shows it).
    times_s, _, _ = plan.profile_segment(dvis, cap=cap, ws=ws, concurrent=False)
    kernels = {k: {"launches_per_step": v[1], "avg_us": round(1e3 * v[0] / v[1], 2)}
               for k, v in times_s.items() if v[1]}
    log("fused kernels (event-timed, serial): " +
        ", ".join(f"{k}={v['avg_us']:.2f} us x{v['launches_per_step']}" for k, v in kernels.items()))
    dom = max((k for k in algo if k in kernels), key=lambda k: times_s[k][0])
    per_step = {k: times_s[k][1] for k in times_s if times_s[k][1]}
    bytes_step, flops_step = algo[dom]
    launches = per_step[dom]
    avg_s = kernels[dom]["avg_us"] * 1e-6
    b_launch, f_launch = bytes_step / launches, flops_step / launches
    gbs = b_launch / avg_s / 1e9
    tfs = f_launch / avg_s / 1e12
    # The transforms' algorithmic work is their flops (5 N log2 N per length-N
    # complex transform; nothing is counted for the row-transformed batch they
    # hand each other through memory, an intermediate of this design), done by
    # the fp32 vector units: their roofline is the fp32 vector peak.  The
    # passes over the segment (dedispersion, gridding) do no flops: theirs is
    # the HBM peak.
    if f_launch:
        roof = {"bound": "alu", "kernel": dom, "achieved": round(tfs, 2), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(tfs / FP32_PEAK_TFLOPS, 4), "traffic": None}
    else:
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None}
    roof.update({"avg_launch_us": round(avg_s * 1e6, 2), "alg_flops_per_launch": f_launch,
                 "alg_bytes_per_launch": b_launch, "launches_per_step": launches,
                 "timing": "HIP start/stop events attached to each dispatch (hipExtLaunchKernel) "
                           "on the launch's stream, one search with the launches in order on one "
                           "stream (the kernel alone on the device)"})
    if N == 1024 and traffic_per_dispatch(dom) is not None:
        roof["traffic"] = round(traffic_per_dispatch(dom))
        roof["traffic_unit"] = ("B per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE): for the "
                                "transforms, the row-transformed batch passed through memory, an "
                                "intermediate the algorithmic figure does not count")
    # the whole step's algorithmic HBM bytes (the segment read once per DM
    # trial) against the HBM bytes its kernels move (counters)
    roof["step_alg_bytes"] = len(p.dms) * in_bytes
    if N == 1024 and all(traffic_per_dispatch(k) is not None for k in per_step):
        moved = sum(traffic_per_dispatch(k) * per_step[k] for k in per_step)
        roof["step_traffic_bytes"] = round(moved)
        roof["step_traffic_over_alg"] = round(moved / roof["step_alg_bytes"], 2)
    for k in algo:
        if k in kernels and k in per_step:
            by, fl = algo[k]
            sec = kernels[k]["avg_us"] * 1e-6 * per_step[k]  # kernel time per step
            kernels[k]["achieved"] = f"{by / sec / 1e9:.0f} GB/s" + (
                f", {fl / sec / 1e12:.2f} TFLOP/s" if fl else "")

    # per-stage HBM rates against the published peak and a measured plain
    # device copy (read + write of 1 GiB)
    copy_gbs = copy_rate(torch, 1 << 30)
    stages = {}
    # the plain gridding step (rf_grid: Stokes I of 64 resampled integrations
    # onto dense grids), event-timed on its stream: bytes = samples read +
    # dense grids written
    if dtype == rf.RF_CF32:
        x64 = dvis[:64].contiguous()
        g64 = torch.empty((64, N, N), dtype=torch.complex64, device=dev)
        plan.grid(x64, out=g64)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(5):
            plan.grid(x64, out=g64)
        ev1.record()
        ev1.synchronize()
        sec = ev0.elapsed_time(ev1) / 5 * 1e-3
        by = x64.numel() * x64.element_size() + g64.numel() * g64.element_size()
        r = by / sec / 1e9
        stages["grid_step"] = {"path": f"rf_grid, 64 integrations onto dense {N}^2 grids",
                               "GBps": round(r, 1), "frac_of_peak": round(r / HBM_PEAK_GBS, 4),
                               "frac_of_copy": round(r / copy_gbs, 4), "us": round(sec * 1e6, 1)}
        del x64, g64
    for k in ("drs", "grid"):
        if k in kernels:
            by = algo[k][0]
            for mode, sec in (("serial", times_s[k][0] * 1e-3 if times_s[k][1] else None),):
                if sec:
                    r = by / sec / 1e9
                    stages.setdefault(k, {})[mode] = {
                        "GBps": round(r, 1), "frac_of_peak": round(r / HBM_PEAK_GBS, 4),
                        "frac_of_copy": round(r / copy_gbs, 4)}
    log(f"copy {copy_gbs:.0f} GB/s; stages: " + ", ".join(
        f"{k} {(v['serial'] if 'serial' in v else v)['GBps']:.0f} GB/s "
        f"({100 * (v['serial'] if 'serial' in v else v)['frac_of_peak']:.0f}% of peak)"
        for k, v in stages.items()))

    plain = None
    if not args.no_plain:
        wsp = plan.workspace(rf.RF_OP_SEGMENT_STEPS)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rows_p, n_p, _ = plan.search_segment(dvis, cap=cap, ws=wsp, steps=True)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        keys_p = {(int(r["dm_idx"]), int(r["width_idx"]), int(r["t_int"]), int(r["x"]), int(r["y"])) for r in rows_p}
        plain = {"path": "rf_search_segment_steps (plain fp32 step chain)", "ms_per_step": round(tp * 1e3, 1),
                 "images_per_s": round(plan.n_images / tp, 1), "rtf": round(seg_s / tp, 3),
                 "same_candidates": keys_p == keys}
        log(f"plain step chain: {tp:.2f}s/step, {plan.n_images / tp:.0f} images/s, same candidates {keys_p == keys}")
        del wsp
        if fp16:
            fp16["speedup_vs_plain_fp32"] = round(tp / (fp16["ms_per_step"] * 1e-3), 2)

    periodic = None
    if not args.no_periodic and (p.nint & (p.nint - 1)) == 0:
        del ws
        torch.cuda.empty_cache()
        wsp = torch.empty(plan.periodic_workspace_bytes(), dtype=torch.uint8, device=dev)
        plan.search_periodic(dvis, cap=cap, ws=wsp)  # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        rows_q, n_q, _ = plan.search_periodic(dvis, cap=cap, ws=wsp)
        torch.cuda.synchronize()
        tq = time.perf_counter() - t
        nimg = len(p.dms) * (p.nint // 2)
        periodic = {"path": "rf_search_periodic (time FFT per DM, one complex image per fluctuation "
                            "frequency 1..T/2, amplitude statistics)",
                    "images_per_step": nimg, "ms_per_step": round(tq * 1e3, 1),
                    "images_per_s": round(nimg / tq, 1), "rtf": round(seg_s / tq, 3),
                    "candidates": n_q}
        log(f"periodicity search: {tq:.2f}s/step, {nimg / tq:.0f} complex images/s, RTF {seg_s / tq:.2f}, "
            f"{n_q} candidates")
        del wsp
        ws = None

    serving = None
    if not args.no_serving:
        del ws, dvis
        torch.cuda.empty_cache()
        serving = serving_leg(args.serving_speedup, args.serving_segments, args.serving_slots, "cf16")

    batching = None
    if args.batching_dms > 0 and not args.dms:
        torch.cuda.empty_cache()
        batching = batching_leg(args.batching_dms)

    large = None
    if args.large_dms_default > 0 and not args.dms:
        torch.cuda.empty_cache()
        large = large_leg(args.large_dms_default, 1)

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
                   "images_per_step": plan.n_images, "path": "rf_search_segment (fused)"},
        "rtf": round(seg_s / step_s, 3),
        "plain_fp32_path": plain,
        "speedup_vs_plain": round(plain["ms_per_step"] / (step_s * 1e3), 2) if plain else None,
        "pulses_recovered": f"{found}/{len(p.pulses)}",
        "candidates": n,
        "kernels": kernels,
        "roofline": roof,
        "hbm_stages": {"copy_GBps": round(copy_gbs, 1), "peak_GBps": HBM_PEAK_GBS, **stages},
        "cpu_baseline": cpu,
        "serving": serving,
        "periodic": periodic,
        "fp16_storage": fp16,
        "batching": batching,
        "large": large,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

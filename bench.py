#!/usr/bin/env python3
"""Throughput of the SSLIC hot path on one MI355X.

One step is one whole ``sslic_run`` (seeding, every iteration of assignment +
update + residual test, and connectivity when the workload asks for it) over
a synthetic image already resident in HBM.  The default workload is the
FIB-SEM-like 3D volume: 1024^3 uint16, S=8, m=20, 10 iterations +
connectivity.  Prints one JSON line:

  value          Mvoxel*iter/s = voxels * iterations * steps / timed seconds
  roofline       the dominant kernel, the sweep (assignment and the map step
                 of the update in one pass), against the 8 TB/s HBM peak: the
                 algorithmic bytes of the two steps per voxel (assignment
                 reads the image and writes the label, the update reads image
                 and label: 2 (C b + 4) bytes) times the voxels of one launch,
                 over its mean launch time (HIP events on the launch stream
                 over the timed region); ``traffic`` comes from committed
                 rocprofv3 FETCH_SIZE/WRITE_SIZE counters when they were taken
                 on the current kernel source, else null.  The vector-ALU view
                 (algorithmic FP32 flops against the FP32 peak without packed
                 FP32) is reported beside it.
  cpu_baseline   the FP64 oracle on the host cores: one thread per crop of
                 the same image, all threads at once (and one thread alone)

Other workloads (--workload): slide-16k (16384^2 RGB uint8, no
connectivity); rgb-256 (256^2 RGB with connectivity: also the latency of one
run replayed from a captured HIP graph, median of --latency-reps replays);
persist-<workload> (the same run with the distance image kept across
iterations, whose dominant kernel is the kept-distance assignment);
batch-512 (the batched form against the same images one at a time); served
(the serving loop, p50/p99 at two offered loads and closed-loop throughput);
contours-<workload> (the contour mask over the image and the labels of one
run); lab-16k (8-bit RGB to CIE-Lab over the 16384^2 image).  The last two are
HBM-bound and report their roofline against 8 TB/s.

--image-cache PATH keeps the generated image in a .npy file: the first run
writes it, later runs load it instead of generating (so a profiled run
dispatches none of the generator's kernels); --gen-only stops after that.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak with packed FP32 disabled (the library compiles every
# kernel): 256 CUs x 64 lanes x 2 flops per FMA x 2.4 GHz = 78.6 TFLOP/s (the
# published 157.3 counts packed FP32 dual issue)
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
BYTES = {"u8": 1, "u16": 2, "f32": 4}


def load_profile(kind: str, kernel: str, workload: str):
    """profiles/<kind>_<kernel>_<workload>.json, if its counters were taken on
    the current code of that kernel, else None."""
    path = os.path.join(ROOT, "profiles", f"{kind}_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    from paper_1806_08741_amd.profsum import kernel_source_hash
    if rec.get("source_hash") != kernel_source_hash(kernel):
        return None
    return rec


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the traffic record (see load_profile)."""
    rec = load_profile("traffic", kernel, workload)
    return None if rec is None else rec.get("bytes_per_launch")


def copy_rate_gbs(mib: int = 1024, reps: int = 10) -> float:
    """Device-to-device copy rate (bytes read + written per second), the
    achievable line beside the 8 TB/s peak."""
    import torch
    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del a, b
    return 2 * (mib << 20) * reps / dt / 1e9


def host_threads() -> int:
    """Host cores the oracle may use: the process's CPU affinity, at most 16
    (a one-GPU share of the GPU host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def run_oracle_jobs(jobs, threads):
    """Run oracle jobs (callables) on ``threads`` host threads at once (the
    oracle's C code runs outside the GIL); returns the wall seconds."""
    import concurrent.futures as cf
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda f: f(), jobs))
    return time.perf_counter() - t0


def cpu_baseline(img_gpu, w, crop, persist=False):
    """The oracle as it stands on the leading crops (side ``crop`` on every
    axis, one per thread, disjoint, along the slowest axes) of the same image:
    first one crop on one thread, then one crop per host thread, all at once.
    Returns the record of the all-threads run with the one-thread rate beside
    it."""
    import oracle
    nd = len(w.dims)
    c = [min(crop, d) for d in w.dims]
    threads = host_threads()
    # crop origins: a grid over the image, axis 0 fastest
    per_axis = [max(1, d // cc) for d, cc in zip(w.dims, c)]
    origins = []
    for lin in range(int(np.prod(per_axis))):
        o, r = [], lin
        for i in range(nd):
            o.append((r % per_axis[i]) * c[i])
            r //= per_axis[i]
        origins.append(o)
    origins = origins[:threads]
    threads = len(origins)
    subs = []
    for o in origins:
        sl = tuple(slice(o[i], o[i] + c[i]) for i in reversed(range(nd)))
        subs.append(img_gpu[sl].contiguous().cpu().numpy())
    vox = int(np.prod(c))

    def job(sub):
        def f():
            r = oracle.run(sub, nd, w.S, w.m, w.iterations, connectivity=w.connectivity,
                           persist_distance=persist)
            assert r["iterations"] == w.iterations
        return f

    one = run_oracle_jobs([job(subs[0])], 1)
    # small images: every thread runs its crop `rep` times, about 10 s in all
    rep = max(1, int(10.0 / max(one, 1e-3)))
    jobs = [job(sb) for sb in subs] * rep
    threads = host_threads() if len(subs) < host_threads() and rep > 1 else threads
    allt = run_oracle_jobs(jobs, threads)
    side = "x".join(str(v) for v in c)
    what = (f"{len(subs)} disjoint {side} crop(s), {len(jobs)} runs on {threads} threads, "
            f"{w.iterations} iterations" + (" + connectivity" if w.connectivity else ""))
    return {"value": round(vox * len(jobs) * w.iterations / allt / 1e6, 3),
            "unit": "Mvoxel*iter/s", "cores": threads, "kind": "oracle", "sample": what,
            "seconds": round(allt, 2),
            "one_thread": {"value": round(vox * w.iterations / one / 1e6, 3), "cores": 1,
                           "seconds": round(one, 2)},
            "cpu_model": cpu_model()}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def workload_image(w, dev, cache: str = ""):
    """The image of workload ``w`` on ``dev``: loaded from ``cache`` (.npy)
    when that file exists, else generated on the GPU (and written there)."""
    import torch
    from paper_1806_08741_amd import synth
    t0 = time.perf_counter()
    if cache and os.path.exists(cache):
        arr = np.load(cache, mmap_mode="r")
        shape = tuple(reversed(w.dims)) + (w.channels,)
        if arr.shape != shape:
            raise SystemExit(f"{cache} holds shape {arr.shape}, not {shape}")
        img = torch.empty(shape, dtype=w.dtype, device=dev)
        flat = img.view(-1, w.channels)
        rows = arr.reshape(-1, w.channels)
        step = 1 << 26
        for a in range(0, rows.shape[0], step):
            part = np.ascontiguousarray(rows[a:a + step])
            if w.dtype == torch.uint16:
                part = part.view(np.int16)
                flat[a:a + step].view(torch.int16).copy_(torch.from_numpy(part))
            else:
                flat[a:a + step].copy_(torch.from_numpy(part))
        torch.cuda.synchronize()
        print(f"[bench] loaded {w.name} {w.dims} from {cache} in "
              f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
        return img
    print(f"[bench] generating {w.name} {w.dims} on the GPU", file=sys.stderr, flush=True)
    img = synth.workload_image(w.name, dev)
    torch.cuda.synchronize()
    print(f"[bench] generated in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    if cache:
        out = np.lib.format.open_memmap(cache, mode="w+", dtype=np.dtype(
            {torch.uint8: np.uint8, torch.uint16: np.uint16, torch.float32: np.float32}[w.dtype]),
            shape=tuple(img.shape))
        flat = out.reshape(-1)
        src = img.view(-1)
        step = 1 << 28
        for a in range(0, src.numel(), step):
            chunk = src[a:a + step]
            if w.dtype == torch.uint16:
                flat[a:a + step] = chunk.view(torch.int16).cpu().numpy().view(np.uint16)
            else:
                flat[a:a + step] = chunk.cpu().numpy()
        out.flush()
        del out
        print(f"[bench] wrote {cache}", file=sys.stderr, flush=True)
    return img


def graph_latency(ctx, img, w, out, reps: int) -> dict:
    """Latency of one whole run (seeding, iterations, connectivity) replayed
    from a captured HIP graph: each replay timed alone with events on the
    replay stream; median and p99 over ``reps`` replays, in microseconds."""
    import torch
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    run = lambda: ctx.run(img, w.S, w.m, w.iterations, connectivity=w.connectivity, out=out,
                          sync=False)
    with torch.cuda.stream(s):
        run()  # sizes the workspace outside the capture
    torch.cuda.synchronize()
    ref = out["labels"].clone()
    with torch.cuda.graph(g, stream=s):
        run()
    torch.cuda.synchronize()
    ts = []
    with torch.cuda.stream(s):
        for _ in range(5):
            g.replay()
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            g.replay()
            b.record(s)
            b.synchronize()
            ts.append(a.elapsed_time(b) * 1e3)
    torch.cuda.synchronize()
    assert torch.equal(out["labels"], ref), "a graph replay changed the result"
    ts = np.array(ts)
    print(f"[bench] graph replay of one run: median {np.median(ts):.1f} us, "
          f"p99 {np.percentile(ts, 99):.1f} us over {reps}", file=sys.stderr, flush=True)
    return {"us_median": round(float(np.median(ts)), 2),
            "us_p99": round(float(np.percentile(ts, 99)), 2), "replays": reps,
            "Mvoxel_iter_s_at_median": round(w.voxels * w.iterations / float(np.median(ts)), 1),
            "how": "whole sslic_run captured in a HIP graph, each replay timed alone with "
                   "events on its stream"}


def bench_batch(args, n_images):
    """The batched workload: n images of the batch recipe (half 2D RGB uint8,
    half 3D float32, uneven sizes, per-image S and m, 10 iterations), timed as
    whole sslic_run_batch calls (graph replays after the first) against the
    same images run one at a time with sslic_run on one stream."""
    import numpy as np
    import torch
    from paper_1806_08741_amd import sslic, synth

    specs = synth.batch_specs(n_images)
    print(f"[bench] generating {n_images} images", file=sys.stderr, flush=True)
    items = [dict(image=synth.batch_image(sp, "cuda"), S=sp.S, m=sp.m, iterations=sp.iterations)
             for sp in specs]
    torch.cuda.synchronize()
    vox = sum(sp.voxels for sp in specs)
    work = sum(sp.voxels * sp.iterations for sp in specs)
    ctx = sslic.Context(0)
    outs = ctx.run_batch(items, graph=True)  # autotune + capture
    items_o = [dict(it, labels=o["labels"], centres=o["centres"], counts=o["counts"],
                    iters=o["iters"]) for it, o in zip(items, outs)]
    for _ in range(args.warmup):
        ctx.run_batch(items_o, graph=True, sync=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.run_batch(items_o, graph=True, sync=False)
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t0) / args.steps
    print(f"[bench] batched: {dt_b * 1e3:.3f} ms per batch", file=sys.stderr, flush=True)

    solo = [dict(labels=torch.empty_like(o["labels"]), centres=torch.empty_like(o["centres"]),
                 counts=torch.empty_like(o["counts"])) for o in outs]

    def one_at_a_time():
        for it, so in zip(items, solo):
            ctx.run(it["image"], it["S"], it["m"], it["iterations"], connectivity=False, out=so,
                    sync=False)

    for _ in range(args.warmup):
        one_at_a_time()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_at_a_time()
    torch.cuda.synchronize()
    dt_s = (time.perf_counter() - t0) / args.steps
    print(f"[bench] one at a time: {dt_s * 1e3:.3f} ms per batch", file=sys.stderr, flush=True)
    # the dominant kernel: the batched sweep, timed with events on direct
    # (not graph) launches of the same batch
    import ctypes
    L = sslic.lib()
    outs_t = [dict(labels=torch.empty_like(o["labels"]), centres=torch.empty_like(o["centres"]),
                   counts=torch.empty_like(o["counts"])) for o in outs]
    items_t = [dict(it, **ot) for it, ot in zip(items, outs_t)]
    ctx.run_batch(items_t, graph=False, sync=False)
    torch.cuda.synchronize()
    sslic._check(L.sslic_profile_enable(ctx._h, 1))
    reps = max(1, min(args.steps, 5))
    for _ in range(reps):
        ctx.run_batch(items_t, graph=False, sync=False)
    torch.cuda.synchronize()
    kern = {}
    for k in ("sweep_batch", "finalize_batch"):
        ms, nl = ctypes.c_double(0), ctypes.c_int64(0)
        sslic._check(L.sslic_profile_read(ctx._h, k.encode(), ctypes.byref(ms), ctypes.byref(nl)))
        kern[k] = {"ms_per_batch": ms.value / reps, "launches_per_batch": nl.value // reps}
    sslic._check(L.sslic_profile_enable(ctx._h, 0))
    bts = {torch.uint8: 1, torch.uint16: 2, torch.float32: 4}
    # algorithmic bytes of every image's assignment + update, all iterations
    alg = sum(sp.voxels * sp.iterations * 2 * (sp.channels * bts[sp.dtype] + 4) for sp in specs)
    sweep_s = kern["sweep_batch"]["ms_per_batch"] * 1e-3
    print(f"[bench] batched sweep {kern['sweep_batch']['ms_per_batch']:.3f} ms per batch "
          f"({kern['sweep_batch']['launches_per_batch']} launches)", file=sys.stderr, flush=True)
    # equal results (integer images bit-identical, float images to 1e-4 of labels)
    worst = 0.0
    for sp, o, so in zip(specs, outs, solo):
        d = float((o["labels"] != so["labels"]).float().mean().item())
        if sp.dtype != torch.float32:
            assert d == 0.0 and torch.equal(o["centres"], so["centres"])
        worst = max(worst, d)
    assert worst <= 1e-4, worst
    rec = {
        "metric": "SLIC Mvoxel*iter/s (whole batch per step; inputs resident in HBM)",
        "value": round(work / dt_b / 1e6, 1),
        "unit": "Mvoxel*iter/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt_b * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch-{n_images}", "images": n_images, "voxels": vox,
                   "recipe": "half 2D RGB u8 sides log-uniform [96,1024], half 3D 1-channel f32 "
                             "sides log-uniform [32,160]; S in {8,12,16}, m in {10,20}; "
                             "Voronoi regions, noise sigma 8; 10 iterations, no connectivity"},
        "one_at_a_time": {"value": round(work / dt_s / 1e6, 1), "ms_per_step": round(dt_s * 1e3, 4),
                          "speedup_of_batch": round(dt_s / dt_b, 3)},
        "label_disagreement_max": worst,
        "roofline": {"bound": "hbm", "kernel": "sweep_batch (all launches of one batch)",
                     "achieved": round(alg / sweep_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(alg / sweep_s / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None,
                     "algorithmic_bytes_per_batch": alg,
                     "algorithmic_bytes_per_voxel_iter": round(alg / work, 3),
                     "sweep_ms_per_batch": round(kern["sweep_batch"]["ms_per_batch"], 4),
                     "finalize_ms_per_batch": round(kern["finalize_batch"]["ms_per_batch"], 4),
                     "whole_batch_hbm_frac": round(alg / dt_b / 1e9 / HBM_PEAK_GBS, 4)},
    }
    if args.cpu_crop != 0:
        rec["cpu_baseline"] = oracle_images_baseline(
            [(it["image"], it["S"], it["m"], it["iterations"]) for it in items[:128]],
            "the first 128 images of the batch, one image per thread at a time, 10 iterations")
    print(json.dumps(rec), flush=True)


def oracle_images_baseline(jobs, what):
    """The oracle on a list of whole images (image, S, m, iterations), no
    connectivity, spread over the host threads (one image per thread at a
    time): aggregate Mvoxel*iter/s."""
    import oracle
    host = [(im.cpu().numpy(), S, m, T) for im, S, m, T in jobs]
    work = sum(int(np.prod(h[0].shape[:-1])) * h[3] for h in host)

    def job(h):
        def f():
            oracle.run(h[0], h[0].ndim - 1, h[1], h[2], h[3], connectivity=False)
        return f

    threads = host_threads()
    sec = run_oracle_jobs([job(h) for h in host], threads)
    return {"value": round(work / sec / 1e6, 3), "unit": "Mvoxel*iter/s", "cores": threads,
            "kind": "oracle", "sample": what, "seconds": round(sec, 2), "cpu_model": cpu_model()}


def bench_served(args):
    """The served stream: Poisson arrivals at 50 and 200 requests/s of the
    70/20/10 mix (2D RGB u8 sides 256-8192, 3D u16 sides 64-512, 3D 4-channel
    f32 up to 512x512x256), each request 10 iterations, no connectivity.
    Continuous batching (serve.Server, 64 GiB admission budget, 3 lanes)
    against one request at a time (serve.fifo) on the same trace: p50/p99
    latency from arrival to completion; then both closed-loop (every request
    queued at time 0) for aggregate throughput."""
    import numpy as np
    import torch
    from paper_1806_08741_amd import serve, synth

    n = args.requests
    trace = synth.request_trace(200.0, n, scale=args.serve_scale)
    print(f"[bench] generating {n} requests", file=sys.stderr, flush=True)
    reqs = serve.make_requests(trace, synth.request_image, "cuda")
    torch.cuda.synchronize()
    base = [r.arrival for r in reqs]
    work = sum(r.voxels * r.iterations for r in reqs)
    srv = serve.Server(hbm_budget=64 << 30, lanes=3, max_batch=64)
    srv.warm(reqs)
    out = {}

    def reset(rate):
        for r, t in zip(reqs, base):
            r.arrival = t * 200.0 / rate if rate else 0.0
            r.start = r.done = float("nan")
            r.out = {}

    for rate in (50.0, 200.0):
        reset(rate)
        s_srv = srv.serve(reqs)
        reset(rate)
        s_fifo = serve.fifo(reqs)
        out[f"{int(rate)}/s"] = {"served": s_srv.as_dict(), "one_at_a_time": s_fifo.as_dict()}
        print(f"[bench] {int(rate)}/s served p50 {s_srv.p50:.2f} p99 {s_srv.p99:.2f} ms; "
              f"one-at-a-time p50 {s_fifo.p50:.2f} p99 {s_fifo.p99:.2f} ms",
              file=sys.stderr, flush=True)
    reset(0)
    c_srv = srv.serve(reqs, closed_loop=True)
    reset(0)
    c_fifo = serve.fifo(reqs, closed_loop=True)
    reset(0)
    print(f"[bench] closed loop: served {c_srv.mvoxel_iter_s:.0f}, one-at-a-time "
          f"{c_fifo.mvoxel_iter_s:.0f} Mvoxel*iter/s", file=sys.stderr, flush=True)
    rec = {
        "metric": "SLIC Mvoxel*iter/s served closed-loop; p50/p99 ms at 50 and 200 requests/s",
        "value": round(c_srv.mvoxel_iter_s, 1),
        "unit": "Mvoxel*iter/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(c_srv.wall_s * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "served", "requests": n, "voxel_iters": work,
                   "scale": args.serve_scale,
                   "recipe": "Poisson arrivals; 70% 2D RGB u8 sides log-uniform [256,8192], "
                             "20% 3D u16 sides [64,512], 10% 3D 4-channel f32 x,y [64,512] z "
                             "[32,256]; S in {8,16}, m=10, 10 iterations, no connectivity; "
                             "64 GiB admission budget, 3 lanes, batches of up to 64"},
        "open_loop": out,
        "closed_loop": {"served": c_srv.as_dict(), "one_at_a_time": c_fifo.as_dict(),
                        "speedup": round(c_srv.mvoxel_iter_s / c_fifo.mvoxel_iter_s, 3)},
        "peak_admitted_bytes": srv.peak_used, "peak_requests_on_gpu": srv.peak_running,
    }
    bts = {torch.uint8: 1, torch.uint16: 2, torch.float32: 4}
    alg = sum(r.voxels * r.iterations * 2 * (int(r.image.shape[-1]) * bts[r.image.dtype] + 4)
              for r in reqs)
    gbs = alg / c_srv.wall_s / 1e9
    rec["roofline"] = {"bound": "hbm", "kernel": "every launch of the closed-loop served run "
                       "(wall clock, host scheduling included)",
                       "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                       "algorithmic_bytes": alg,
                       "algorithmic_bytes_per_voxel_iter": round(alg / work, 3)}
    if args.cpu_crop != 0:
        sample, tot = [], 0
        for r in reqs:
            if tot >= 2e9:
                break
            sample.append((r.image, r.S, r.m, r.iterations))
            tot += r.voxels * r.iterations
        rec["cpu_baseline"] = oracle_images_baseline(
            sample, f"the first {len(sample)} requests of the trace, closed loop, one request "
                    "per thread at a time")
    print(json.dumps(rec), flush=True)


def bench_contours(args, base: str):
    """The contour mask (sslic_mask_contours) over a whole image of workload
    ``base`` (slide-16k or fibsem-1k), on the labels of one run of it: the
    image and labels are read once, the masked image written once."""
    import torch
    from paper_1806_08741_amd import sslic, synth

    w = synth.WORKLOADS[base]
    print(f"[bench] generating {w.name} {w.dims} on the GPU", file=sys.stderr, flush=True)
    img = synth.workload_image(w.name, "cuda")
    ctx = sslic.Context(0)
    lab = ctx.run(img, w.S, w.m, w.iterations, connectivity=w.connectivity)["labels"]
    out = torch.empty_like(img)
    for _ in range(args.warmup):
        ctx.mask_contours(img, lab, out=out)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        ctx.mask_contours(img, lab, out=out)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    dt_name = {torch.uint8: "u8", torch.uint16: "u16", torch.float32: "f32"}[w.dtype]
    N = w.voxels
    per_vox = 4 + 2 * w.channels * BYTES[dt_name]
    gbs = N * per_vox / (ms * 1e-3) / 1e9
    print(f"[bench] mask_contours {ms:.4f} ms, {gbs:.0f} GB/s", file=sys.stderr, flush=True)
    rec = {
        "metric": "contour mask Gvoxel/s (whole image per step; inputs resident in HBM)",
        "value": round(N / (ms * 1e-3) / 1e9, 2), "unit": "Gvoxel/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dt_name, "data": "synthetic",
        "config": {"workload": f"contours-{base}", "dims": list(w.dims), "channels": w.channels,
                   "image_dtype": dt_name, "labels": f"one {w.iterations}-iteration run"},
        "roofline": {"bound": "hbm", "kernel": "mask_contours", "achieved": round(gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic("contours", f"contours-{base}"),
                     "algorithmic_bytes_per_launch": N * per_vox,
                     "hbm_achievable_copy": round(copy_rate_gbs(), 1)},
    }
    # the oracle, one thread, on the leading crop of image and labels
    import oracle
    nd = len(w.dims)
    side = 16384 if nd == 2 else 512
    sl = tuple(slice(0, min(side, d)) for d in reversed(w.dims))
    sub = img[sl].contiguous().cpu().numpy()
    sub_lab = lab.view(*reversed(w.dims))[sl].contiguous().cpu().numpy()
    t0 = time.perf_counter()
    oracle.mask_contours(sub, nd, sub_lab)
    sec = time.perf_counter() - t0
    vox = int(np.prod(sub_lab.shape))
    rec["cpu_baseline"] = {"value": round(vox / sec / 1e9, 4), "unit": "Gvoxel/s", "cores": 1,
                           "kind": "oracle", "seconds": round(sec, 2),
                           "sample": "leading " + "x".join(str(min(side, d)) for d in w.dims) + " crop"}
    print(json.dumps(rec), flush=True)


def bench_lab(args):
    """RGB to CIE-Lab (sslic_rgb_to_lab) over the 16384x16384 slide-like RGB
    image: 3 bytes read and 12 written per pixel."""
    import torch
    from paper_1806_08741_amd import sslic, synth

    w = synth.WORKLOADS["slide-16k"]
    print(f"[bench] generating {w.name} {w.dims} on the GPU", file=sys.stderr, flush=True)
    img = synth.workload_image(w.name, "cuda")
    ctx = sslic.Context(0)
    out = torch.empty(img.shape, dtype=torch.float32, device=img.device)
    for _ in range(args.warmup):
        ctx.rgb_to_lab(img, out=out)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        ctx.rgb_to_lab(img, out=out)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    N = w.voxels
    gbs = N * 15 / (ms * 1e-3) / 1e9
    print(f"[bench] rgb_to_lab {ms:.4f} ms, {gbs:.0f} GB/s", file=sys.stderr, flush=True)
    rec = {
        "metric": "RGB to CIE-Lab Gpixel/s (whole image per step; inputs resident in HBM)",
        "value": round(N / (ms * 1e-3) / 1e9, 2), "unit": "Gpixel/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "lab-16k", "dims": list(w.dims), "input": "u8 RGB", "output": "f32 Lab"},
        "roofline": {"bound": "hbm", "kernel": "rgb_to_lab", "achieved": round(gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic("lab", "lab-16k"),
                     "algorithmic_bytes_per_launch": N * 15,
                     "hbm_achievable_copy": round(copy_rate_gbs(), 1)},
    }
    # the oracle, one thread, on the leading 4096x4096 crop
    import oracle
    sub = img[:4096, :4096].contiguous().cpu().numpy()
    t0 = time.perf_counter()
    oracle.rgb_to_lab(sub)
    sec = time.perf_counter() - t0
    rec["cpu_baseline"] = {"value": round(sub.shape[0] * sub.shape[1] / sec / 1e9, 4),
                           "unit": "Gpixel/s", "cores": 1, "kind": "oracle",
                           "seconds": round(sec, 2), "sample": "leading 4096x4096 crop"}
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fibsem-1k")
    ap.add_argument("--image-cache", default="",
                    help="single-image workloads: .npy file holding the image (written "
                         "on the first run, loaded afterwards)")
    ap.add_argument("--gen-only", action="store_true",
                    help="with --image-cache: write the image file and stop")
    ap.add_argument("--latency-reps", type=int, default=200,
                    help="rgb-256: graph replays timed one by one for the latency")
    ap.add_argument("--requests", type=int, default=300, help="served workload: requests")
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="served workload: factor on every image side")
    ap.add_argument("--cpu-crop", type=int, default=-1,
                    help="side of the crop the CPU oracle is timed on (0 = skip; "
                         "default 4096 in 2D, 224 in 3D)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent images would shard over GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1806_08741_amd import sslic, synth

    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload.startswith("batch-"):
        return bench_batch(args, int(args.workload.split("-")[1]))
    if args.workload == "served":
        return bench_served(args)
    if args.workload.startswith("contours-"):
        return bench_contours(args, args.workload.split("-", 1)[1])
    if args.workload == "lab-16k":
        return bench_lab(args)
    # persist-<workload>: the literal loop of Sec. 2.2 and Sec. 3.1 (distance
    # image set to infinity once, in stage 1, and kept across iterations)
    persist = args.workload.startswith("persist-")
    w = synth.WORKLOADS[args.workload.split("-", 1)[1] if persist else args.workload]
    wl_name = ("persist-" if persist else "") + w.name
    dev = torch.device("cuda", 0)
    img = workload_image(w, dev, args.image_cache)
    if args.gen_only:
        return

    ctx = sslic.Context(0)
    N = w.voxels
    K = sslic.num_clusters(w.dims, w.S)
    out = {"labels": torch.empty(N, dtype=torch.int32, device=dev),
           "centres": torch.empty((K, w.channels + len(w.dims)), dtype=torch.float64, device=dev),
           "counts": torch.empty(K, dtype=torch.int64, device=dev)}

    def step():
        ctx.run(img, w.S, w.m, w.iterations, connectivity=w.connectivity, out=out, sync=False,
                persist_distance=persist)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    L = sslic.lib()
    import ctypes
    sslic._check(L.sslic_profile_enable(ctx._h, 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = {}
    for k in ("seed", "bins", "sweep", "assign_persist", "update", "finalize", "connectivity"):
        ms = ctypes.c_double(0)
        n = ctypes.c_int64(0)
        sslic._check(L.sslic_profile_read(ctx._h, k.encode(), ctypes.byref(ms), ctypes.byref(n)))
        if n.value:
            prof[k] = {"ms_total": ms.value, "launches": n.value, "ms_mean": ms.value / n.value}
    sslic._check(L.sslic_profile_enable(ctx._h, 0))
    print(f"[bench] timed {args.steps} steps in {dt:.3f}s; kernels: "
          + ", ".join(f"{k} {v['ms_mean']:.3f} ms" for k, v in prof.items()),
          file=sys.stderr, flush=True)

    # sanity: the timed result is a labelling of the whole image (connectivity
    # adds labels K, K+1, ...)
    lab = out["labels"]
    n_labels = ctx.run(img, w.S, w.m, w.iterations, connectivity=w.connectivity,
                       out=out, persist_distance=persist)["n_labels"]
    assert int(lab.min()) >= 0 and int(lab.max()) < n_labels

    ms_step = dt / args.steps * 1e3
    value = N * w.iterations * args.steps / dt / 1e6
    # the iteration loop alone (bin sort, sweep, reduce step over every iteration)
    loop_ms = sum(prof[k]["ms_total"] for k in ("bins", "sweep", "assign_persist", "update", "finalize")
                  if k in prof) / args.steps
    copy_gbs = copy_rate_gbs()
    valu = None if persist else load_profile("valu", "sweep", w.name)
    dt_name = {torch.uint8: "u8", torch.uint16: "u16", torch.float32: "f32"}[w.dtype]
    cb = w.channels * BYTES[dt_name]
    # Algorithmic bytes per voxel of one launch of the dominant kernel.  The
    # sweep carries out both steps of an iteration: the assignment reads the
    # image and writes the label, the update reads image and label, so
    # 2 (C b + 4) bytes (it moves C b + 4 itself, being fused).  The
    # kept-distance assignment reads image and distance and writes label and
    # distance: C b + 12.
    per_vox = cb + 12 if persist else 2 * (cb + 4)
    moved_vox = cb + 12 if persist else cb + 4
    dom = "assign_persist" if persist else "sweep"
    bytes_launch = N * per_vox
    sec_launch = prof[dom]["ms_mean"] * 1e-3
    achieved = bytes_launch / sec_launch / 1e9
    traffic = load_traffic(dom, wl_name)
    # algorithmic FP32 work: every window covering a voxel costs one distance,
    # 3 flops per term (difference, multiply-add) over nd + C terms, with the
    # compare in place of the first term's add; windows cover K prod(2 S_i)
    # voxels in all (centres off the integer grid, no clipping)
    nd = len(w.dims)
    cover = K * float(np.prod([2 * s for s in w.S])) / N
    flops_vox = cover * 3 * (nd + w.channels)
    flops_launch = N * flops_vox
    tflops = flops_launch / sec_launch / 1e12
    rec = {
        "metric": "SLIC Mvoxel*iter/s (whole sslic_run per step; inputs resident in HBM)",
        "value": round(value, 1),
        "unit": "Mvoxel*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl_name, "dims": list(w.dims), "channels": w.channels,
                   "image_dtype": dt_name, "S": list(w.S), "m": w.m,
                   "iterations": w.iterations, "connectivity": w.connectivity, "K": K,
                   "distance_image": "kept across iterations" if persist else "reset every iteration",
                   "recipe": w.recipe},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_voxel": per_vox,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "launch_ms": round(prof[dom]["ms_mean"], 4),
                     "bytes_moved_per_voxel": moved_vox,
                     "hbm_achievable_copy": round(copy_gbs, 1),
                     "alu": {"achieved": round(tflops, 3), "peak": round(ALU_PEAK_TFLOPS, 1),
                             "unit": "TFLOP/s", "frac": round(tflops / ALU_PEAK_TFLOPS, 4),
                             "algorithmic_flops_per_launch": round(flops_launch),
                             "flops_per_voxel": round(flops_vox, 2),
                             "valu_busy": None if valu is None else valu.get("valu_busy")}},
        "stages": {"iteration_loop": {"Mvoxel_iter_s": round(N * w.iterations / loop_ms / 1e3, 1),
                                      "ms_per_run": round(loop_ms, 4)},
                   "end_to_end": {"Mvoxel_iter_s": round(value, 1), "ms_per_run": round(ms_step, 4)}},
        "kernels_ms": {k: round(v["ms_mean"], 4) for k, v in prof.items()},
    }
    if w.name == "rgb-256" and not persist:
        rec["latency"] = graph_latency(ctx, img, w, out, args.latency_reps)
    crop = args.cpu_crop if args.cpu_crop >= 0 else (4096 if len(w.dims) == 2 else 224)
    if crop > 0:
        rec["cpu_baseline"] = cpu_baseline(img, w, crop, persist)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark: grayscale reconstruction by dilation on one MI355X.

Contract: ``python bench.py --gpus N --steps K --warmup W`` prints ONE JSON
line.  A step is one whole reconstruction (all tiles, scans, seed detection,
queue propagation, cross-tile fixed point) of one synthetic workload whose
inputs are already resident in HBM.  Before each step the marker is restored
from a pristine device copy; that copy is not part of the step's timed
region (hipEvents around the library call on the bench's stream).

Workloads (--workload):
  c3i32  32768x32768 int32 smooth field, h-dome marker I - 4096 (default: the
         largest single-image configuration, in the paper's 32-bit integers)
  c1     512x512 uint8 Gaussian blobs, h-dome marker (latency bound)
  c2     4096x4096 uint8 tissue-like ellipses, fill-holes marker
  c3u8   32768x32768 uint8 ellipses, fill-holes marker
  c4     256 images, sides log-uniform 512..4096, one batched launch
         (HIP graph) vs the per-image loop
  c5     served stream: Poisson arrivals at 2000 req/s into the
         continuous-batching server
  edt    Euclidean distance transform (IWPP site propagation) of the 4096x4096
         tissue image: distance of every pixel outside the ellipses to the
         nearest ellipse pixel (ellipse pixels, value > 50, are background)
  edt32k the same on the 32768x32768 ellipse image of c3u8

Operation (--op, single-image workloads):
  dilate  reconstruction by dilation of the workload (default)
  erode   reconstruction by erosion of the dual workload: mask and marker
          complemented (255 - x / -1 - x), so the marker lies above the mask
  fill    fill holes of the workload's mask (frame-marker kernel plus the
          reconstruction by erosion, both inside the timed region)

Parameters: the library defaults, except for c4 (and any workload run with
--autotune on), where the library's autotuner (iwpp_autotune) first times its
candidate parameter sets on the resident workload, outside the timed steps;
the set used is reported in config.params.  Explicit flags override both.

Extras in the JSON line:
  roofline      for the dominant kernel (the persistent tile kernel):
                algorithmic bytes 3*sizeof(T) per pixel per launch over its
                hipEvent-measured duration, against 8 TB/s; `traffic` from the
                committed rocprofv3 counter summary when it matches the
                current kernel source, else null.
  parity        sha256 of the inputs and of the last timed output against the
                digests of the CPU oracle's result stored in
                tests/golden/full_size_sha256.txt (bit-exact check of the
                timed work itself).
  cv_protocol   the paper's timing protocol (10 runs, coefficient of variation
                at most 1%): whether the timed steps met it.
  also          (single-image default) the 4096^2 and 32768^2 uint8
                fill-holes workloads, timed the same way with fewer steps.
  cpu_baseline  the CPU oracle (sequential C) timed on this host: one core on
                the whole image for single images (the paper's serial
                baseline), all host cores (a process pool, one image or
                request per task) for the batch and the served stream.
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
sys.path.insert(0, ROOT)

METRIC = "Mpixel/s reconstruction (bit-exact) + % HBM roofline; batched p50/p99 latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SRCS = [os.path.join(ROOT, "paper_1605_00930_amd", "csrc", f)
               for f in ("iwpp_kernels.hip", "iwpp_edt.hip", "iwpp_device.h", "iwpp_internal.h")]


def log(msg: str) -> None:
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """sha256 (first 16 hex digits) over the device sources, in order."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def persistent_kernel_name(dtype: str, params: dict, mode: int) -> str:
    """The persistent kernel a single-image call launches: 32-row int32 tiles
    (the int32 default) in the plain persistent mode run the worker that
    prefetches the next tile."""
    tile_h = params.get("tile_h") or (32 if dtype == "i32" else 64)
    if dtype == "i32" and tile_h == 32 and not mode and not params.get("max_tile_visits"):
        return "k_persistent_pf (tile worker, next-tile prefetch)"
    return "k_persistent (tile worker)"


def load_traffic(workload: str):
    """HBM bytes per launch from profiles/traffic_k_persistent_<workload>.txt, or None if the
    summary is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_k_persistent_%s.txt" % workload)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


GOLDEN = os.path.join(ROOT, "tests", "golden", "full_size_sha256.txt")


def golden():
    """name -> (sha256 I, sha256 J, sha256 R) of the oracle's result, from the
    digests written by tests/golden/make_full_size_hashes.py."""
    out = {}
    if os.path.exists(GOLDEN):
        for ln in open(GOLDEN):
            if ln.startswith("#") or not ln.strip():
                continue
            f = ln.split()
            out[f[0]] = (f[4], f[5], f[6])
    return out


def host_cores() -> int:
    """Host threads for the pooled CPU baselines: the ones this process may
    run on, at most 16 (a one-GPU share of a host that serves several GPUs)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def make_workload(name: str, scale: int = 1):
    import synth

    if name == "c1":
        return [synth.c1()], "u8", "512x512 u8 gaussian blobs, h-dome h=40, 8-conn"
    if name == "c2":
        return [synth.c2()], "u8", "4096x4096 u8 ellipses (3000), fill-holes frame marker, 8-conn"
    if name == "c3u8":
        n = 32768 // scale
        return [synth.c3_u8(H=n, W=n)], "u8", "%dx%d u8 ellipses, fill-holes frame marker, 8-conn" % (n, n)
    if name == "c3i32":
        n = 32768 // scale
        return [synth.c3_i32(H=n, W=n)], "i32", "%dx%d i32 9x9-box field, h-dome h=4096, 8-conn" % (n, n)
    if name == "c4":
        return synth.c4(), "u8", "256 u8 images, sides log-uniform 512..4096, h-dome h~U{10..80}, 8-conn"
    raise ValueError(name)


def edt_image(name: str, scale: int = 1):
    """Binary image for the distance-transform workloads (0 = background =
    ellipse pixels)."""
    import synth

    if name == "edt":
        I, _ = synth.c2()
    else:
        n = 32768 // scale
        I, _ = synth.c3_u8(H=n, W=n)
    return np.where(I > 50, 0, 1).astype(np.uint8)


def bench_edt(args, torch, iwpp):
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    img = edt_image(args.workload, args.scale)
    log("generated %s in %.1f s" % (args.workload, time.perf_counter() - t0))
    H, W = img.shape
    it = torch.from_numpy(img).to(dev)
    del img
    sites = torch.empty((H, W), dtype=torch.int32, device=dev)
    dist2 = torch.empty_like(sites)
    stream = torch.cuda.Stream()
    params = {"timing": 1}
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    call_ms, kern_ms, stats = [], [], None
    torch.cuda.synchronize()
    for step in range(args.warmup + args.steps):
        with torch.cuda.stream(stream):
            ev0.record(stream)
            iwpp.edt_async(it, 8, sites=sites, dist2=dist2, params=params, stream=stream)
            ev1.record(stream)
        st = iwpp.stream_status(stream)
        log("step %d: %.3f ms (kernel %.3f ms, visits %d)"
            % (step, ev0.elapsed_time(ev1), st["kernel_ms"], st["tile_visits"]))
        if step >= args.warmup:
            call_ms.append(ev0.elapsed_time(ev1))
            kern_ms.append(st["kernel_ms"])
            stats = st
    ms = float(np.mean(call_ms))
    kms = float(np.mean(kern_ms))
    px = H * W
    achieved = 8 * px / (kms * 1e-3) / 1e9
    return {
        "metric": METRIC, "value": round(px / (ms * 1e-3) / 1e6, 2), "unit": "Mpixel/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "op": "edt", "H": H, "W": W, "conn": 8,
                   "desc": "distance to the nearest ellipse pixel (uint8 in, int32 sites and "
                           "squared distances out)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "k_persistent_edt (tile worker)",
                     "kernel_ms": round(kms, 4), "algorithmic_bytes_per_launch": 8 * px},
        "step_stats": {k: stats[k] for k in ("tiles", "tile_visits", "sweep_rounds", "idle_ms",
                                             "load_ms", "solve_ms", "store_ms", "sync_ms")},
        "ms_min": round(float(np.min(call_ms)), 4), "ms_cv": round(float(np.std(call_ms) / ms), 4),
    }


def _oracle_task(spec):
    """One pooled oracle run (a child process): reconstruct image or request
    ``k`` of the batch / pool recipe and return (pixels, seconds)."""
    import oracle
    import synth

    kind, k = spec
    if kind == "c4":
        (I, J), = synth.c4(only=[k])
    else:
        (I, J, _), = synth.c5_pool(n=256, only=[k])
    t0 = time.perf_counter()
    rc, _ = oracle.reconstruct(J, I, 8)
    dt = time.perf_counter() - t0
    assert rc == oracle.OK
    return I.size, dt


def cpu_baseline(name: str, budget_s: float = 0.0, op: str = "dilate", pool: int = 256):
    """Time the oracle on this host.

    Single images: one core on the whole image (the paper's serial baseline),
    repeated while within ``budget_s`` (at least once, at most 10 runs).
    Batch and served stream: a process pool over all host cores (at most the
    16 of one GPU's share), one image or request per task, over the whole
    batch or pool; the rate is pixels (or requests) over the pool's wall time.
    ``budget_s`` > 0 bounds the 32768^2 images to their first run."""
    import oracle
    import synth

    if name in ("c4", "c5"):
        from concurrent.futures import ProcessPoolExecutor

        n = 256 if name == "c4" else pool
        cores = host_cores()
        specs = [(name, k) for k in range(n)]
        t0 = time.perf_counter()
        with ProcessPoolExecutor(max_workers=cores) as ex:
            res = list(ex.map(_oracle_task, specs, chunksize=1))
        wall = time.perf_counter() - t0
        px = sum(r[0] for r in res)
        busy = sum(r[1] for r in res)
        out = {"value": round(px / wall / 1e6, 3), "unit": "Mpixel/s", "cores": cores,
               "kind": "oracle",
               "sample": "all %d %s on a pool of %d processes (generation included in the "
                         "wall time, %.1f s of it reconstructing)" % (
                             n, "images of the batch" if name == "c4" else
                             "requests of the pool", cores, busy)}
        if name == "c5":
            out["req_s"] = round(n / wall, 2)
        return out
    if name in ("edt", "edt32k"):
        img = edt_image("edt")
        px = t = 0.0
        runs = 0
        while runs < 1 or (t < max(budget_s, 10.0) and runs < 10):
            t0 = time.perf_counter()
            rc, _, _ = oracle.edt(img, 8)
            t += time.perf_counter() - t0
            assert rc == 0
            px += img.size
            runs += 1
        return {"value": round(px / t / 1e6, 3), "unit": "Mpixel/s", "cores": 1,
                "kind": "oracle", "sample": "4096x4096 image of the edt recipe, %d run(s), "
                                            "%.1f s of CPU time" % (runs, t)}
    if name == "c1":
        I, J = synth.c1()
    elif name == "c2":
        I, J = synth.c2()
    elif name == "c3u8":
        I, J = synth.c3_u8()
    elif name == "c3i32":
        I, J = synth.c3_i32()
    else:
        raise ValueError(name)
    if op == "erode":
        J, I = np.invert(J), np.invert(I)
    big = I.size > 1 << 26
    limit = budget_s if budget_s > 0 else (0.0 if big else 20.0)
    times = []
    while not times or (sum(times) < limit and len(times) < 10):
        t0 = time.perf_counter()
        if op == "fill":
            rc, _ = oracle.fill_holes(I, 8)
        elif op == "erode":
            rc, _ = oracle.reconstruct_erode(J, I, 8)
        else:
            rc, _ = oracle.reconstruct(J, I, 8)
        times.append(time.perf_counter() - t0)
        assert rc == 0
    t = float(np.median(times))
    return {"value": round(I.size / t / 1e6, 3), "unit": "Mpixel/s", "cores": 1,
            "kind": "oracle",
            "sample": "whole %dx%d image, median of %d run(s) on one core, %.1f s of CPU time"
                      % (I.shape[0], I.shape[1], len(times), sum(times))}


def cv_protocol(times):
    """The paper's protocol: 10 runs per configuration with a coefficient of
    variation of at most 1%."""
    cv = float(np.std(times) / np.mean(times))
    return {"runs": len(times), "cv": round(cv, 4), "bound": 0.01,
            "held": bool(len(times) >= 10 and cv <= 0.01)}


def bench_single(args, torch, iwpp, workload=None, steps=None, warmup=None, quiet=False):
    workload = workload or args.workload
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    pairs, dt, desc = make_workload(workload, args.scale)
    log("generated %s in %.1f s" % (workload, time.perf_counter() - t0))
    (I, J), = pairs
    if args.op == "erode":
        I, J = np.invert(I), np.invert(J)
    H, W = I.shape
    import synth

    in_sha = {"I": synth.sha256(I), "J": synth.sha256(J)}
    Jt0 = torch.from_numpy(J).to(dev)
    It = torch.from_numpy(I).to(dev)
    del pairs, I, J
    Jt = torch.empty_like(Jt0)
    stream = torch.cuda.Stream()
    params = {"timing": 1}
    tuned = None
    # the tuner times reconstructions by dilation: it runs for --op dilate
    if args.autotune == "on" and args.op == "dilate":
        t0 = time.perf_counter()
        tuned = {k: v for k, v in iwpp.autotune(Jt0, It, 8, stream=stream).items() if v}
        log("autotuned in %.1f s: %s" % (time.perf_counter() - t0, tuned))
        params.update(tuned)
    for k in ("tile_h", "sweeps", "mode", "seed_queue", "queue_waves", "bands", "first_pass"):
        v = getattr(args, k)
        if v is not None:
            params[k] = v
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    call_ms, kern_ms, stats = [], [], None
    torch.cuda.synchronize()
    for step in range(warmup + steps):
        if step == warmup:
            torch.cuda.synchronize()
            t_wall0 = time.perf_counter()
        with torch.cuda.stream(stream):
            if args.op == "fill":
                ev0.record(stream)
                iwpp.fill_holes(It, Jt, 8, params=params, stream=stream, check=False)
                ev1.record(stream)
            else:
                Jt.copy_(Jt0)
                ev0.record(stream)
                iwpp.reconstruct_async(Jt, It, 8, params=params, stream=stream,
                                       erosion=args.op == "erode")
                ev1.record(stream)
        st = iwpp.stream_status(stream)
        if not quiet or step == warmup + steps - 1:
            log("%s step %d: %.3f ms (kernel %.3f ms, visits %d)"
                % (workload, step, ev0.elapsed_time(ev1), st["kernel_ms"], st["tile_visits"]))
        if st["rc"] != iwpp.OK:
            raise RuntimeError("%s step %d: status %d" % (workload, step, st["rc"]))
        if step >= warmup:
            call_ms.append(ev0.elapsed_time(ev1))
            kern_ms.append(st["kernel_ms"])
            stats = st
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall0
    # bit-exactness of the last timed output: its digest against the oracle's
    out_sha = synth.sha256(Jt.cpu().numpy())
    want = golden().get(workload) if (args.op == "dilate" and args.scale == 1) else None
    if want is None:
        parity = {"checked": False, "reason": "no stored oracle digest for this workload/op/scale",
                  "inputs_sha256": in_sha, "output_sha256": out_sha}
    else:
        parity = {"checked": True, "inputs_match": in_sha["I"] == want[0] and in_sha["J"] == want[1],
                  "bit_exact": out_sha == want[2], "inputs_sha256": in_sha,
                  "output_sha256": out_sha, "oracle_sha256": want[2]}
    del Jt, Jt0, It
    torch.cuda.empty_cache()
    es = 1 if dt == "u8" else 4
    ms = float(np.mean(call_ms))
    kms = float(np.mean(kern_ms))
    px = H * W
    achieved = 3 * es * px / (kms * 1e-3) / 1e9
    traffic = load_traffic(workload) if args.op == "dilate" else None
    res = {
        "metric": METRIC, "value": round(px / (ms * 1e-3) / 1e6, 2), "unit": "Mpixel/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dt,
        "data": "synthetic",
        "config": {"workload": workload, "op": args.op, "desc": desc, "H": H, "W": W,
                   "conn": 8, "autotuned": tuned is not None,
                   "params": {k: v for k, v in params.items() if k != "timing"}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": persistent_kernel_name(dt, params, params.get("mode", 0)),
                     "kernel_ms": round(kms, 4),
                     "algorithmic_bytes_per_launch": 3 * es * px},
        "parity": parity,
        "step_stats": dict({k: stats[k] for k in ("tiles", "tile_visits", "sweep_rounds",
                                                  "pixels_queued", "queue_overflows",
                                                  "reprocessed", "requeued", "launches",
                                                  "queue_iterations", "idle_ms", "load_ms",
                                                  "solve_ms", "store_ms", "sync_ms")},
                           visits_per_tile=round(stats["tile_visits"] / stats["tiles"], 3)),
        "ms_min": round(float(np.min(call_ms)), 4), "ms_cv": round(float(np.std(call_ms) / ms), 4),
        "cv_protocol": cv_protocol(call_ms),
        "wall_ms_per_step_incl_restore": round(wall * 1e3 / steps, 4),
    }
    return res


def bench_batched(args, torch, iwpp):
    dev = torch.device("cuda:0")
    import synth

    pairs, dt, desc = make_workload("c4")
    want = golden()
    inputs_match = all(synth.sha256(I) == want.get("c4/%d" % k, ("",) * 3)[0]
                       and synth.sha256(J) == want.get("c4/%d" % k, ("",) * 3)[1]
                       for k, (I, J) in enumerate(pairs))
    pristine = [torch.from_numpy(J).to(dev) for I, J in pairs]
    masks = [torch.from_numpy(I).to(dev) for I, J in pairs]
    px = sum(I.size for I, J in pairs)
    del pairs
    work = [p.clone() for p in pristine]
    stream = torch.cuda.Stream()
    params = {"timing": 1}
    tuned = None
    if args.autotune != "off":
        # the plan resolves its parameters for the size class of its largest
        # image: tune on that image (on a scratch copy; not timed)
        big = max(range(len(masks)), key=lambda k: masks[k].numel())
        t0 = time.perf_counter()
        tuned = {k: v for k, v in iwpp.autotune(pristine[big], masks[big], 8,
                                                stream=stream).items() if v}
        log("autotuned on image %d in %.1f s: %s" % (big, time.perf_counter() - t0, tuned))
        params.update(tuned)
    if args.tile_h:
        params["tile_h"] = args.tile_h
    if args.sweeps is not None:
        params["sweeps"] = args.sweeps
    if args.first_pass is not None:
        params["first_pass"] = args.first_pass
    plan = iwpp.Batch(list(zip(work, masks)), 8, params=params)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    times, kern = [], []
    torch.cuda.synchronize()
    for step in range(args.warmup + args.steps):
        if step == args.warmup:
            torch.cuda.synchronize()
            t_wall0 = time.perf_counter()
        with torch.cuda.stream(stream):
            for w, p in zip(work, pristine):
                w.copy_(p)
            ev0.record(stream)
        plan.launch(stream=stream, graph=True)
        with torch.cuda.stream(stream):
            ev1.record(stream)
        st = plan.status()
        log("step %d: %.3f ms (kernel %.3f ms)" % (step, ev0.elapsed_time(ev1), st["kernel_ms"]))
        if step >= args.warmup:
            times.append(ev0.elapsed_time(ev1))
            kern.append(st["kernel_ms"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall0
    plan.close()
    # bit-exactness of the last timed launch: every image's digest against the oracle's
    differ = [k for k, w in enumerate(work)
              if synth.sha256(w.cpu().numpy()) != want.get("c4/%d" % k, ("",) * 3)[2]]
    parity = {"checked": len(want) > 0, "images": len(work), "inputs_match": inputs_match,
              "bit_exact": not differ, "images_differing": differ[:16]}
    # the plain per-image path on the same GPU, for comparison
    per_image = []
    lat = []
    for rep in range(2):
        with torch.cuda.stream(stream):
            for w, p in zip(work, pristine):
                w.copy_(p)
            ev0.record(stream)
        for w, m in zip(work, masks):
            e_a = torch.cuda.Event(enable_timing=True)
            e_b = torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(stream):
                e_a.record(stream)
            iwpp.reconstruct_async(w, m, 8, params={k: v for k, v in params.items() if k != "timing"},
                                   stream=stream)
            with torch.cuda.stream(stream):
                e_b.record(stream)
            if rep == 1:
                lat.append((e_a, e_b))
        with torch.cuda.stream(stream):
            ev1.record(stream)
        torch.cuda.synchronize()
        if rep == 1:
            per_image.append(ev0.elapsed_time(ev1))
    lats = sorted(a.elapsed_time(b) for a, b in lat)
    ms = float(np.mean(times))
    kms = float(np.mean(kern))
    achieved = 3 * px / (kms * 1e-3) / 1e9
    return {
        "metric": METRIC, "value": round(px / (ms * 1e-3) / 1e6, 2), "unit": "Mpixel/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dt,
        "data": "synthetic",
        "config": {"workload": "c4", "desc": desc, "images": len(pristine), "pixels": px,
                   "conn": 8, "graph": True,
                   "params": {k: v for k, v in params.items() if k != "timing"},
                   "autotuned": tuned is not None},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic("c4"), "kernel": "k_persistent (tile worker)",
                     "kernel_ms": round(kms, 4), "algorithmic_bytes_per_launch": 3 * px},
        "per_image_loop": {"ms": round(per_image[0], 4),
                           "value": round(px / (per_image[0] * 1e-3) / 1e6, 2),
                           "image_ms_p50": round(lats[len(lats) // 2], 4),
                           "image_ms_p99": round(lats[min(len(lats) - 1, int(0.99 * len(lats)))], 4)},
        "batched_speedup_vs_loop": round(per_image[0] / ms, 3),
        "parity": parity,
        "cv_protocol": cv_protocol(times),
        "wall_ms_per_step_incl_restore": round(wall * 1e3 / args.steps, 4),
    }


def bench_served(args, torch, iwpp):
    """Poisson arrivals into the continuous-batching server.  A pool of
    distinct requests is generated once and kept on the device; each arrival
    picks one, gets its own working marker (filled from the pristine copy by
    the server on the device) and is submitted at its arrival time."""
    import threading

    import synth

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    pool = synth.c5_pool(seed=4, n=args.pool)
    log("generated %d pool requests in %.1f s" % (len(pool), time.perf_counter() - t0))
    masks = [torch.from_numpy(I).to(dev) for I, J, _ in pool]
    pristine = [torch.from_numpy(J).to(dev) for I, J, _ in pool]
    px = [I.size for I, J, _ in pool]
    del pool
    # working markers per pool request: enough that the submitting loop
    # rarely waits for one to be collected (arrivals stay open-loop)
    copies = args.copies
    work = [[torch.empty_like(p) for _ in range(copies)] for p in pristine]
    times, idx = synth.c5_arrivals(seed=4, rate=args.rate, duration=args.duration, pool=len(masks))
    srv = iwpp.Server(int(args.budget_gb * 1e9), "u8", 8, streams=args.streams,
                      max_inflight=args.max_inflight)
    # warm the kernels and the slots
    for k in range(min(8, len(masks))):
        srv.wait(srv.submit(work[k][0], masks[k], marker_init=pristine[k]))
    torch.cuda.synchronize()
    lat, done_px, errors = [], [0], [0]
    lock = threading.Lock()

    def waiter(q):
        while True:
            item = q.get()
            if item is None:
                return
            t, k, ev = item
            rc, l = srv.wait(t)
            with lock:
                if rc != iwpp.OK:
                    errors[0] += 1
                lat.append(l)
                done_px[0] += px[k]
            ev.set()  # the working marker may be reused

    import queue as _queue

    qq = _queue.Queue()
    th = threading.Thread(target=waiter, args=(qq,), daemon=True)
    th.start()
    busy = {}  # (pool index, copy) -> event set when its last request was collected
    uses = [0] * len(masks)
    late = 0
    start = time.perf_counter()
    for ta, k in zip(times, idx):
        k = int(k)
        delay = start + ta - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        elif delay < -0.005:
            late += 1
        key = (k, uses[k] % copies)
        uses[k] += 1
        prev = busy.get(key)
        if prev is not None:
            prev.wait()
        ev = threading.Event()
        t = srv.submit(work[k][key[1]], masks[k], marker_init=pristine[k])
        busy[key] = ev
        qq.put((t, k, ev))
    qq.put(None)
    th.join()
    wall = time.perf_counter() - start
    srv.close()
    # bit-exactness: the last result held by working marker 0 of every pool
    # request that ran, against the oracle's digest (the pool of 256 requests
    # drawn with seed 4 is the one the digests cover)
    want = golden()
    used = [k for k in range(len(masks)) if uses[k] > 0]
    if len(masks) == 256:
        differ = [k for k in used
                  if synth.sha256(work[k][0].cpu().numpy()) != want.get("c5/%d" % k, ("",) * 3)[2]]
        parity = {"checked": True, "requests_checked": len(used), "bit_exact": not differ,
                  "requests_differing": differ[:16]}
    else:
        parity = {"checked": False, "reason": "digests cover the 256-request pool only"}
    lat_ms = sorted(x / 1e3 for x in lat)
    value = done_px[0] / wall / 1e6
    return {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": len(lat), "warmup": 8, "ms_per_step": round(wall * 1e3 / max(1, len(lat)), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "c5", "rate_req_s": args.rate, "duration_s": args.duration,
                   "pool": len(masks), "copies": copies, "streams": args.streams,
                   "max_inflight": args.max_inflight, "budget_gb": args.budget_gb, "conn": 8},
        "served": {"requests": len(lat), "errors": errors[0], "req_s": round(len(lat) / wall, 1),
                   "offered_req_s": round(len(times) / args.duration, 1),
                   "late_arrivals": late,
                   "p50_ms": round(lat_ms[len(lat_ms) // 2], 3),
                   "p99_ms": round(lat_ms[min(len(lat_ms) - 1, int(0.99 * len(lat_ms)))], 3),
                   "max_ms": round(lat_ms[-1], 3), "wall_s": round(wall, 3)},
        "parity": parity,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3i32",
                    choices=["c1", "c2", "c3u8", "c3i32", "c4", "c5", "edt", "edt32k"])
    ap.add_argument("--scale", type=int, default=1, help="divide the 32K side (c3*) by this")
    ap.add_argument("--op", default="dilate", choices=["dilate", "erode", "fill"],
                    help="single-image workloads: which operation to time")
    ap.add_argument("--tile-h", dest="tile_h", type=int, default=None)
    ap.add_argument("--sweeps", type=int, default=None)
    ap.add_argument("--mode", type=int, default=None)
    ap.add_argument("--seed-queue", dest="seed_queue", type=int, default=None)
    ap.add_argument("--queue-waves", dest="queue_waves", type=int, default=None)
    ap.add_argument("--first-pass", dest="first_pass", type=int, default=None, choices=[1, 2],
                    help="order of the first visits' tile groups: 1 by rows, 2 diagonals first")
    ap.add_argument("--bands", type=int, default=None, help="gray-level classes (mode 2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", choices=["auto", "on", "off"], default="auto",
                    help="tune parameters on the resident workload before timing, outside the "
                         "timed region (auto: on for c4 only, whose recipe asks for it)")
    ap.add_argument("--rate", type=float, default=2000.0, help="c5 arrivals per second")
    ap.add_argument("--duration", type=float, default=10.0, help="c5 seconds of arrivals")
    ap.add_argument("--pool", type=int, default=256, help="c5 distinct requests")
    ap.add_argument("--copies", type=int, default=4, help="c5 working markers per pool request")
    ap.add_argument("--streams", type=int, default=2, help="c5 server launch slots")
    ap.add_argument("--max-inflight", dest="max_inflight", type=int, default=64)
    ap.add_argument("--budget-gb", dest="budget_gb", type=float, default=64.0)
    ap.add_argument("--cpu-budget", type=float, default=0.0,
                    help="seconds of oracle runs for single images (0: one run of a 32768^2 "
                         "image, up to 20 s of runs otherwise)")
    ap.add_argument("--also", default="auto",
                    help="comma-separated single-image workloads timed after the main one and "
                         "reported under 'also' (auto: c2,c3u8 when the main workload is the "
                         "default c3i32 dilation; none: skip)")
    ap.add_argument("--also-steps", dest="also_steps", type=int, default=10)
    ap.add_argument("--calib-copy-mib", default="",
                    help="comma-separated sizes in MiB: run the library copy kernel on each "
                         "(the known-size reference that scales the profiler's byte counters)")
    args = ap.parse_args()
    if args.op != "dilate" and args.workload in ("c4", "c5", "edt", "edt32k"):
        ap.error("--op applies to single-image workloads only")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only (the multi-GPU split is a design, not code); --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1605_00930_amd as iwpp

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if not os.path.exists(iwpp.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    iwpp._load()

    for mib in [int(m) for m in args.calib_copy_mib.split(",") if m]:
        n = mib << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(3):
            iwpp.device_copy(b, a)
        torch.cuda.synchronize()
        del a, b

    if args.workload == "c4":
        res = bench_batched(args, torch, iwpp)
    elif args.workload == "c5":
        res = bench_served(args, torch, iwpp)
    elif args.workload in ("edt", "edt32k"):
        res = bench_edt(args, torch, iwpp)
    else:
        res = bench_single(args, torch, iwpp)
        also = args.also
        if also == "auto":
            also = "c2,c3u8" if (args.workload == "c3i32" and args.op == "dilate"
                                 and args.scale == 1 and args.mode is None) else "none"
        if also != "none":
            res["also"] = {}
            for w in also.split(","):
                r = bench_single(args, torch, iwpp, workload=w, steps=args.also_steps,
                                 warmup=3, quiet=True)
                res["also"][w] = {k: r[k] for k in ("value", "unit", "ms_per_step", "dtype",
                                                    "config", "roofline", "parity",
                                                    "cv_protocol", "step_stats")}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_budget, args.op, args.pool)
    res["kernel_source_sha256"] = kernel_source_hash()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

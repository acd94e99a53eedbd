#!/usr/bin/env python3
"""Throughput benchmark of the gfx950 two-pass connected component labeling.

One step = one full ccl_label call (tile scan, boundary merge, flatten,
rank scan, component labels, labeling pass) on a device-resident image.
Default workload: the paper-scale single image, 21568 x 21568 uint8
(465.18 Mpx, the size of the paper's largest NLCD image at one byte per
pixel), i.i.d. Bernoulli foreground p = 0.5 from seed 0, 8-connectivity.

Prints ONE JSON line with the throughput (Gpixel/s), the roofline of the
dominant kernel (its duration from HIP events recorded on the stream it runs
on, during the timed steps), the CPU oracle timed on the host, whether the
benchmarked output is bit-exact against that oracle, the two-row vs one-row
scan comparison, the batched forms (256 uneven images: one batch call, the
captured graph, a loop of single calls) and the served form (Poisson request
streams through the continuous-batching server: p50/p99 latency, Gpixel/s,
alone == mix).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E peak, GB/s
BYTES_PER_PX = 5            # compulsory: 1 B image read + 4 B int32 label write
# algorithmic bytes per pixel of each phase's launch: the tile scan reads the
# image (1 B/px); the labeling pass writes the labels (4 B/px) and reads the
# image information once more, as a 1-bit mask in place of the bytes
# (1/8 B/px)
PHASE_BYTES_PER_PX = {"tile_scan": 1.0, "labeling_pass": 4.125}
METRIC = "Gpixel/s and % of HBM roofline, 8-conn, bit-exact; batched/served vs single"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("paper_1606_05973_amd/csrc/ccl_kernels.hpp", "paper_1606_05973_amd/csrc/ccl_api.hip"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_counters(kernel: str, workload_key: str) -> dict:
    """A kernel's figures from committed rocprofv3 counter runs (HBM bytes per
    launch, VALU busy and lane use), if they were taken on the current kernel
    sources; else an empty dict."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return {}
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        return {}
    if data.get("kernel_source_sha") != kernel_source_hash():
        return {}
    return data.get("workloads", {}).get(workload_key, {}).get(kernel) or {}


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _median_ms(torch, fn, reps):
    """Median over reps of fn()'s duration, HIP events on the current stream."""
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts)


def bench_batched(torch, n, conn, reps, verify):
    """The uneven batch: n images, one ccl_label_batch call (autotuned tile)
    vs a loop of single ccl_label calls vs a replay of the captured graph."""
    import tempfile

    from paper_1606_05973_amd import autotune, ccl, inputs
    dev = torch.device("cuda:0")
    specs = inputs.batch_specs(n, seed=0)
    imgs = [inputs.make(sp, device=dev) for sp in specs]
    log(f"batched conn {conn}: {n} images made")
    outs = [torch.empty(tuple(im.shape), dtype=torch.int32, device=dev) for im in imgs]
    single = [torch.empty_like(o) for o in outs]
    px = sum(im.numel() for im in imgs)
    with tempfile.TemporaryDirectory() as td:
        plan = autotune.Autotuner(os.path.join(td, "tiles.json")).plan_batch(imgs, [conn] * n)
    tiles = plan["tiles"]
    log(f"batched conn {conn}: schedule {plan['schedule']} ({plan['ms']})")
    ccl.reserve(ccl.batch_workspace_bytes([tuple(im.shape) for im in imgs], conn, tiles=tiles))

    def loop():
        for im, o in zip(imgs, single):
            ccl.label(im, conn, out=o)
    for _ in range(2):
        ccl.label_batch(imgs, conn, outs=outs, tiles=tiles)
        loop()
    t_batch = _median_ms(torch, lambda: ccl.label_batch(imgs, conn, outs=outs, tiles=tiles), reps)
    t_loop = _median_ms(torch, loop, reps)
    g = ccl.BatchGraph(imgs, conn, outs=outs, tiles=tiles)
    g.launch()
    t_graph = _median_ms(torch, g.launch, reps)
    g.close()
    torch.cuda.synchronize()
    log(f"batched conn {conn}: timed")
    rec = {
        "images": n, "conn": conn, "mpx": round(px / 1e6, 2),
        "schedule": plan["schedule"], "tuned_ms": plan["ms"],
        "tile": list(ccl.tile_shape(plan["one_tile"], conn)) if plan["schedule"] == "one tile" else "per bucket",
        "batched_gpx_per_s": round(px / (t_batch * 1e-3) / 1e9, 2),
        "graph_gpx_per_s": round(px / (t_graph * 1e-3) / 1e9, 2),
        "single_loop_gpx_per_s": round(px / (t_loop * 1e-3) / 1e9, 2),
        "batched_ms": round(t_batch, 3), "graph_ms": round(t_graph, 3), "single_loop_ms": round(t_loop, 3),
        "batched_equals_single": all(torch.equal(a, b) for a, b in zip(outs, single)),
    }
    if verify:
        import numpy as np

        import oracle
        rec["bit_exact"] = all(np.array_equal(o.cpu().numpy(), oracle.cclremsp(im.cpu().numpy(), conn)[0])
                               for im, o in zip(imgs, outs))
    return rec


def bench_served(torch, rates, nreq, verify):
    """Request streams through the continuous-batching server: Poisson
    arrivals at each rate, then a closed-loop run ("max": every request
    submitted at once) that measures the served capacity."""
    import numpy as np

    from paper_1606_05973_amd import ccl, inputs, serve
    dev = torch.device("cuda:0")
    _, specs = inputs.serve_specs(1, 1.0, seed=0, pool=256)
    pool = [inputs.make(sp, device=dev) for sp in specs]
    # one label buffer per (pool image, connectivity): requests for the same
    # pair write the same labels, and submission stays cheap enough on the
    # host to offer the higher rates
    outs = {(i, c): torch.empty(tuple(im.shape), dtype=torch.int32, device=dev)
            for i, im in enumerate(pool) for c in (4, 8)}
    torch.cuda.synchronize()
    log("served: pool made")
    res = {"pool_images": len(pool), "requests_per_rate": nreq, "rates": {}}
    all_ok = True
    # one server for all rates: its slot workspaces are allocated once
    srv = serve.Server(hbm_budget=16 << 30, n_streams=3, max_batch=64, device=dev)
    warm, _ = inputs.serve_specs(64, 1000.0, seed=1, pool=256)
    for q in warm:
        srv.submit(pool[q["img"]], q["conn"], out=outs[(q["img"], q["conn"])], ready=False)
    srv.drain()
    for rate in rates:
        closed = rate == "max"
        reqs, _ = inputs.serve_specs(nreq, 1000.0 if closed else float(rate), seed=0, pool=256)
        before = srv.stats()
        kept, late = [], 0.0
        t0 = time.perf_counter()
        for n, q in enumerate(reqs):
            if not closed:
                # sleep until the arrival time; requests already due go at once
                wait = t0 + q["t"] - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
                else:
                    late = max(late, -wait)
            r = srv.submit(pool[q["img"]], q["conn"], out=outs[(q["img"], q["conn"])], ready=False)
            if n % 97 == 0:
                kept.append(r)
        t_sub = time.perf_counter()
        srv.drain()
        t1 = time.perf_counter()
        st = srv.stats(t0, t1)
        done = st["completed"] - before["completed"]
        # per-rate latency percentiles: over this rate's requests only
        rate_stats = srv.latency_stats(int(before["submitted"]) + 1, int(st["submitted"]))
        mpx = sum(pool[q["img"]].numel() for q in reqs) / 1e6
        ok = True
        for r in kept:
            alone = ccl.label(r.img, r.conn)
            ok &= bool(torch.equal(alone, r.labels))
        if verify:
            import oracle
            for r in kept[:4]:
                ok &= bool(np.array_equal(r.labels.cpu().numpy(), oracle.cclremsp(r.img.cpu().numpy(), r.conn)[0]))
        all_ok &= ok
        px = st["pixels_completed"] - before["pixels_completed"]
        log(f"served rate {rate}: {done} done in {t1 - t0:.2f} s, p50 {rate_stats['p50_ms']:.2f} ms, "
            f"p99 {rate_stats['p99_ms']:.2f} ms, {px / (t1 - t0) / 1e9:.1f} Gpx/s")
        rec = {
            "gpx_per_s": round(px / (t1 - t0) / 1e9, 2),
            "req_per_s": round(done / (t1 - t0), 1),
            "p50_ms": round(rate_stats["p50_ms"], 3), "p99_ms": round(rate_stats["p99_ms"], 3),
            "mean_ms": round(rate_stats["mean_ms"], 3), "completed": done, "mpx": round(mpx, 1),
            "batches": st["batches"] - before["batches"], "max_batches_in_flight": st["max_batches_in_flight"],
            "host_submit_s": round(t_sub - t0, 3),
            "alone_equals_mix_checked": len(kept),
        }
        if closed:
            rec["offered"] = "all requests submitted at once (closed loop)"
        else:
            rec["offered_gpx_per_s"] = round(mpx / 1e3 / reqs[-1]["t"], 2)
            rec["max_submit_lag_ms"] = round(late * 1e3, 3)
        res["rates"][str(rate)] = rec
    srv.close()
    res["alone_equals_mix"] = all_ok
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=21568, help="image side (square)")
    ap.add_argument("--p", type=float, default=0.5, help="Bernoulli foreground probability")
    ap.add_argument("--content", choices=["bernoulli", "grf", "gray"], default="bernoulli",
                    help="gray: grayscale bytes binarized inside the labeling at --level")
    ap.add_argument("--gray-bins", type=int, default=0,
                    help="gray-level labeling (equal-valued neighbours connect) of the grayscale field "
                         "quantized into this many-wide value bins (0 = binary labeling)")
    ap.add_argument("--level", type=int, default=None,
                    help="foreground iff byte > level (default 0 = nonzero; 127 for --content gray)")
    ap.add_argument("--sigma", type=float, default=8.0, help="GRF smoothing (px) when --content grf")
    ap.add_argument("--q", type=float, default=0.5, help="GRF threshold quantile when --content grf")
    ap.add_argument("--pitch", type=int, default=0,
                    help="image row pitch in bytes (0 = W); e.g. 256 rounds rows up to 256-byte alignment")
    ap.add_argument("--conn", type=int, default=8)
    ap.add_argument("--scan", choices=["pair", "row"], default="pair",
                    help="tile-local scan: runs of row pairs (default, 8-conn) or of single rows")
    ap.add_argument("--tile", type=int, default=0, help="tile configuration id (0 = default)")
    ap.add_argument("--cpu-runs", type=int, default=3, help="oracle runs for cpu_baseline (0 = skip)")
    ap.add_argument("--cpu-threads", default="1,2,4,8,16",
                    help="thread counts of the host PARemSP curve ('' = skip; capped at 16 and at the host's)")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--ablation-steps", type=int, default=5,
                    help="steps of the one-row vs two-row scan comparison (0 = skip)")
    ap.add_argument("--order-steps", type=int, default=10,
                    help="steps of the provisional-order (paper numbering) measurement (0 = skip)")
    ap.add_argument("--batch", type=int, default=256, help="images in the batched measurement (0 = skip)")
    ap.add_argument("--batch-reps", type=int, default=10)
    ap.add_argument("--serve-rates", default="1000,5000,10000,20000,50000,max",
                    help="Poisson request rates (req/s) for the served measurement, 'max' = closed loop "
                         "('' = skip)")
    ap.add_argument("--serve-requests", type=int, default=20000, help="requests per rate")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after timing, run one device-to-device copy of this many MiB (a plain copy kernel "
                         "of known size, used to scale rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build labels on one GPU; --gpus must be 1 "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1606_05973_amd import ccl, inputs

    dev = torch.device("cuda:0")
    S = args.size
    stride = S if args.pitch <= 0 else (S + args.pitch - 1) // args.pitch * args.pitch
    gray = args.gray_bins > 0
    if gray and args.content != "gray":
        ap.error("--gray-bins needs --content gray")
    level = args.level if args.level is not None else (127 if args.content == "gray" and not gray else 0)
    if args.content == "grf":
        img = inputs.grf(S, S, args.sigma, args.q, seed=0, device=dev, stride=stride)
        content = f"thresholded Gaussian random field sigma={args.sigma} q={args.q} seed 0"
    elif args.content == "gray":
        img = inputs.gray(S, S, args.sigma, seed=0, device=dev, stride=stride)
        content = f"grayscale Gaussian field sigma={args.sigma} seed 0"
        if args.gray_bins > 0:
            img.copy_(img // args.gray_bins)
            content += f", bytes // {args.gray_bins}, gray-level labeling"
    else:
        img = inputs.bernoulli(S, S, args.p, seed=0, device=dev, stride=stride)
        content = f"Bernoulli p={args.p} seed 0"
    out = torch.empty((S, S), dtype=torch.int32, device=dev)
    kdev = torch.zeros(1, dtype=torch.int32, device=dev)
    scan = ccl.SCAN_ROW if args.scan == "row" else ccl.SCAN_PAIR
    ccl.reserve(ccl.workspace_bytes(S, S, args.conn, args.tile, scan) * (2 if gray else 1))
    th, tw = ccl.tile_shape(args.tile, args.conn, scan, gray)

    def step(kout=None):
        if gray:
            ccl.label_gray(img, args.conn, out=out, tile=args.tile, num_components=kout, level=level)
        else:
            ccl.label(img, args.conn, out=out, tile=args.tile, num_components=kout, level=level, scan=scan)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ccl.profile(True)
    ccl.profile_read()
    # one event before every step and one after the last, all on the stream
    # the library runs on (torch's current stream): per-step times without a
    # host synchronisation inside the timed region
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks[0].record()
    for i in range(args.steps):
        step(kdev)
        marks[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ccl.profile(False)
    phases, ncalls = ccl.profile_read()
    step_ms = [marks[i].elapsed_time(marks[i + 1]) for i in range(args.steps)]
    ms_step = statistics.median(step_ms)
    ms_mean = marks[0].elapsed_time(marks[-1]) / args.steps
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    px = S * S
    gpx = px / (ms_step * 1e-3) / 1e9
    phase_ms = {k: v / max(ncalls, 1) for k, v in phases.items()}
    dom = max(PHASE_BYTES_PER_PX, key=lambda k: phase_ms[k])
    dom_ms = phase_ms[dom]
    alg_bytes = PHASE_BYTES_PER_PX[dom] * px
    achieved = alg_bytes / (dom_ms * 1e-3) / 1e9
    workload_key = {"bernoulli": f"bernoulli{args.p}", "grf": f"grf{args.sigma}_{args.q}",
                    "gray": f"gray{args.sigma}_level{level}" + (f"_bins{args.gray_bins}" if gray else "")}[args.content] + \
        f"_{S}x{S}_conn{args.conn}_tile{th}x{tw}" + (f"_pitch{stride}" if stride != S else "") + \
        ("_scanrow" if args.scan == "row" else "")
    counters = load_counters(dom, workload_key)
    traffic = counters.get("hbm_bytes_per_launch")

    record = {
        "metric": METRIC,
        "value": round(gpx, 3),
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_mean": round(ms_mean, 4),
        "ms_per_step_min_max": [round(min(step_ms), 4), round(max(step_ms), 4)],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": f"{S}x{S} uint8 {content}, {args.conn}-connectivity, canonical int32 labels"
                        + (f", foreground iff byte > {level}" if level else ""),
            "H": S, "W": S, "stride": stride, "conn": args.conn, "tile": [th, tw], "parallelism": "single GPU",
            "level": level, "scan": args.scan, "gray_levels": gray,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": int(alg_bytes),
            "kernel_ms": round(dom_ms, 4),
            # a kernel limited by VALU issue rather than HBM (the tile scan on
            # dense noise) shows it here: the share of cycles in which a CU
            # issued a VALU instruction, and the share of active lanes in
            # those instructions (rocprofv3 SQ counters; null when absent)
            "valu_busy": counters.get("valu_busy"),
            "lane_use": counters.get("lane_use"),
        },
        "path_roofline_frac": round(BYTES_PER_PX * px / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "phase_ms": {k: round(v, 4) for k, v in phase_ms.items()},
        "wall_s_timed": round(wall, 4),
        "num_components": int(kdev.item()),
    }

    if args.cpu_runs > 0 or not args.no_verify:
        import numpy as np

        import oracle
        host = img.cpu().numpy()  # H x W view (row pitch dropped on copy)
        if level and not gray:
            host = oracle.binarize(host, level)
        if level and gray:
            host = np.where(host > level, host, 0).astype(np.uint8)
        label_fn = oracle.gray if gray else oracle.cclremsp
        times, ref = [], None
        for _ in range(max(args.cpu_runs, 1)):
            t = time.perf_counter()
            ref, kref = label_fn(host, args.conn)
            times.append(time.perf_counter() - t)
        if args.cpu_runs > 0:
            med = statistics.median(times)
            cpu = host_cpu_model()
            record["cpu_baseline"] = {
                "value": round(px / med / 1e9, 4),
                "unit": "Gpixel/s",
                "cores": 1,
                "kind": "oracle",
                "cpu_model": cpu,
                "host_threads": os.cpu_count(),
                "sample": f"the full {S}x{S} image, single-threaded C "
                          f"{'gray-level two-pass labeling' if gray else 'CCLRemSP'}, median of {len(times)} runs "
                          f"({med:.2f} s each) on one core of {cpu}",
            }
        if not args.no_verify:
            record["bit_exact"] = bool(np.array_equal(out.cpu().numpy(), ref)) and int(kdev.item()) == kref
        threads = [int(t) for t in args.cpu_threads.split(",") if t.strip()] if not gray else []
        threads = [t for t in threads if t <= min(16, os.cpu_count() or 1)]
        if threads and args.cpu_runs > 0:
            # the paper's own parallel method on the host (PARemSP, one
            # thread per row chunk, Algorithm 8's locked boundary unions):
            # its thread-count curve, as the paper reports speedups
            curve, same = {}, True
            for t in threads:
                t0_ = time.perf_counter()
                lab_t, k_t = oracle.paremsp_threads(host, args.conn, nthreads=t)
                curve[str(t)] = round(time.perf_counter() - t0_, 3)
                same &= bool(k_t == kref and np.array_equal(lab_t, ref))
                del lab_t
                log(f"cpu paremsp {t} threads: {curve[str(t)]:.2f} s")
            record["cpu_paremsp"] = {
                "seconds": curve, "unit": "s per image",
                "speedup_vs_1_thread": {k: round(curve[str(threads[0])] / v, 2) for k, v in curve.items()}
                if threads[0] == 1 else None,
                "gpx_per_s_best": round(px / min(curve.values()) / 1e9, 4),
                "equals_oracle": same,
                "kind": "PARemSP (Algorithms 7, 8) with POSIX threads; the whole call incl. flatten, labeling "
                        "and canonical numbering, one run per thread count",
            }

    if args.ablation_steps > 0 and args.conn == 8 and not gray:
        # the paper's scan comparison (Table II) inside a tile: one-row runs
        # vs two-row runs, same image, same everything else
        other = ccl.SCAN_ROW if scan == ccl.SCAN_PAIR else ccl.SCAN_PAIR
        ccl.reserve(ccl.workspace_bytes(S, S, 8, args.tile, other))
        ccl.label(img, 8, out=out, tile=args.tile, level=level, scan=other)
        t_other = _median_ms(torch, lambda: ccl.label(img, 8, out=out, tile=args.tile, level=level, scan=other),
                             args.ablation_steps)
        t_this = _median_ms(torch, lambda: ccl.label(img, 8, out=out, tile=args.tile, level=level, scan=scan),
                            args.ablation_steps)
        pair_ms, row_ms = (t_this, t_other) if scan == ccl.SCAN_PAIR else (t_other, t_this)
        record["scan_ablation"] = {"pair_rows_ms": round(pair_ms, 4), "single_rows_ms": round(row_ms, 4),
                                   "pair_speedup": round(row_ms / pair_ms, 3)}
        log(f"scan ablation: pair {pair_ms:.3f} ms, row {row_ms:.3f} ms")
    if args.order_steps > 0 and not gray and args.scan == "pair" and not level:
        # the paper's own numbering (Algorithm 3's flatten over provisional
        # labels): same image, consecutive labels in (tile, component) order
        ccl.label_provisional(img, args.conn, out=out, tile=args.tile)
        ccl.profile(True)
        ccl.profile_read()
        t_prov = _median_ms(torch, lambda: ccl.label_provisional(img, args.conn, out=out, tile=args.tile),
                            args.order_steps)
        ccl.profile(False)
        pph, pn = ccl.profile_read()
        rec_p = {"ms_per_step": round(t_prov, 4), "gpx_per_s": round(px / (t_prov * 1e-3) / 1e9, 2),
                 "phase_ms": {k: round(v / max(pn, 1), 4) for k, v in pph.items()},
                 "canonical_ms_per_step": round(ms_step, 4)}
        if not args.no_verify:
            import numpy as np

            import oracle
            th_, tw_ = ccl.tile_shape(args.tile, args.conn)
            kp = torch.zeros(1, dtype=torch.int32, device=dev)
            ccl.label_provisional(img, args.conn, out=out, tile=args.tile, num_components=kp)
            pref, pk = oracle.provisional(img.cpu().numpy(), args.conn, th_, tw_, 2 if args.conn == 8 else 1)
            rec_p["bit_exact"] = bool(np.array_equal(out.cpu().numpy(), pref)) and int(kp.item()) == pk
        record["provisional_order"] = rec_p
        log(f"provisional order: {t_prov:.3f} ms")
    del out, img
    torch.cuda.empty_cache()
    ccl.release()
    log(f"single image done: {record['value']} Gpx/s")
    if args.batch > 0:
        log("batched")
        record["batched"] = [bench_batched(torch, args.batch, c, args.batch_reps, not args.no_verify)
                             for c in (args.conn, 12 - args.conn)]
        torch.cuda.empty_cache()
        ccl.release()
    rates = [x.strip() if x.strip() == "max" else int(x) for x in args.serve_rates.split(",") if x.strip()]
    if rates and args.serve_requests > 0:
        log("served")
        record["served"] = bench_served(torch, rates, args.serve_requests, not args.no_verify)

    print(json.dumps(record), flush=True)


if __name__ == "__main__":
    main()

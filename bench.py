"""Benchmark: exact 1-NN queries/s over 100M x 256 random walks on one MI355X.

One step = one batch of queries answered exactly through the library's C ABI
(default mode: BF16 matrix-core candidate filter with the proven margin, home
leaf of the iSAX index for the initial best-so-far, FP32 refinement, top-k with
the compensated tie guard).  Inputs are resident in HBM before timing.  Also
reported: index build seconds, queries/s of every mode, p50/p99 latency of the
serving loop, the roofline of the dominant kernel (HIP events inside the
library, on the stream it runs on), and the CPU oracle timed on a bounded
sample.  Progress goes to stderr; the result is one JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"bf16": 2500.0, "fp8": 5000.0, "f32": 157.3}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--len", type=int, default=256)
    ap.add_argument("--m", type=int, default=1000)
    ap.add_argument("--k", type=int, default=1)
    ap.add_argument("--mode", default="bf16", choices=["index", "scan", "bf16", "fp8"])
    ap.add_argument("--modes", default="index,scan,bf16,fp8", help="modes measured once each besides the timed one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-series", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample-queries", type=int, default=4)
    ap.add_argument("--serve-requests", type=int, default=3000)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="also run a plain device copy of this many bytes (3 times) to scale HBM counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (see DESIGN.md, sharding)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2009_01614_amd as isax
    import workload

    isax.lib()  # fails loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, L, m, k = args.n, args.len, args.m, args.k

    log(f"generating {n} x {L} random walks on the device")
    X = workload.random_walks(n, L, seed=20090163, device=dev)
    Q, src, sig = workload.noisy_queries(X, m, seed=20091163)
    torch.cuda.synchronize()

    # ---------------------------------------------------------------- build
    precision = 0
    for md in set(args.modes.split(",")) | {args.mode}:
        precision |= {"bf16": 1, "fp8": 2}.get(md, 0)
    log("building the index (twice; the second is timed)")
    idx = isax.Index(X, 16, 8, precision=precision)
    del idx
    torch.cuda.synchronize()
    isax.profile_enable(True)
    isax.profile_reset()
    t0 = time.perf_counter()
    idx = isax.Index(X, 16, 8, precision=precision)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    build_prof = isax.profile_read()
    t0 = time.perf_counter()
    idx_plain = isax.Index(X, 16, 8, precision=0)
    torch.cuda.synchronize()
    build_plain_s = time.perf_counter() - t0
    del idx_plain
    log(f"build {build_s:.3f} s (iSAX layout only: {build_plain_s:.3f} s)")

    # ---------------------------------------------------------------- timed steps
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ids, d = idx.query(Q, k=k, mode=args.mode, stream=stream)
    torch.cuda.synchronize()
    isax.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ids, d = idx.query(Q, k=k, mode=args.mode, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = isax.profile_read()
    hit = float((ids[:, 0].cpu().numpy() == src).mean())
    qps = m * args.steps / dt
    log(f"{args.mode}: {qps:.1f} queries/s, {dt / args.steps * 1e3:.2f} ms/step")

    dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
    avg_ms = dom["total_ms"] / max(dom["launches"], 1)
    if dom_name.startswith("filter_"):
        dt_ = dom_name.split("_")[1]
        per_launch_flop = 2.0 * L * n * m / max(dom["launches"] / args.steps, 1)
        achieved = per_launch_flop / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 1), "peak": PEAK_TFLOPS[dt_], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_TFLOPS[dt_], 4), "traffic": None, "kernel": "k_filter",
                "avg_launch_ms": round(avg_ms, 3), "algorithmic_flop_per_launch": per_launch_flop}
    elif dom_name == "brute_scan":
        per_launch_flop = 3.0 * L * n * m / max(dom["launches"] / args.steps, 1)
        achieved = per_launch_flop / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 1), "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_TFLOPS["f32"], 4), "traffic": None, "kernel": "k_brute_scan",
                "avg_launch_ms": round(avg_ms, 3), "algorithmic_flop_per_launch": per_launch_flop}
    else:
        bytes_per_launch = dom["algorithmic_bytes"] / max(dom["launches"], 1)
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None, "kernel": "k_" + dom_name,
                "avg_launch_ms": round(avg_ms, 3), "algorithmic_bytes_per_launch": bytes_per_launch}
    # HBM traffic of the dominant kernel from the committed rocprofv3 counter summary,
    # only while the profiled kernel source is unchanged
    try:
        import hashlib
        cnt = json.load(open(os.path.join(ROOT, "profiles", "hbm_counters_100Mx256_m1000.json")))
        key = "k_filter" if dom_name.startswith("filter_") else "k_" + dom_name
        srcf = {"k_filter": "filter_kernels.hip", "k_index_scan": "query_kernels.hip"}.get(key)
        if (srcf and key in cnt and n == 100_000_000 and m == 1000 and (key != "k_filter" or dom_name == "filter_bf16")):
            with open(os.path.join(ROOT, "paper_2009_01614_amd", "csrc", srcf), "rb") as fh:
                cur = hashlib.sha256(fh.read()).hexdigest()[:16]
            if cur == cnt[key]["source_sha256_16"]:
                per = cnt[key]["hbm_bytes_per_step"] / max(dom["launches"] / args.steps, 1)
                roof["traffic"] = round(per / 1e9, 3)
                roof["traffic_unit"] = "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    except (OSError, ValueError, KeyError):
        pass
    kernels = {kname: {"ms_per_step": round(v["total_ms"] / args.steps, 3), "launches": v["launches"]}
               for kname, v in sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"])}

    # ---------------------------------------------------------------- other modes, once each
    modes_qps = {}
    for md in args.modes.split(","):
        if not md:
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ids_m, _ = idx.query(Q, k=k, mode=md, stream=stream)
        torch.cuda.synchronize()
        modes_qps[md] = round(m / (time.perf_counter() - t0), 1)
        assert torch.equal(ids_m, ids), f"mode {md} disagrees with {args.mode}"
        log(f"mode {md}: {modes_qps[md]} queries/s")

    # ---------------------------------------------------------------- serving latency
    serving = None
    if not args.no_serving and args.serve_requests > 0:
        rate = 0.5 * qps
        log(f"serving {args.serve_requests} Poisson arrivals at {rate:.0f}/s")
        srv = isax.Server([idx], mode=args.mode, max_batch=512, streams=4)
        Qh = Q.cpu().numpy()
        rng = np.random.default_rng(7)
        res = {}

        def producer():
            tnext = time.perf_counter()
            for i in range(args.serve_requests):
                tnext += rng.exponential(1.0 / rate)
                while time.perf_counter() < tnext:
                    time.sleep(min(1e-4, max(0.0, tnext - time.perf_counter())))
                srv.submit(0, Qh[i % m], k, i)

        th = threading.Thread(target=producer)
        ts = time.perf_counter()
        th.start()
        deadline = time.time() + 120
        while len(res) < args.serve_requests and time.time() < deadline:
            for r in srv.poll(100):
                res[r["tag"]] = r
        th.join()
        te = time.perf_counter() - ts
        srv.close()
        lat = np.array([(r["t_done"] - r["t_submit"]) * 1e3 for r in res.values()])
        bad = sum(1 for i, r in res.items() if r["ids"][0] != int(ids[i % m, 0]))
        serving = {"requests": len(res), "offered_rate": round(rate, 1), "qps": round(len(res) / te, 1),
                   "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                   "mean_batch": round(float(np.mean([r["batch_size"] for r in res.values()])), 1),
                   "mismatches": bad}
        log(f"serving: {serving}")

    # ---------------------------------------------------------------- CPU oracle on a bounded sample
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import knn_ref
        ns = min(args.cpu_sample_series, n)
        mq = min(args.cpu_sample_queries, m)
        log(f"oracle: {mq} queries x first {ns} series on the host")
        Xs = X[:ns].cpu().numpy()
        Qs = Q[:mq].cpu().numpy()
        threads = knn_ref.num_threads()
        t0 = time.perf_counter()
        st = knn_ref.KnnState(Qs, k)
        st.merge(Xs, 0)
        tc = time.perf_counter() - t0
        cpu_qps = mq / tc * (ns / n)
        cpu = {"value": round(cpu_qps, 4), "unit": "queries/s", "cores": threads, "kind": "oracle",
               "sample": f"{mq} queries x first {ns} of {n} series (FP64 brute force, {tc:.1f} s), "
                         f"scaled by {ns}/{n}"}
        log(f"oracle: {cpu}")
        del Xs

    if args.calibrate_copy:
        src_t = torch.ones(args.calibrate_copy // 4, dtype=torch.float32, device=dev)
        dst_t = torch.empty_like(src_t)
        for _ in range(3):
            dst_t.copy_(src_t)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calibrate_copy} bytes done (3 launches)")
        del src_t, dst_t

    out = {
        "metric": "exact 1-NN queries/s @100M x 256", "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.mode if args.mode in ("bf16", "fp8") else "f32",
        "data": "synthetic",
        "config": {"workload": f"{n} x {L} z-normalised FP32 random walks, 16 segments, 8-bit iSAX; {m} noisy-copy "
                               f"queries (sigma 0.01/0.1/1), exact k={k}",
                   "mode": args.mode, "refine_dtype": "f32", "source_hit_rate": hit},
        "build_s": round(build_s, 4), "build_isax_only_s": round(build_plain_s, 4),
        "build_kernels_ms": {kk: round(v["total_ms"], 3) for kk, v in build_prof.items()},
        "modes_qps": modes_qps, "serving": serving, "kernels": kernels,
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

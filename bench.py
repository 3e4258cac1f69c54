"""Benchmark: exact 1-NN queries/s over 100M x 256 random walks on one MI355X.

One step = one batch of queries answered exactly through the library's C ABI
(default mode: hybrid.  The home leaf of the iSAX index gives each query its
initial best-so-far and one leaf pass counts the leaves within it.  Queries
with few such leaves take the iSAX rounds: leaf lists, series bounds, FP32
refinement.  The others take the BF16 matrix-core candidate filter with the
proven margin, then FP32 refinement.  Top-k uses the compensated tie guard.)  Inputs are resident in HBM before timing.  Also
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


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), for the oracle's report."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
    ap.add_argument("--mode", default="hybrid", choices=["index", "scan", "bf16", "fp8", "hybrid"])
    ap.add_argument("--modes", default="index,scan,bf16,bf16_full,fp8",
                    help="modes measured once each besides the timed one (bf16_full: BF16 filter on the full rows)")
    ap.add_argument("--no-spectral", action="store_true",
                    help="build no spectral copy: the BF16 filter (and hybrid) then read the full-length rows")
    ap.add_argument("--spectral-dim", type=int, default=0, help="coefficients of the spectral copy (0: the default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-series", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample-queries", type=int, default=128)
    ap.add_argument("--serve-requests", type=int, default=6000)
    ap.add_argument("--serve-alone", type=int, default=40, help="requests sent one at a time for batch-1 latency")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-sweep", action="store_true",
                    help="instead of the headline: serve 50M x 256 + 20M x 128 at swept Poisson rates")
    ap.add_argument("--sweep-mode", default="bf16", choices=["index", "scan", "bf16", "fp8", "hybrid"])
    ap.add_argument("--serve-mode", default="bf16", choices=["index", "scan", "bf16", "fp8", "hybrid"],
                    help="mode of the serving leg (BF16 serves mixed traffic with the lowest latency)")
    ap.add_argument("--serve-batches", action="store_true",
                    help="batch-level admission in the serving legs (default for BF16 / FP8: step level)")
    ap.add_argument("--serve-chunks", type=int, default=8, help="step level: steps per sweep of a collection")
    ap.add_argument("--serve-rows", type=int, default=512, help="step level: rows of a collection's table")
    ap.add_argument("--precision-report", action="store_true",
                    help="instead of the headline: 10M x 256, batches of 1024, modes and filter error vs FP64")
    ap.add_argument("--sigma-report", action="store_true",
                    help="instead of the headline: 100M x 256, queries split by noise level, k = 1, 10, 100")
    ap.add_argument("--next-report", action="store_true",
                    help="instead of the headline: DTW on the index, raw data in pinned host memory, embeddings")
    ap.add_argument("--next-n", type=int, default=10_000_000, help="collection size of the next-rows report")
    ap.add_argument("--host-report", action="store_true",
                    help="instead of the headline: a collection in pinned host memory larger than HBM holds "
                         "with its BF16 copy (--host-n series of 256 points)")
    ap.add_argument("--host-n", type=int, default=60_000_000,
                    help="series of the host report (60M = 61.4 GB: the largest page-locked block the test box "
                         "granted, 80M failed)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="also run a plain device copy of this many bytes (3 times) to scale HBM counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; a sharded design is described "
              "with the rest of the design notes",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2009_01614_amd as isax
    import workload

    isax.lib()  # fails loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.serving_sweep:
        return serving_sweep(args, dev)
    if args.next_report:
        return next_report(args, dev)
    if args.host_report:
        return host_report(args, dev)
    if args.sigma_report:
        return sigma_report(args, dev)
    if args.precision_report:
        return precision_report(args, dev)
    n, L, m, k = args.n, args.len, args.m, args.k

    log(f"generating {n} x {L} random walks on the device")
    X = workload.random_walks(n, L, seed=20090163, device=dev)
    Q, src, sig = workload.noisy_queries(X, m, seed=20091163)
    torch.cuda.synchronize()

    # ---------------------------------------------------------------- build
    # the BF16 filter (and hybrid mode) read the spectral copy unless --no-spectral; bf16_full reads the rows
    bf16_bits = isax.PREC_BF16 if args.no_spectral else isax.PREC_SPECTRAL
    bits = {"bf16": bf16_bits, "fp8": isax.PREC_FP8, "hybrid": bf16_bits, "bf16_full": isax.PREC_BF16}
    precision = 0
    for md in set(args.modes.split(",")) | {args.mode}:
        precision |= bits.get(md, 0)
    precision |= bits.get(args.serve_mode, 0) if not args.no_serving else 0
    sdim = args.spectral_dim if precision & isax.PREC_SPECTRAL else 0
    log("building the index (twice; the second is timed)")
    idx = isax.Index(X, 16, 8, precision=precision, spectral_dim=sdim)
    del idx
    torch.cuda.synchronize()
    isax.profile_enable(True)
    isax.profile_reset()
    t0 = time.perf_counter()
    idx = isax.Index(X, 16, 8, precision=precision, spectral_dim=sdim)
    spec_dim = idx.info()["spectral_dim"]
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

    # queries the filter answers: all of them, or under hybrid those the planner hands to it
    m_filter, split = m, None
    if args.mode == "hybrid":
        _, _, st = idx.query(Q, k=k, mode="hybrid", stream=stream, stats=True)
        m_filter = sum(1 for x in st if x["path"] == isax.MODE_BF16)
        split = {"index": m - m_filter, "bf16": m_filter}
        log(f"hybrid split: {split}")
    dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
    avg_ms = dom["total_ms"] / max(dom["launches"], 1)
    if dom_name.startswith("filter_"):
        dt_ = dom_name.split("_")[1]
        # 2 flops per coefficient of the copy the filter reads, per (query, series) pair
        fdim = spec_dim if (dt_ == "bf16" and spec_dim) else L
        per_launch_flop = 2.0 * fdim * n * m_filter / max(dom["launches"] / args.steps, 1)
        achieved = per_launch_flop / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 1), "peak": PEAK_TFLOPS[dt_], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_TFLOPS[dt_], 4), "traffic": None, "kernel": "k_filter",
                "avg_launch_ms": round(avg_ms, 3), "algorithmic_flop_per_launch": per_launch_flop,
                "flop_per_pair": 2 * fdim}
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
        kname = "k_filter" if dom_name.startswith("filter_") else "k_" + dom_name
        srcf = {"k_filter": "filter_kernels.hip", "k_index_scan": "query_kernels.hip"}.get(kname)
        key = f"{kname}@{args.mode}"  # counters of this kernel in this query mode
        if (srcf and key in cnt and n == 100_000_000 and m == 1000 and k == 1
                and (kname != "k_filter" or dom_name == "filter_bf16")):
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
        if md == "bf16_full":
            ids_m, _ = idx.query(Q, k=k, mode="bf16", stream=stream, flags=isax.QF_FULL_ROWS)
        else:
            ids_m, _ = idx.query(Q, k=k, mode=md, stream=stream)
        torch.cuda.synchronize()
        modes_qps[md] = round(m / (time.perf_counter() - t0), 1)
        assert torch.equal(ids_m, ids), f"mode {md} disagrees with {args.mode}"
        log(f"mode {md}: {modes_qps[md]} queries/s")

    # ---------------------------------------------------------------- serving latency
    serving = None
    if not args.no_serving and args.serve_requests > 0:
        # half of the serving mode's batch throughput (measured above when it is not the timed mode)
        rate = 0.5 * (qps if args.serve_mode == args.mode else modes_qps.get(args.serve_mode, qps))
        log(f"serving {args.serve_requests} Poisson arrivals at {rate:.0f}/s")
        step = args.serve_mode in ("bf16", "fp8") and not args.serve_batches
        srv = isax.Server([idx], mode=args.serve_mode, max_batch=args.serve_rows if step else 512, streams=4,
                          batches=args.serve_batches, chunks=args.serve_chunks)
        Qh = Q.cpu().numpy()
        rng = np.random.default_rng(7)
        # batch-1 latency: one request at a time on the idle server
        one = []
        for i in range(args.serve_alone + 1):
            t0 = time.perf_counter()
            srv.submit(0, Qh[i % m], k, 10 ** 9 + i)
            got = []
            while not got:
                got = srv.poll(100)
            if i:
                one.append((got[0]["t_done"] - got[0]["t_submit"]) * 1e3)
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
        offered_real, achieved = _serve_rates(res)
        serving = {"mode": args.serve_mode, "admission": "step" if step else "batch",
                   "requests": len(res), "offered_rate": round(rate, 1), "offered_realised": round(offered_real, 1),
                   "qps": round(achieved, 1), "qps_incl_drain": round(len(res) / te, 1),
                   "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                   "mean_batch": round(float(np.mean([r["batch_size"] for r in res.values()])), 1),
                   "mismatches": bad,
                   "batch1_p50_ms": round(float(np.percentile(one, 50)), 3) if one else None,
                   "batch1_p99_ms": round(float(np.percentile(one, 99)), 3) if one else None}
        if step:
            serving["chunks"] = args.serve_chunks
            serving["rows"] = args.serve_rows
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
               "cpu_model": cpu_model(),
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
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"bf16": "bf16", "fp8": "fp8", "hybrid": "bf16"}.get(args.mode, "f32"),
        "data": "synthetic",
        "config": {"workload": f"{n} x {L} z-normalised FP32 random walks, 16 segments, 8-bit iSAX; {m} noisy-copy "
                               f"queries (sigma 0.01/0.1/1), exact k={k}",
                   "mode": args.mode, "refine_dtype": "f32", "source_hit_rate": hit, "hybrid_split": split,
                   "filter_copy": f"spectral, {spec_dim} of {L} coefficients" if spec_dim else "full rows"},
        "build_s": round(build_s, 4), "build_isax_only_s": round(build_plain_s, 4),
        "build_kernels_ms": {kk: round(v["total_ms"], 3) for kk, v in build_prof.items()},
        "modes_qps": modes_qps, "serving": serving, "kernels": kernels,
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _serve_rates(res):
    """(offered, achieved) queries/s of a run, on the library's clock: requests between the
    first and the last submission, and completions between the first and the last answer.
    A stable server completes at the rate requests arrive; dividing the count by the whole
    run instead would also count the drain of the last requests against it."""
    ts = sorted(r["t_submit"] for r in res.values())
    td = sorted(r["t_done"] for r in res.values())
    n = len(ts)
    if n < 2:
        return float("nan"), float("nan")
    return (n - 1) / max(ts[-1] - ts[0], 1e-9), (n - 1) / max(td[-1] - td[0], 1e-9)


def _serve_run(isax, srv, reqs, rate, rng, max_wait_s=120.0):
    """Submit reqs [(collection, host query, k)] at Poisson rate; return results by tag and wall time."""
    res = {}

    def producer():
        tnext = time.perf_counter()
        for i, (c, q, kk) in enumerate(reqs):
            tnext += rng.exponential(1.0 / rate) if rate > 0 else 0.0
            while time.perf_counter() < tnext:
                time.sleep(min(1e-4, max(0.0, tnext - time.perf_counter())))
            srv.submit(c, q, kk, i)

    th = threading.Thread(target=producer)
    t0 = time.perf_counter()
    th.start()
    deadline = time.time() + max_wait_s
    while len(res) < len(reqs) and time.time() < deadline:
        for r in srv.poll(50):
            res[r["tag"]] = r
    th.join()
    return res, time.perf_counter() - t0


def serving_sweep(args, dev):
    """Serving configuration: two resident collections, Poisson arrivals at swept rates.

    Collections 50M x 256 and 20M x 128 (z-normalised random walks); requests go
    50/50 to the collections, k uniform over {1, 10, 100}, noisy copies with sigma
    uniform over {0.01, 0.1, 1}.  Saturation is measured with a burst; each rate
    then runs a Poisson stream.  A sample of every rate's results is compared with
    the same queries run alone (ids equal, distances bit-identical).
    """
    import numpy as np
    import torch

    import paper_2009_01614_amd as isax
    import workload

    mode = args.sweep_mode
    log("generating 50M x 256 and 20M x 128")
    cols = [workload.random_walks(50_000_000, 256, seed=20090165, device=dev),
            workload.random_walks(20_000_000, 128, seed=20090166, device=dev)]

    def prec(L):
        # the spectral copy where three quarters of the padded length leave coefficients out (len 256: 192)
        bf16_bits = isax.PREC_BF16 if args.no_spectral or L < 256 else isax.PREC_SPECTRAL
        return {"bf16": bf16_bits, "fp8": isax.PREC_FP8, "hybrid": bf16_bits}.get(mode, 0)
    idx = [isax.Index(X, 16, 8, precision=prec(X.shape[1])) for X in cols]
    rng = np.random.default_rng(20091165)
    pools = []
    for ci, X in enumerate(cols):
        qs = []
        for sgm in (0.01, 0.1, 1.0):
            q, _, _ = workload.noisy_queries(X, 700, seed=20091165 + ci * 10 + int(sgm * 100), sigmas=(sgm,))
            qs.append(q.cpu().numpy())
        pools.append(np.concatenate(qs))

    def make_reqs(count):
        out = []
        for _ in range(count):
            c = int(rng.integers(2))
            out.append((c, pools[c][int(rng.integers(len(pools[c])))], int(rng.choice([1, 10, 100]))))
        return out

    step = mode in ("bf16", "fp8") and not args.serve_batches
    srv = isax.Server(idx, mode=mode, max_batch=args.serve_rows if step else 512, streams=4,
                      batches=args.serve_batches, chunks=args.serve_chunks)
    _serve_run(isax, srv, make_reqs(512), 0.0, rng)          # warm-up
    burst = make_reqs(4096)
    res, wall = _serve_run(isax, srv, burst, 0.0, rng)
    sat = len(res) / wall
    log(f"saturation {sat:.0f} queries/s (burst of {len(burst)})")
    points = []
    for frac in (0.1, 0.25, 0.5, 0.75, 1.0, 1.2):
        rate = frac * sat
        count = int(min(6000, max(300, rate * 3.0)))
        reqs = make_reqs(count)
        res, wall = _serve_run(isax, srv, reqs, rate, rng)
        lat = np.array([(r["t_done"] - r["t_submit"]) * 1e3 for r in res.values()])
        # alone vs mix on a sample
        bad = 0
        for tag in list(res)[:: max(1, len(res) // 40)]:
            c, q, kk = reqs[tag]
            ids1, d1 = idx[c].query(torch.from_numpy(q[None]).to(dev), k=kk, mode=mode)
            r = res[tag]
            bad += int(r["ids"] != ids1[0].tolist() or
                       not np.array_equal(np.array(r["dists"], np.float32), d1[0].cpu().numpy()))
        offered_real, achieved = _serve_rates(res)
        pt = {"offered_frac": frac, "offered_qps": round(rate, 1), "offered_realised": round(offered_real, 1),
              "requests": len(res), "achieved_qps": round(achieved, 1),
              "achieved_incl_drain": round(len(res) / wall, 1), "p50_ms": round(float(np.percentile(lat, 50)), 2),
              "p99_ms": round(float(np.percentile(lat, 99)), 2),
              "mean_batch": round(float(np.mean([r["batch_size"] for r in res.values()])), 1),
              "alone_vs_mix_mismatches": bad}
        log(f"rate {frac:.2f} x sat: {pt}")
        points.append(pt)
        last = (reqs, res)
    srv.close()
    # the FP64 oracle on a sample of the last rate's requests, streamed over each collection
    from oracle import knn_ref
    reqs, res = last
    oracle_bad, oracle_n = 0, 0
    for c, X in enumerate(cols):
        tags = [t for t in sorted(res) if reqs[t][0] == c][:: 25][:24]
        if not tags:
            continue
        kk = max(reqs[t][2] for t in tags)
        st = knn_ref.KnnState(np.stack([reqs[t][1] for t in tags]).astype(np.float32), kk)
        for a in range(0, X.shape[0], 5_000_000):
            st.merge(X[a:a + 5_000_000].cpu().numpy(), a)
        for j, t in enumerate(tags):
            kq = reqs[t][2]
            r = res[t]
            ok = r["ids"] == st.ids[j, :kq].tolist() and np.allclose(r["dists"], np.sqrt(st.d2[j, :kq]), rtol=1e-4,
                                                                       atol=0)
            oracle_bad += int(not ok)
            oracle_n += 1
        log(f"oracle sample of collection {c}: {len(tags)} requests checked")
    admission = (f"step level: {args.serve_rows} rows per collection, {args.serve_chunks} steps per sweep"
                 if step else "batch level: dynamic batching (max 512), 4 streams, 4 GiB scratch budget")
    print(json.dumps({"metric": "serving p50/p99 latency and queries/s", "mode": mode,
                      "config": {"workload": "50M x 256 + 20M x 128 random walks resident; Poisson arrivals; "
                                             "k in {1,10,100}; sigma in {0.01,0.1,1}; " + admission},
                      "saturation_qps": round(sat, 1), "sweep": points,
                      "oracle_sample": {"requests": oracle_n, "mismatches": oracle_bad}}), flush=True)


def precision_report(args, dev):
    """Precision configuration: 10M x 256, 4 batches of 1024 queries, k = 1 and 10.

    Reports queries/s of every mode (all exact, ids compared) and, for sampled
    queries, the reduced-precision filter's error against plain FP64 distances:
    max |ED^2 - approx| / M (<= 1 by the proof), mean margin M and the fraction
    of series the filter keeps at the final bound.
    """
    import numpy as np
    import torch

    import paper_2009_01614_amd as isax
    import workload

    n, L = 10_000_000, 256
    log("generating 10M x 256")
    X = workload.random_walks(n, L, seed=20090162, device=dev)
    Q, _, _ = workload.noisy_queries(X, 4096, seed=20091164)
    # BF16 on the spectral copy (mode bf16) and on the full rows (bf16_full), FP8
    idx = isax.Index(X, 16, 8, precision=isax.PREC_BF16 | isax.PREC_FP8 | isax.PREC_SPECTRAL)
    out = {"metric": "exact k-NN queries/s by mode; filter error vs FP64", "config": {
        "workload": "10M x 256 random walks, 4 batches of 1024 noisy queries (sigma 0.01/0.1/1)",
        "spectral_dim": idx.info()["spectral_dim"]}, "qps": {}, "split": {}}
    for k in (1, 10):
        ref = None
        for mode in ("bf16", "bf16_full", "fp8", "index", "scan"):
            kw = {"mode": "bf16", "flags": isax.QF_FULL_ROWS} if mode == "bf16_full" else {"mode": mode}
            idx.query(Q[:1024].contiguous(), k=k, **kw)
            torch.cuda.synchronize()
            isax.profile_reset()
            isax.profile_enable(True)
            t0 = time.perf_counter()
            ids = [idx.query(Q[b:b + 1024].contiguous(), k=k, batch=1024, **kw)[0] for b in range(0, 4096, 1024)]
            torch.cuda.synchronize()
            out["qps"][f"{mode}_k{k}"] = round(4096 / (time.perf_counter() - t0), 1)
            prof = isax.profile_read()
            isax.profile_enable(False)
            if mode in ("bf16", "bf16_full", "fp8"):
                # where a filter batch's time goes, and how many series it refines per query
                _, _, st = idx.query(Q[:1024].contiguous(), k=k, stats=True, **kw)
                fk = "filter_fp8" if mode == "fp8" else "filter_bf16"
                out["split"][f"{mode}_k{k}"] = {
                    "filter_ms_per_batch": round(prof.get(fk, {}).get("total_ms", 0.0) / 4, 2),
                    "refine_ms_per_batch": round(prof.get("refine_filtered", {}).get("total_ms", 0.0) / 4, 2),
                    "refined_per_query": round(float(np.mean([x["series_refined"] for x in st])), 1),
                    "kept_fraction": float(np.mean([x["series_refined"] for x in st])) / n,
                    "full_rows_switches": int(prof.get("filter_full_rows_switch", {}).get("algorithmic_bytes", 0))}
            ids = torch.cat(ids)
            if ref is None:
                ref = ids
            assert torch.equal(ids, ref), f"{mode} disagrees"
            log(f"k={k} {mode}: {out['qps'][f'{mode}_k{k}']} queries/s {out['split'].get(f'{mode}_k{k}', '')}")
    del idx
    torch.cuda.empty_cache()
    # scores of the full rows and of FP8 (an index without the spectral copy), then of the spectral copy
    idx = isax.Index(X, 16, 8, precision=isax.PREC_BF16 | isax.PREC_FP8)
    log("filter error vs FP64 on 4 sampled queries")
    sample = Q[[0, 1, 2, 3]].contiguous()
    # the bound check: plain FP64 squared distances (PyTorch on the device, in chunks)
    d64 = np.empty((4, n), np.float64)
    q64 = sample.double()
    for c0 in range(0, n, 1 << 20):
        xc = X[c0:c0 + (1 << 20)].double()
        for j in range(4):
            d64[j, c0:c0 + xc.shape[0]] = ((xc - q64[j]) ** 2).sum(dim=1).cpu().numpy()
        del xc
    for mode in ("bf16", "fp8"):
        ap, mg = (t.cpu().numpy().astype(np.float64) for t in idx.filter_scores(sample, mode))
        err = np.abs(d64 - ap)
        tau = np.sort(d64, axis=1)[:, 0:1]
        out[f"filter_{mode}"] = {"max_err_over_margin": float((err / mg).max()), "mean_margin": float(mg.mean()),
                                 "mean_abs_err": float(err.mean()),
                                 "kept_fraction_at_final_bound_k1": float(((ap - mg) <= tau).mean())}
        log(f"{mode}: {out[f'filter_{mode}']}")
    del idx
    torch.cuda.empty_cache()
    # the spectral copy's scores bound ED^2 from below only (approx - M <= ED^2)
    idx = isax.Index(X, 16, 8, precision=isax.PREC_SPECTRAL)
    ap, mg = (t.cpu().numpy().astype(np.float64) for t in idx.filter_scores(sample, "bf16"))
    tau = np.sort(d64, axis=1)[:, 0:1]
    out["filter_bf16_spectral"] = {"max_lower_bound_minus_ed2": float((ap - mg - d64).max()),
                                   "mean_margin": float(mg.mean()),
                                   "mean_gap_ed2_minus_approx": float((d64 - ap).mean()),
                                   "kept_fraction_at_final_bound_k1": float(((ap - mg) <= tau).mean())}
    log(f"bf16 spectral: {out['filter_bf16_spectral']}")
    print(json.dumps(out), flush=True)


def sigma_report(args, dev):
    """Per-noise-level breakdown at the headline size: the 1000 noisy queries split by
    sigma (0.01 / 0.1 / 1), each third answered as one batch in the BF16, index and
    hybrid modes at k = 1, 10 and 100, with the index path's pruning statistics and
    the share of queries the hybrid mode keeps on the index path."""
    import numpy as np
    import torch

    import paper_2009_01614_amd as isax
    import workload

    n, L, m = args.n, args.len, args.m
    log(f"generating {n} x {L}")
    X = workload.random_walks(n, L, seed=20090163, device=dev)
    Q, src, sig = workload.noisy_queries(X, m, seed=20091163)
    prec = isax.PREC_BF16 | (0 if args.no_spectral else isax.PREC_SPECTRAL)
    idx = isax.Index(X, 16, 8, precision=prec, spectral_dim=args.spectral_dim if not args.no_spectral else 0)
    out = {"metric": "exact k-NN queries/s and pruning by query noise level",
           "config": {"workload": f"{n} x {L} random walks, {m} noisy queries split by sigma",
                      "spectral_dim": idx.info()["spectral_dim"],
                      "timing": "best of 3 calls per cell, one batch of the third of the queries"}, "by_sigma": {}}
    modes = ("bf16", "index", "hybrid") + (() if args.no_spectral else ("bf16_full",))
    for sg in (0.01, 0.1, 1.0):
        sel = torch.from_numpy(np.where(sig == sg)[0]).to(dev)
        Qs = Q[sel].contiguous()
        rec = {"queries": int(Qs.shape[0])}
        for k in (1, 10, 100):
            for mode in modes:
                kw = {"mode": "bf16", "flags": isax.QF_FULL_ROWS} if mode == "bf16_full" else {"mode": mode}
                idx.query(Qs[:8].contiguous(), k=k, **kw)
                best = float("inf")
                for _ in range(3):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    res = idx.query(Qs, k=k, **kw)
                    torch.cuda.synchronize()
                    best = min(best, time.perf_counter() - t0)
                rec[f"{mode}_k{k}_qps"] = round(Qs.shape[0] / best, 1)
                if mode in ("index", "hybrid"):
                    res = idx.query(Qs, k=k, mode=mode, stats=True)  # untimed
                if mode == "hybrid":
                    rec[f"hybrid_k{k}_index_share"] = round(
                        float(np.mean([x["path"] == isax.MODE_INDEX for x in res[2]])), 3)
                if mode == "index":
                    st = res[2]
                    rec[f"index_k{k}_leaves_kept_frac"] = round(
                        float(np.mean([x["leaves_kept"] / max(x["leaves_scanned"], 1) for x in st])), 4)
                    rec[f"index_k{k}_series_refined"] = round(float(np.mean([x["series_refined"] for x in st])), 1)
        out["by_sigma"][str(sg)] = rec
        log(f"sigma {sg}: {rec}")
    print(json.dumps(out), flush=True)


# ALU bound of the DTW recurrence: a band cell takes at least 3 VALU lane operations
# (subtract, three-way minimum, fused multiply-add); 256 CUs x 64 FP32 lanes per
# clock (no packed FP32) x 2.4 GHz = 39.3 T lane operations/s.
PEAK_VALU_OPS = 256 * 64 * 2.4e9
DTW_OPS_PER_CELL = 3


def host_report(args, dev):
    """Raw rows in pinned host memory (the paper's plan for data larger than GPU memory, Sec. V).

    n x 256 random walks are drawn on the device chunk by chunk into page-locked host
    memory (isax_host_alloc); the index keeps the iSAX layout and the full-row BF16 copy in
    HBM (the refinement precheck reads that copy and crosses the bus only for rows that can
    matter).  1000 noisy queries, k = 1 and 10, index / BF16 / hybrid modes (answers equal
    across modes); 4 queries checked exactly against the C oracle streamed over the rows;
    then the same collection in HBM for comparison where it fits.
    """
    import numpy as np
    import torch

    import paper_2009_01614_amd as isax
    import workload
    from oracle import knn_ref

    n, L = args.host_n, 256
    log(f"allocating {n} x {L} pinned host rows ({n * L * 4 / 1e9:.1f} GB)")
    rows = isax.HostRows(n, L)  # exactly n x L x 4 bytes of page-locked memory
    Xh = rows.tensor
    t0 = time.perf_counter()
    workload.random_walks(n, L, seed=20090167, device=dev, out=Xh)
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    Q, src, sig = workload.noisy_queries(Xh, 1000, seed=20091167)
    Q = Q.to(dev).contiguous()
    _, hbm = torch.cuda.mem_get_info()
    t0 = time.perf_counter()
    idx = isax.Index(Xh, 16, 8, precision=isax.PREC_BF16)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = idx.info()
    out = {"metric": "exact k-NN queries/s, rows in pinned host memory",
           "config": {"n": n, "len": L, "host_row_bytes": n * L * 4, "device_bytes": info["device_bytes"],
                      "hbm_bytes": hbm, "rows_plus_bf16_copy_fit_in_hbm": n * L * 4 + info["device_bytes"] <= hbm,
                      "workload": f"{n} x {L} random walks in pinned host memory, 1000 noisy queries"},
           "build_s": round(build_s, 2), "qps": {}, "rows_read_per_query": {}}
    log(f"built in {build_s:.1f} s; device bytes {info['device_bytes'] / 1e9:.1f} GB of {hbm / 1e9:.1f}")
    for k in (1, 10):
        ref = None
        for mode in ("index", "bf16", "hybrid"):
            idx.query(Q[:64].contiguous(), k=k, mode=mode)
            (ids, _), dt, _ = _timed_query(isax, idx, Q, k=k, mode=mode)
            ref = ids if ref is None else ref
            assert torch.equal(ids, ref), f"host rows: {mode} disagrees"
            out["qps"][f"{mode}_k{k}"] = round(1000 / dt, 1)
            _, _, st = idx.query(Q[:100].contiguous(), k=k, mode=mode, stats=True)
            out["rows_read_per_query"][f"{mode}_k{k}"] = round(float(np.mean([x["series_refined"] for x in st])), 1)
            log(f"k={k} {mode}: {out['qps'][f'{mode}_k{k}']} q/s, rows read per query "
                f"{out['rows_read_per_query'][f'{mode}_k{k}']}")
        last = ref
    # the oracle over the whole collection for 4 queries (one per noise level and a fresh one's rows)
    sample = [int(np.where(sig == sg)[0][0]) for sg in (0.01, 0.1, 1.0)] + [3]
    t0 = time.perf_counter()
    st = knn_ref.KnnState(Q[sample].cpu().numpy(), 10)
    for a in range(0, n, 10_000_000):
        st.merge(Xh[a:a + 10_000_000].numpy(), a)
    ok = bool(np.array_equal(last[sample].cpu().numpy(), st.ids))
    out["oracle_check"] = {"queries": len(sample), "k": 10, "ids_equal": ok, "seconds": round(time.perf_counter() - t0, 1)}
    log(f"oracle check: {out['oracle_check']}")
    assert ok, "host rows: answers differ from the oracle"
    idx.close()
    # the same collection in HBM, where rows and copy fit there too
    if 2 * n * L * 4 + 16 * n < hbm:
        Xd = Xh.to(dev)
        idd = isax.Index(Xd, 16, 8, precision=isax.PREC_BF16)
        out["device_qps"] = {}
        for k in (1, 10):
            for mode in ("index", "bf16", "hybrid"):
                idd.query(Q[:64].contiguous(), k=k, mode=mode)
                (ids, _), dt, _ = _timed_query(isax, idd, Q, k=k, mode=mode)
                out["device_qps"][f"{mode}_k{k}"] = round(1000 / dt, 1)
        out["host_over_device"] = {key: round(out["qps"][key] / v, 3) for key, v in out["device_qps"].items()}
        log(f"rows in HBM: {out['device_qps']}; host / device: {out['host_over_device']}")
        idd.close()
        del Xd
        torch.cuda.empty_cache()
    del Xh
    rows.close()
    print(json.dumps(out), flush=True)


def _timed_query(isax, idx, Q, **kw):
    import torch
    isax.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = idx.query(Q, **kw)
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0, isax.profile_read()


def next_report(args, dev):
    """Next rows, each exact (answers compared across modes; the DTW CPU baseline's answer too).

    DTW: n x 256 random walks, Sakoe-Chiba half-width 25 (10 %), 100 noisy
    queries, k = 1 and 10, index and plain-scan modes; DTW cells/s against the
    ALU bound.  Host-resident raw data: the same collection in pinned host
    memory (summaries, layout and the BF16 copy in HBM), 1000 queries, index and
    BF16 modes.  Embeddings: n x 128 and n x 384 clustered vectors, 1000 queries;
    16 segments with the standard-normal edges, and dim / 8 segments with the
    collection's own (empirical) edges; then the same vectors at unit norm, dim / 8
    segments, standard-normal against empirical edges (index mode).
    """
    import numpy as np
    import torch

    import paper_2009_01614_amd as isax
    import workload
    from oracle import knn_ref

    n, L, r = args.next_n, 256, 25
    out = {"metric": "exact k-NN queries/s, next rows", "config": {"n": n}, "dtw": {}, "host_resident": {},
           "embeddings": {}}
    isax.profile_enable(True)
    log(f"generating {n} x {L}")
    X = workload.random_walks(n, L, seed=20090165, device=dev)
    Q100, _, _ = workload.noisy_queries(X, 100, seed=20091165)
    # BF16 copy for the host-resident section; FP32 rows in leaf order for the DTW section
    idx = isax.Index(X, 16, 8, precision=5)
    # ---- DTW
    res = {}
    for k in (1, 10):
        for mode in ("index", "scan"):
            idx.query(Q100[:8].contiguous(), k=k, mode=mode, metric="dtw", window=r)
            (ids, d, st), dt, prof = _timed_query(isax, idx, Q100, k=k, mode=mode, metric="dtw", window=r, stats=True)
            cells = sum(s_["dtw_cells"] for s_ in st)
            kern_ms = prof.get("dtw_scan", {}).get("total_ms", 0.0) + prof.get("homeleaf", {}).get("total_ms", 0.0)
            cps = cells / (kern_ms / 1e3) if kern_ms > 0 else 0.0
            res[(k, mode)] = ids
            out["dtw"][f"{mode}_k{k}"] = {
                "qps": round(100 / dt, 2), "dtw_series_per_query": round(sum(s_["dtw_series"] for s_ in st) / 100),
                "lb_keogh_per_query": round(sum(s_["series_refined"] for s_ in st) / 100),
                "cells_per_s": cps, "alu_frac": cps * DTW_OPS_PER_CELL / PEAK_VALU_OPS}
            log(f"dtw k={k} {mode}: {out['dtw'][f'{mode}_k{k}']}")
        assert torch.equal(res[(k, "index")], res[(k, "scan")]), "DTW index and scan disagree"
    log("DTW CPU baseline: the oracle on 1 query (all host threads)")
    Xh = X.cpu().numpy()
    t0 = time.perf_counter()
    ref_ids, _ = knn_ref.knn_dtw_c(Xh, Q100[:1].cpu().numpy(), 10, r)
    cpu_s = time.perf_counter() - t0
    assert np.array_equal(res[(10, "index")][:1].cpu().numpy(), ref_ids), "DTW differs from the oracle"
    out["dtw"]["config"] = {"workload": f"{n} x {L} random walks, window {r}, 100 noisy queries",
                            "rows": "FP32 copy in leaf order"}
    out["dtw"]["roofline"] = {"bound": "alu", "peak_cells_per_s": PEAK_VALU_OPS / DTW_OPS_PER_CELL,
                              "ops_per_cell": DTW_OPS_PER_CELL}
    out["dtw"]["cpu_baseline"] = {"value": round(1 / cpu_s, 4), "unit": "queries/s", "cores": knn_ref.num_threads(),
                                  "cpu_model": cpu_model(),
                                  "kind": "oracle", "sample": "1 query against the whole collection, k = 10"}
    # ---- raw data in pinned host memory (compared with the same build, data in HBM)
    idx.close()
    idx = isax.Index(X, 16, 8, precision=1)
    Q = workload.noisy_queries(X, 1000, seed=20091166)[0]
    dev_ids = {}
    for mode in ("index", "bf16"):
        idx.query(Q[:64].contiguous(), k=1, mode=mode)
        (ids, _), dt, _ = _timed_query(isax, idx, Q, k=1, mode=mode)
        dev_ids[mode] = ids
        out["host_resident"][f"device_{mode}_qps"] = round(1000 / dt, 1)
    idx.close()
    Xp = torch.empty(X.shape, dtype=torch.float32, pin_memory=True)
    Xp.copy_(X)
    del X
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    idx_h = isax.Index(Xp, 16, 8, precision=1)
    torch.cuda.synchronize()
    out["host_resident"]["build_s"] = round(time.perf_counter() - t0, 3)
    for mode in ("index", "bf16"):
        idx_h.query(Q[:64].contiguous(), k=1, mode=mode)
        (ids, _), dt, _ = _timed_query(isax, idx_h, Q, k=1, mode=mode)
        assert torch.equal(ids, dev_ids[mode]), f"host-resident {mode} differs"
        out["host_resident"][f"host_{mode}_qps"] = round(1000 / dt, 1)
        log(f"host-resident {mode}: {out['host_resident'][f'host_{mode}_qps']} q/s")
    out["host_resident"]["device_bytes"] = idx_h.info()["device_bytes"]
    idx_h.close()
    del Xp
    # ---- embeddings
    for dim in (128, 384):
        g = torch.Generator(device=dev).manual_seed(dim)
        centres = torch.randn(1000, dim, device=dev, generator=g) * 3.0
        E = torch.empty((n, dim), dtype=torch.float32, device=dev)
        for c0 in range(0, n, 1 << 22):
            c1 = min(n, c0 + (1 << 22))
            lab = torch.randint(0, 1000, (c1 - c0,), device=dev, generator=g)
            E[c0:c1] = centres[lab] + torch.randn(c1 - c0, dim, device=dev, generator=g) * 0.7
        QE = (centres[torch.randint(0, 1000, (1000,), device=dev, generator=g)] +
              torch.randn(1000, dim, device=dev, generator=g) * 0.7).contiguous()
        ie = isax.Index(E, 16, 8, precision=1)
        ref = None
        for mode in ("bf16", "index", "scan"):
            ie.query(QE[:64].contiguous(), k=10, mode=mode)
            (ids, _), dt, _ = _timed_query(isax, ie, QE, k=10, mode=mode)
            ref = ids if ref is None else ref
            assert torch.equal(ids, ref), f"embeddings {mode} disagrees"
            out["embeddings"][f"d{dim}_{mode}_k10_qps"] = round(1000 / dt, 1)
            log(f"embeddings d={dim} {mode}: {out['embeddings'][f'd{dim}_{mode}_k10_qps']} q/s")
        _, _, st = ie.query(QE[:100].contiguous(), k=10, mode="index", stats=True)
        out["embeddings"][f"d{dim}_w16_normal_refined_per_query"] = round(sum(x["series_refined"] for x in st) / 100)
        ie.close()
        # dim / 8 segments with the collection's own region edges
        w = dim // 8
        ie = isax.Index(E, w, 8, precision=1, edges="empirical")
        for mode in ("index", "hybrid"):
            ie.query(QE[:64].contiguous(), k=10, mode=mode)
            (ids, _), dt, _ = _timed_query(isax, ie, QE, k=10, mode=mode)
            assert torch.equal(ids, ref), f"embeddings {mode} (w={w}, empirical edges) disagrees"
            out["embeddings"][f"d{dim}_w{w}_empirical_{mode}_k10_qps"] = round(1000 / dt, 1)
            log(f"embeddings d={dim} w={w} empirical {mode}: {round(1000 / dt, 1)} q/s")
        _, _, st = ie.query(QE[:100].contiguous(), k=10, mode="index", stats=True)
        out["embeddings"][f"d{dim}_w{w}_empirical_refined_per_query"] = round(
            sum(x["series_refined"] for x in st) / 100)
        ie.close()
        # the same vectors scaled to unit norm (their segment means sit near 0, far narrower
        # than N(0, 1)): dim / 8 segments, standard-normal against empirical edges
        E /= E.norm(dim=1, keepdim=True)
        QE /= QE.norm(dim=1, keepdim=True)
        ref = None
        for edges in ("normal", "empirical"):
            ie = isax.Index(E, w, 8, precision=1, edges=edges)
            ie.query(QE[:64].contiguous(), k=10, mode="index")
            (ids, _), dt, _ = _timed_query(isax, ie, QE, k=10, mode="index")
            ref = ids if ref is None else ref
            assert torch.equal(ids, ref), f"unit embeddings ({edges} edges) disagree"
            _, _, st = ie.query(QE[:100].contiguous(), k=10, mode="index", stats=True)
            out["embeddings"][f"unit_d{dim}_w{w}_{edges}_index_k10_qps"] = round(1000 / dt, 1)
            out["embeddings"][f"unit_d{dim}_w{w}_{edges}_refined_per_query"] = round(
                sum(x["series_refined"] for x in st) / 100)
            log(f"unit embeddings d={dim} w={w} {edges}: {round(1000 / dt, 1)} q/s")
            ie.close()
        del E
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the Fast and Robust ICP hot path on one MI355X.

Default workload: robust point-to-point registrations (Algorithm 1, Welsch
metric, Anderson m = 5) of a 100k-point source against a 100k-point target
(bumpy sphere, 70% overlap, 10% outliers, noise 2e-3 diag, rotation <= 45
deg; nu from 3 x median down to 1e-3 diag; cluster-pruned exact closest
point), eight seeded pairs taken in turn (the number of passes an Anderson-
accelerated registration takes varies from pair to pair). A step is one full
registration from T0 = I to the returned transform with the inputs already
resident in HBM. Reported: registrations/s of the
device-resident graph engine, the same for the plain host-synchronised loop
(same kernels, one sync per pass), closest-point queries/s, p50/p99 latency,
final RMSE of both loops, the dominant kernel's roofline position and the CPU
oracle on a bounded sample.

Usage: python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
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

FP32_PEAK_TFLOPS = 157.3  # MI355X vector FP32 (packed FMA), published
FLOPS_PER_PAIR = 8        # 3 sub, 1 mul, 2 FMA per (source, target) distance
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "nn_traffic_robust_p2p_100k.md")
TRAFFIC_SOURCES = ["paper_2007_07627_amd/csrc/nn.hip", "paper_2007_07627_amd/csrc/icp_internal.h"]
COPY_CALIBRATION_BYTES = 256 << 20


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sources_digest():
    """sha256 over the code of the closest-point kernel sources (the counters
    in the traffic summary hold only for the code they were taken from): line
    comments, trailing blanks and empty lines are left out, so that a change
    of comments alone keeps the record valid."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            for line in f:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per closest-point launch (cull + slice of one pass) from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when it is
    missing or was taken from other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            txt = f.read()
    except OSError:
        return None, "no counter summary"
    tag = "<!-- traffic: "
    if tag not in txt:
        return None, "no counter summary"
    rec = json.loads(txt.split(tag, 1)[1].split(" -->", 1)[0])
    if rec.get("sources_sha256") != sources_digest():
        return None, "counters predate the current kernel sources"
    return float(rec["bytes_per_launch"]), "rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a plain copy"


def copy_calibration(torch):
    """A plain device copy of known size, for scaling the HBM counters of a
    rocprofv3 --pmc run (FETCH_SIZE / WRITE_SIZE in KiB per dispatch)."""
    n = COPY_CALIBRATION_BYTES // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: 4 copies of {COPY_CALIBRATION_BYTES} bytes")


def workload(name):
    from paper_2007_07627_amd import binding as B
    from paper_2007_07627_amd import synth
    if name == "robust-p2p-100k":
        ds = [synth.partial_sphere_pair(synth.rng_for(2, i)) for i in range(8)]
        prms = [B.icp_params_default(B.ICP_P2P_WELSCH, nu_min=d["nu_min"], nn=B.ICP_NN_CLUSTER) for d in ds]
        cfg = {"workload": "robust point-to-point (Algorithm 1) + Anderson m=5, bumpy sphere 70% overlap, "
                           "10% outliers, noise 2e-3 diag, rotation <= 45 deg; 8 seeded pairs in turn",
               "M": 100000, "N": 100000, "pairs": 8, "nn": "cluster", "anderson_m": 5,
               "nu": "3 x median -> 1e-3 diag", "eps": 1e-5}
        return ds, prms, cfg
    if name == "fast-icp-4096":
        d = synth.fast_icp_pair(synth.rng_for(1, 0))
        prm = B.icp_params_default(B.ICP_P2P_L2, eps=1e-6, iter_first=50, iter_cap=50, nn=B.ICP_NN_BRUTE)
        cfg = {"workload": "Fast ICP (L2 + Anderson m=5), bumpy sphere, same points, noise 1e-3 diag",
               "M": 4096, "N": 4096, "nn": "brute", "anderson_m": 5, "max_iter": 50, "eps": 1e-6}
        return [d], [prm], cfg
    if name == "robust-p2pl-500k":
        d = synth.height_field_pair(synth.rng_for(3, 0))
        prm = B.icp_params_default(B.ICP_P2PL_WELSCH, anderson_m=6, nu_min=d["nu_min"], nn=B.ICP_NN_CLUSTER)
        cfg = {"workload": "robust point-to-plane (Algorithm 2) + Anderson m=6, height field 60% overlap, "
                           "5% outliers, noise 1e-3",
               "M": 200000, "N": 500000, "nn": "cluster", "anderson_m": 6, "nu": "3 x median -> 1e-3"}
        return [d], [prm], cfg
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(d, prm, passes_per_reg, budget_s=12.0):
    """The oracle as it stands, on a bounded sample: full-size map evaluations
    (exhaustive closest point + alignment) at T0, scaled to registrations/s by
    the closest-point passes one registration takes."""
    import oracle
    mode = int(prm.mode)
    nu = float(prm.nu_min) if mode != 0 else 0.0
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        oracle.eval_map(d["P"], d["Q"], d["Qn"] if mode == 2 else None, mode, np.eye(4), max(nu, 1e-3))
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > budget_s or len(times) >= 30:
            break
    t_pass = float(np.median(times))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    M, N = len(d["P"]), len(d["Q"])
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": 1.0 / (t_pass * passes_per_reg), "unit": "registrations/s", "cores": cores,
            "kind": "oracle", "cpu": model,
            "sample": f"{len(times)} full-size map evaluations ({M} x {N} exhaustive FP32 closest point + "
                      f"FP64 alignment) at T0, median {t_pass:.3f} s each; registrations/s = "
                      f"1 / (t_eval x {passes_per_reg:.0f} closest-point passes per registration)",
            "nn_queries_per_s": M / t_pass}


def brute_roofline(ctx, B, torch):
    """Exhaustive closest-point kernel at M = N = 100k (1e10 pairs per launch)."""
    from paper_2007_07627_amd import synth
    d = synth.partial_sphere_pair(synth.rng_for(2, 0))
    P = torch.from_numpy(d["P"]).cuda()
    Q = torch.from_numpy(d["Q"]).cuda()
    idx = torch.empty(len(d["P"]), dtype=torch.int32, device="cuda")
    d2 = torch.empty(len(d["P"]), dtype=torch.float32, device="cuda")
    B.icp_nn_query_dev(ctx, P, Q, d["T_gt"], B.ICP_NN_BRUTE, idx, d2)  # warm-up
    B.icp_profile(ctx, True)
    reps = 5
    for _ in range(reps):
        B.icp_nn_query_dev(ctx, P, Q, d["T_gt"], B.ICP_NN_BRUTE, idx, d2)
    st = B.icp_profile_read(ctx)
    B.icp_profile(ctx, False)
    pairs = float(len(d["P"])) * float(len(d["Q"]))
    ms = st["nn_ms"] / max(1, st["passes"])
    tf = pairs * FLOPS_PER_PAIR / (ms * 1e-3) / 1e12
    return {"kernel": "nn_kernel (exhaustive)", "M": len(d["P"]), "N": len(d["Q"]), "ms_per_launch": ms,
            "pairs_per_s": pairs / (ms * 1e-3), "achieved_tflops": tf, "peak_tflops": FP32_PEAK_TFLOPS,
            "frac": tf / FP32_PEAK_TFLOPS}


def brute_batch_roofline(B, count=256):
    """Exhaustive closest point over a batch of config-1 shapes: `count` Fast
    ICP pairs of 4096 x 4096 (L2 + Anderson m = 5, brute force) advanced
    together by the batch engine, each pass's closest-point kernels timed
    with HIP events on the library's stream; work = the pairs examined."""
    from paper_2007_07627_amd import synth
    prm = lambda: B.icp_params_default(B.ICP_P2P_L2, eps=1e-6, iter_first=50, iter_cap=50, nn=B.ICP_NN_BRUTE)
    ds = [synth.fast_icp_pair(synth.rng_for(1, i)) for i in range(count)]
    reqs = [(d["P"], d["Q"], None, prm()) for d in ds]
    ctx = B.icp_create(0, 8 << 30)
    B.icp_batch_config(ctx, 4, count)
    _wait_tickets(B, ctx, B.icp_batch_submit(ctx, reqs[:8]))  # warm-up
    B.icp_profile(ctx, True)
    t0 = time.perf_counter()
    res = _wait_tickets(B, ctx, B.icp_batch_submit(ctx, reqs))
    wall = time.perf_counter() - t0
    st = B.icp_profile_read(ctx)
    B.icp_profile(ctx, False)
    B.icp_destroy(ctx)
    pairs = float(sum(r["nn_pairs"] for r in res))
    passes = max(1, st["passes"])
    tf = pairs * FLOPS_PER_PAIR / (max(st["nn_ms"], 1e-9) * 1e-3) / 1e12
    return {"kernel": "nn_kernel (exhaustive, batch engine)", "pairs": count, "M": 4096, "N": 4096,
            "batch_passes": passes, "pairs_examined_per_pass": pairs / passes,
            "nn_ms_per_pass": st["nn_ms"] / passes, "achieved_tflops": tf, "peak_tflops": FP32_PEAK_TFLOPS,
            "frac": tf / FP32_PEAK_TFLOPS, "registrations_per_s_profiled": count / wall}


def _params_for(B, d):
    if d["mode"] == 2:
        return B.icp_params_default(B.ICP_P2PL_WELSCH, anderson_m=6, nu_min=d["nu_min"])
    return B.icp_params_default(B.ICP_P2P_WELSCH, nu_min=d["nu_min"])


def _wait_tickets(B, ctx, tickets):
    out = {}
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                rc, r = B.icp_poll(ctx, t)
                if rc == B.ICP_OK:
                    out[t] = r
                elif rc != B.ICP_ERR_NOT_READY:
                    raise RuntimeError(B.icp_status_str(rc))
        time.sleep(0.0005)
    return [out[t] for t in tickets]


def batch_bench(args):
    """Config 4: 256 independent pairs (M, N log-uniform in [2k, 200k], mode and
    generator by seeded coins) advanced together by the batch engine, against
    the plain one-pair-at-a-time loop over the same pairs."""
    from paper_2007_07627_amd import binding as B
    from paper_2007_07627_amd import metrics, synth
    count = args.batch_pairs
    log(f"generating {count} pairs")
    pairs = synth.batch_pairs(count=count)
    reqs = [(d["P"], d["Q"], d["Qn"] if d["mode"] == 2 else None, _params_for(B, d)) for d in pairs]
    ctx = B.icp_create(0, 32 << 30)
    B.icp_batch_config(ctx, args.passes_per_replay, min(1024, count))
    _wait_tickets(B, ctx, B.icp_batch_submit(ctx, reqs[: min(16, count)]))  # warm-up
    log("batched run")
    t0 = time.perf_counter()
    tickets = B.icp_batch_submit(ctx, reqs)
    t_sub = time.perf_counter() - t0
    res = _wait_tickets(B, ctx, tickets)
    wall = time.perf_counter() - t0
    log(f"batched: {count} registrations in {wall:.2f} s; plain loop")
    t0 = time.perf_counter()
    res_p = []
    for P, Q, Qn, prm in reqs:
        prm.engine = B.ICP_ENGINE_PLAIN
        res_p.append(B.icp_register(ctx, P, Q, Qn, prm))
    wall_p = time.perf_counter() - t0
    rm = [metrics.rmse(d["T_gt"], r["T"], d["P"]) / d["diag"] for d, r in zip(pairs, res)]
    rm_p = [metrics.rmse(d["T_gt"], r["T"], d["P"]) / d["diag"] for d, r in zip(pairs, res_p)]
    same = sum(bool(np.array_equal(a["T"], b["T"])) for a, b in zip(res, res_p))
    M = sum(len(d["P"]) for d in pairs)
    N = sum(len(d["Q"]) for d in pairs)
    queries = sum(len(d["P"]) * r["nn_passes"] for d, r in zip(pairs, res))
    lat = [r["latency_ms"] for r in res]
    B.icp_destroy(ctx)
    return {
        "metric": "registrations/s & NN queries/s vs plain loop at equal RMSE; p50/p99 latency",
        "value": count / wall, "unit": "registrations/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 distances / f64 reductions and solves",
        "data": "synthetic (seeded generators standing in for the paper's scans)",
        "config": {"workload": f"batched registration: {count} pairs, M,N log-uniform in [2k,200k], "
                               "robust p2p / p2pl by seeded coin", "sum_M": M, "sum_N": N,
                   "passes_per_replay": args.passes_per_replay},
        "nn_queries_per_s": queries / wall,
        "submit_ms": t_sub * 1e3,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "plain_loop": {"value": count / wall_p, "unit": "registrations/s",
                       "nn_queries_per_s": queries / wall_p},
        "speedup_vs_plain": wall_p / wall,
        "rmse_over_diag_mean": float(np.mean(rm)), "rmse_over_diag_mean_plain": float(np.mean(rm_p)),
        "bit_identical_to_plain": f"{same}/{count}",
    }


def serve_bench(args):
    """Config 5: height-field requests with M, N log-uniform in [1k, 1M] arriving
    as a Poisson process at 80% of the measured batched capacity; latency from
    submission to completion. The FIFO comparator serves the same arrival trace
    one request at a time with each request's measured plain-loop time."""
    from paper_2007_07627_amd import binding as B
    from paper_2007_07627_amd import metrics, synth
    n_cap, n_req = args.serve_capacity_requests, args.serve_requests
    log(f"generating {n_cap} + {n_req} requests")
    cap_reqs = synth.served_requests(n_cap, start=10000)
    reqs = synth.served_requests(n_req)
    as_req = lambda d: (d["P"], d["Q"], d["Qn"], _params_for(B, d))
    ctx = B.icp_create(0, 64 << 30)
    B.icp_batch_config(ctx, args.passes_per_replay, 256)
    _wait_tickets(B, ctx, B.icp_batch_submit(ctx, [as_req(d) for d in cap_reqs[:4]]))  # warm-up
    t0 = time.perf_counter()
    _wait_tickets(B, ctx, B.icp_batch_submit(ctx, [as_req(d) for d in cap_reqs]))
    capacity = n_cap / (time.perf_counter() - t0)
    rate = 0.8 * capacity
    log(f"closed-loop capacity {capacity:.2f} req/s -> Poisson rate {rate:.2f} req/s")
    rng = np.random.default_rng(5)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    tickets = [None] * n_req
    t0 = time.perf_counter()
    for i, d in enumerate(reqs):
        delay = arrivals[i] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets[i] = B.icp_batch_submit(ctx, [as_req(d)])[0]
    res = _wait_tickets(B, ctx, tickets)
    wall = time.perf_counter() - t0
    lat = np.array([r["latency_ms"] for r in res])
    log("plain-loop service times")
    svc, res_p = [], []
    for d in reqs:
        P, Q, Qn, prm = as_req(d)
        prm.engine = B.ICP_ENGINE_PLAIN
        t = time.perf_counter()
        res_p.append(B.icp_register(ctx, P, Q, Qn, prm))
        svc.append(time.perf_counter() - t)
    finish, lat_f = 0.0, []
    for a, s_ in zip(arrivals, svc):
        start = max(a, finish)
        finish = start + s_
        lat_f.append((finish - a) * 1e3)
    drm = max(abs(metrics.rmse(d["T_gt"], a["T"], d["P"]) - metrics.rmse(d["T_gt"], b["T"], d["P"]))
              for d, a, b in zip(reqs, res, res_p))
    B.icp_destroy(ctx)
    return {
        "metric": "registrations/s & NN queries/s vs plain loop at equal RMSE; p50/p99 latency",
        "value": n_req / wall, "unit": "registrations/s", "n_gpus": 1, "steps": n_req, "warmup": 4,
        "ms_per_step": wall / n_req * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 distances / f64 reductions and solves",
        "data": "synthetic (seeded generators standing in for the paper's scans)",
        "config": {"workload": f"served stream: {n_req} height-field requests, M,N log-uniform in [1k,1M], "
                               f"Poisson arrivals at 0.8 x closed-loop capacity ({capacity:.2f} req/s)"},
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "fifo_plain": {"value": n_req / (finish - arrivals[0] + svc[0]) if n_req else None,
                       "p50_ms": float(np.percentile(lat_f, 50)), "p99_ms": float(np.percentile(lat_f, 99))},
        "max_abs_delta_rmse_vs_fifo": drm,
    }


def concurrent_run(args, B, ctx, ds, prms, ref):
    """The same seeded pairs submitted together to the batch engine, so that
    they advance in one pass sequence (a throughput figure beside the
    one-at-a-time `value`). The batch API takes host arrays: uploads and the
    request setup are inside the timed region."""
    reqs = []
    for d, p in zip(ds, prms):
        p.engine = B.ICP_ENGINE_GRAPH
        reqs.append((d["P"], d["Q"], d["Qn"] if int(p.mode) == 2 else None, p))
    B.icp_batch_config(ctx, args.passes_per_replay, len(reqs))
    _wait_tickets(B, ctx, B.icp_batch_submit(ctx, reqs[:2]))  # warm-up
    t0 = time.perf_counter()
    res = _wait_tickets(B, ctx, B.icp_batch_submit(ctx, reqs))
    wall = time.perf_counter() - t0
    lat = [r["latency_ms"] for r in res]
    same = all(np.array_equal(r["T"], ref[k]["T"]) for k, r in enumerate(res) if k in ref)
    log(f"in flight: {len(reqs)} registrations in {wall:.3f} s")
    return {"pairs_in_flight": len(reqs), "value": len(reqs) / wall, "unit": "registrations/s",
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "inputs": "host arrays (upload and setup timed)", "identical_to_one_at_a_time": bool(same)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="robust-p2p-100k",
                    choices=["robust-p2p-100k", "fast-icp-4096", "robust-p2pl-500k", "batch-256", "serve"])
    ap.add_argument("--batch-pairs", type=int, default=256)
    ap.add_argument("--passes-per-replay", type=int, default=4)
    ap.add_argument("--serve-requests", type=int, default=120)
    ap.add_argument("--serve-capacity-requests", type=int, default=40)
    ap.add_argument("--plain-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-brute", action="store_true")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="skip the run with all pairs of the workload in flight at once")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain device copy of known size (for HBM counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the registration path runs on a single MI355X "
              "(multi-GPU sharding is not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch-256":
        print(json.dumps(batch_bench(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(serve_bench(args)), flush=True)
        return

    import torch

    from paper_2007_07627_amd import binding as B
    from paper_2007_07627_amd import metrics

    log(f"workload {args.workload}")
    ds, prms, cfg = workload(args.workload)
    dev = torch.device("cuda:0")
    npair = len(ds)
    Ps = [torch.from_numpy(d["P"]).to(dev) for d in ds]
    Qs = [torch.from_numpy(d["Q"]).to(dev) for d in ds]
    Qns = [torch.from_numpy(d["Qn"]).to(dev) if d["Qn"] is not None and int(p.mode) == 2 else None
           for d, p in zip(ds, prms)]
    ctx = B.icp_create(0, 16 << 30)
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        copy_calibration(torch)

    def run(engine, steps, profile=False):
        lat, res = [], []
        if profile:
            B.icp_profile(ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            k = i % npair
            prms[k].engine = engine
            t = time.perf_counter()
            r = B.icp_register_dev(ctx, Ps[k], Qs[k], Qns[k], prms[k], stream)
            lat.append((time.perf_counter() - t) * 1e3)
            res.append(r)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = B.icp_profile_read(ctx) if profile else None
        if profile:
            B.icp_profile(ctx, False)
        return wall, lat, res, prof

    for i in range(args.warmup):
        k = i % npair
        prms[k].engine = B.ICP_ENGINE_GRAPH
        B.icp_register_dev(ctx, Ps[k], Qs[k], Qns[k], prms[k], stream)
        log(f"warm-up {i + 1}/{args.warmup}")
    K = args.steps
    wall, lat, res, _ = run(B.ICP_ENGINE_GRAPH, K)
    log(f"graph engine: {K} registrations in {wall:.3f} s")
    # kernel durations: HIP events around every pass kernel on the library's
    # stream, over a second run of the same K registrations
    wall_prof, _, res_prof, prof = run(B.ICP_ENGINE_GRAPH, K, profile=True)
    log(f"profiled run: {K} registrations in {wall_prof:.3f} s, {prof['passes']} passes timed")
    Kp = args.plain_steps or K
    wall_p, lat_p, res_p, _ = run(B.ICP_ENGINE_PLAIN, Kp)
    log(f"plain loop: {Kp} registrations in {wall_p:.3f} s")

    # per pair: the first graph result is the reference of every other run of it
    ref = {}
    for i, r in enumerate(res):
        ref.setdefault(i % npair, r)
    same = all(np.array_equal(r["T"], ref[i % npair]["T"]) for i, r in enumerate(res)) and \
        all(np.array_equal(r["T"], ref[i % npair]["T"]) for i, r in enumerate(res_p) if i % npair in ref)
    rm = [metrics.rmse(ds[k]["T_gt"], ref[k]["T"], ds[k]["P"]) for k in sorted(ref)]
    rm_p = [metrics.rmse(ds[i % npair]["T_gt"], r["T"], ds[i % npair]["P"]) for i, r in enumerate(res_p[:npair])]
    rmse, rmse_p = float(np.mean(rm)), float(np.mean(rm_p))
    diag = float(np.mean([ds[k]["diag"] for k in sorted(ref)]))
    M = len(ds[0]["P"])
    passes = float(np.mean([r["nn_passes"] for r in res]))
    value = K / wall
    # dominant kernel: the closest-point search
    pairs = float(np.sum([r["nn_pairs"] for r in res_prof]))
    nn_ms = max(prof["nn_ms"], 1e-9)
    launches = max(1, prof["passes"])
    achieved = pairs * FLOPS_PER_PAIR / (nn_ms * 1e-3) / 1e12
    traffic, traffic_note = measured_traffic() if args.workload == "robust-p2p-100k" else (None, "")
    roof = {"bound": "alu", "kernel": "nn_kernel", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic,
            "traffic_note": traffic_note,
            "ms_per_launch": nn_ms / launches, "launches": launches,
            "algorithmic_flops_per_launch": pairs * FLOPS_PER_PAIR / launches,
            "work": "8 flops per (source, target) pair run through the filter (chunks some lane can need)",
            "share_of_pass_time": nn_ms / max(1e-9, nn_ms + prof["reduce_ms"] + prof["solve_ms"]),
            "reduce_ms_per_launch": prof["reduce_ms"] / launches,
            "solve_ms_per_launch": prof["solve_ms"] / launches}
    out = {
        "metric": "registrations/s & NN queries/s vs plain loop at equal RMSE; p50/p99 latency",
        "value": value,
        "unit": "registrations/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 distances / f64 reductions and solves",
        "data": "synthetic (seeded generators standing in for the paper's scans)",
        "config": cfg,
        "nn_queries_per_s": M * passes * K / wall,
        "nn_passes_per_registration": passes,
        "us_per_pass": wall / K / passes * 1e6,
        "iterations_per_registration": float(np.mean([r["iterations"] for r in res])),
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "plain_loop": {"value": Kp / wall_p, "unit": "registrations/s",
                       "p50_ms": float(np.percentile(lat_p, 50)), "p99_ms": float(np.percentile(lat_p, 99)),
                       "rmse": rmse_p},
        "speedup_vs_plain": value / (Kp / wall_p),
        "rmse": rmse, "rmse_over_diag": rmse / diag, "equal_rmse": bool(rmse == rmse_p),
        "bit_identical_all_steps": bool(same),
        "effective_pairs_per_s": M * float(len(ds[0]["Q"])) * passes * K / wall,
        "roofline": roof,
    }
    if not args.no_concurrent and npair > 1:
        out["in_flight"] = concurrent_run(args, B, ctx, ds, prms, ref)
    if not args.no_brute:
        log("exhaustive kernel roofline (100k x 100k)")
        out["nn_brute_roofline"] = brute_roofline(ctx, B, torch)
        if args.workload == "fast-icp-4096":
            log("exhaustive closest point over 256 config-1 pairs in the batch engine")
            out["nn_brute_batch_roofline"] = brute_batch_roofline(B)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(ds[0], prms[0], passes)
    B.icp_destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

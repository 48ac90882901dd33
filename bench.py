#!/usr/bin/env python3
"""Benchmark of the Fast and Robust ICP hot path on one MI355X.

Headline (default workload `batch-256`): 256 independent registration pairs,
M and N log-uniform in [2k, 200k] (bumpy sphere; full-resample or
70%-overlap generator and robust point-to-point (Algorithm 1, Anderson m = 5)
or robust point-to-plane (Algorithm 2, m = 6) by seeded coins; nu from
3 x median down to 1e-3 diag), advanced together by the batch engine. The
pairs' arrays are uploaded to HBM before the timed region; a step is one
batch: all 256 registrations submitted with device pointers, timed to the
last result. `value` is registrations/s over K steps. Beside it: the same
batch submitted as host arrays (the PCIe-inclusive rate), the plain
one-pair-at-a-time loop over the same 256 pairs (host-synchronised passes),
latency percentiles, the per-pair RMSE distribution, the closest-point
kernels' roofline position in that run, and the CPU oracle on a bounded
sample of the same pairs.

Secondary fields: `serve` (height-field requests, M, N log-uniform in
[1k, 1M], Poisson arrivals at 0.8 x the batch engine's closed-loop capacity,
500 warm-up + 5000 measured requests, against a FIFO plain loop replaying the
same arrival trace), `robust_p2p_100k` (one 100k x 100k pair at a time, inputs
resident in HBM, graph engine vs plain loop), and the exhaustive closest-point
kernel at 100k x 100k and over 256 pairs of 4096 x 4096.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "registrations/s & NN queries/s vs plain loop at equal RMSE; p50/p99 latency"
FP32_PEAK_TFLOPS = 157.3  # MI355X vector FP32 (packed FMA), published
FLOPS_PER_PAIR = 8        # 3 sub, 1 mul, 2 FMA per (source, target) distance
TRAFFIC_SOURCES = ["paper_2007_07627_amd/csrc/nn.hip", "paper_2007_07627_amd/csrc/icp_internal.h"]
TRAFFIC_FILES = {"robust-p2p-100k": os.path.join(ROOT, "profiles", "nn_traffic_robust_p2p_100k.md"),
                 "batch-256": os.path.join(ROOT, "profiles", "nn_traffic_batch_256.md")}
COPY_CALIBRATION_BYTES = 256 << 20
DTYPE = "f32 distances / f64 reductions and solves"
DATA = "synthetic (seeded generators standing in for the paper's scans)"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ------------------------------------------------------------------ inputs

def _gen_batch_pair(i):
    from paper_2007_07627_amd import synth
    return synth.batch_pair(i)


def _gen_served(i):
    from paper_2007_07627_amd import synth
    return synth.served_request(i)


def _gen_fast(i):
    from paper_2007_07627_amd import synth
    return synth.fast_icp_pair(synth.rng_for(1, i))


def _gen_sphere(i):
    from paper_2007_07627_amd import synth
    return synth.partial_sphere_pair(synth.rng_for(2, i))


def generate(fn, count, workers):
    """Seeded inputs generated in forked workers (numpy only; before any GPU
    call of this process)."""
    if workers <= 1 or count <= 1:
        return [fn(i) for i in range(count)]
    with cf.ProcessPoolExecutor(max_workers=min(workers, count), mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(fn, range(count), chunksize=max(1, count // (4 * workers))))


# ------------------------------------------------------------------ helpers

def sources_digest():
    """sha256 over the code of the closest-point kernel sources (the counters
    in a traffic summary hold only for the code they were taken from): line
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


def measured_traffic(workload):
    """HBM bytes per closest-point launch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary of this workload, or None when it is
    missing or was taken from other kernel sources."""
    path = TRAFFIC_FILES.get(workload)
    try:
        with open(path) as f:
            txt = f.read()
    except (OSError, TypeError):
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


def _params_for(B, d):
    if d["mode"] == 2:
        return B.icp_params_default(B.ICP_P2PL_WELSCH, anderson_m=6, nu_min=d["nu_min"])
    return B.icp_params_default(B.ICP_P2P_WELSCH, nu_min=d["nu_min"])


def _request(B, d):
    return (d["P"], d["Q"], d["Qn"] if d["mode"] == 2 else None, _params_for(B, d))


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


def _pct(v, q):
    return float(np.percentile(np.asarray(v, np.float64), q))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        return ""


def _omp():
    """The OpenMP runtime the oracle links (thread count control)."""
    import ctypes
    import oracle
    oracle.lib()
    try:
        return ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None


def nn_roofline(prof, pairs, workload, note):
    """Closest-point kernels of a pass (cull + slice, exhaustive items): 8
    flops per (source, target) pair run through the filter, over their HIP
    event time on the library's stream."""
    nn_ms = max(prof["nn_ms"], 1e-9)
    launches = max(1, prof["passes"])
    achieved = pairs * FLOPS_PER_PAIR / (nn_ms * 1e-3) / 1e12
    traffic, tnote = measured_traffic(workload)
    total = max(1e-9, nn_ms + prof["reduce_ms"] + prof["solve_ms"])
    return {"bound": "alu", "kernel": "nn_kernels (cull + slice + exhaustive items)", "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": traffic, "traffic_note": tnote,
            "ms_per_launch": nn_ms / launches, "launches": launches,
            "algorithmic_flops_per_launch": pairs * FLOPS_PER_PAIR / launches,
            "work": "8 flops per (source, target) pair run through the filter (chunks some lane can need)",
            "share_of_pass_time": nn_ms / total,
            "reduce_ms_per_launch": prof["reduce_ms"] / launches,
            "solve_ms_per_launch": prof["solve_ms"] / launches, "note": note}


# ------------------------------------------------------------------ batch-256 (headline)

def tuning_used(B, ctx, shapes, batch):
    """The autotuner's partition each (M, N, mode) uses in an engine kind:
    distinct settings with their pair counts, and how many shapes had their
    own tuned bucket."""
    seen, found = {}, [0, 0, 0]
    for M, N, mode in shapes:
        t, f = B.icp_tuning_lookup(ctx, M, N, mode, B.ICP_NN_AUTO, batch)
        key = json.dumps(t, sort_keys=True)
        seen[key] = seen.get(key, 0) + 1
        found[f] += 1
    return {"arch": B.icp_device_arch(0), "table_entries": len(B.icp_tuning_entries(ctx)),
            "pairs_with_own_bucket": found[2], "pairs_with_nearby_bucket": found[1],
            "pairs_with_defaults": found[0],
            "settings": [dict(json.loads(k), pairs=v) for k, v in sorted(seen.items(), key=lambda x: -x[1])]}


def counter_run(B, torch, pairs, passes_per_replay):
    """One batch-256 step from device inputs, without timing events or
    comparators: the run that rocprofv3 --pmc counts. Prints the batch's
    passes (the highest per-pair count) as a JSON line."""
    dev = torch.device("cuda:0")
    dreqs = [(torch.from_numpy(P).to(dev), torch.from_numpy(Q).to(dev),
              None if Qn is None else torch.from_numpy(Qn).to(dev), prm)
             for P, Q, Qn, prm in (_request(B, d) for d in pairs)]
    torch.cuda.synchronize()
    ctx = B.icp_create(0, 32 << 30)
    B.icp_batch_config(ctx, passes_per_replay, min(1024, len(pairs)))
    t0 = time.perf_counter()
    res = _wait_tickets(B, ctx, B.icp_batch_submit_dev(ctx, dreqs, torch.cuda.current_stream()))
    log(f"counter run: {len(res)} registrations in {time.perf_counter() - t0:.2f} s")
    B.icp_destroy(ctx)
    print(json.dumps({"counter_run": "batch-256", "pairs": len(res),
                      "max_pair_passes": int(max(r["nn_passes"] for r in res))}), flush=True)


def batch_bench(args, B, pairs):
    """Batch-256: the pairs' arrays are uploaded to HBM first; a step submits
    all of them (device pointers, icp_batch_submit_dev) and waits for the last
    result. Beside it the same batch from host arrays (copied by the library
    and uploaded: the PCIe-inclusive rate) and the plain one-at-a-time loop
    on the same device arrays."""
    import torch
    from paper_2007_07627_amd import metrics
    count = len(pairs)
    reqs = [_request(B, d) for d in pairs]
    dev = torch.device("cuda:0")
    dreqs = [(torch.from_numpy(P).to(dev), torch.from_numpy(Q).to(dev),
              None if Qn is None else torch.from_numpy(Qn).to(dev), prm) for P, Q, Qn, prm in reqs]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ctx = B.icp_create(0, 32 << 30)
    tuning = tuning_used(B, ctx, [(len(d["P"]), len(d["Q"]), 2 if d["mode"] == 2 else 1) for d in pairs], 1)
    B.icp_batch_config(ctx, args.passes_per_replay, min(1024, count))

    def run_dev():
        return _wait_tickets(B, ctx, B.icp_batch_submit_dev(ctx, dreqs, stream))

    for w in range(args.warmup):
        run_dev()
        log(f"batch warm-up {w + 1}/{args.warmup}")
    walls, lat, res0 = [], [], None
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for k in range(args.steps):
        t0 = time.perf_counter()
        res = run_dev()
        walls.append(time.perf_counter() - t0)
        lat += [r["latency_ms"] for r in res]
        if res0 is None:
            res0 = res
        elif not all(np.array_equal(a["T"], b["T"]) for a, b in zip(res0, res)):
            raise RuntimeError("batch results differ between steps")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_all
    log(f"batched (inputs in HBM): {args.steps} x {count} registrations in {wall:.2f} s")
    # the same batch from host arrays: validation, copies into library-owned
    # host memory and uploads are inside the timed region
    t0 = time.perf_counter()
    res_h = _wait_tickets(B, ctx, B.icp_batch_submit(ctx, reqs))
    wall_h = time.perf_counter() - t0
    host_same = sum(bool(np.array_equal(a["T"], b["T"])) for a, b in zip(res0, res_h))
    log(f"batched (host arrays): {count} registrations in {wall_h:.2f} s")
    # the same batch once more with per-pass kernel timing (HIP events)
    B.icp_profile(ctx, True)
    res_prof = run_dev()
    prof = B.icp_profile_read(ctx)
    B.icp_profile(ctx, False)
    log(f"profiled batch: {prof['passes']} batch passes timed")
    # plain loop: the same pairs one at a time from the same device arrays,
    # host-synchronised passes
    lat_p, res_p = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for P, Q, Qn, prm in ([] if args.no_plain else dreqs):
        prm.engine = B.ICP_ENGINE_PLAIN
        t = time.perf_counter()
        res_p.append(B.icp_register_dev(ctx, P, Q, Qn, prm, stream))
        lat_p.append((time.perf_counter() - t) * 1e3)
        prm.engine = B.ICP_ENGINE_GRAPH
    wall_p = time.perf_counter() - t0
    if args.no_plain:
        res_p, lat_p, wall_p = res0, [float("nan")], float("nan")
    log(f"plain loop: {len(res_p)} registrations in {wall_p:.2f} s")
    B.icp_destroy(ctx)
    rm = np.array([metrics.rmse(d["T_gt"], r["T"], d["P"]) / d["diag"] for d, r in zip(pairs, res0)])
    rm_p = np.array([metrics.rmse(d["T_gt"], r["T"], d["P"]) / d["diag"] for d, r in zip(pairs, res_p)])
    rot = np.array([metrics.rotation_error_rad(d["T_gt"], r["T"]) for d, r in zip(pairs, res0)])
    same = sum(bool(np.array_equal(a["T"], b["T"])) for a, b in zip(res0, res_p))
    passes = np.array([r["nn_passes"] for r in res0], np.float64)
    M = np.array([len(d["P"]) for d in pairs], np.float64)
    N = np.array([len(d["Q"]) for d in pairs], np.float64)
    queries = float((M * passes).sum())
    value = count * args.steps / wall
    far = rot > np.radians(10.0)
    far_pairs = []
    for i in np.flatnonzero(far):
        E = np.asarray(pairs[i]["T_gt"])[:3, :3].T @ np.asarray(res0[i]["T"])[:3, :3]
        w = np.array([E[2, 1] - E[1, 2], E[0, 2] - E[2, 0], E[1, 0] - E[0, 1]])
        far_pairs.append({"pair": int(i), "M": int(M[i]), "N": int(N[i]), "mode": int(pairs[i]["mode"]),
                          "rotation_error_deg": float(np.degrees(rot[i])),
                          "error_axis_z": float(abs(w[2]) / max(np.linalg.norm(w), 1e-300))})
    out = {
        "metric": METRIC, "value": value, "unit": "registrations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE, "data": DATA,
        "config": {"workload": f"batched registration: {count} independent pairs, M,N log-uniform in "
                               "[2k,200k], bumpy sphere (full resample or 70% overlap with 10% outliers), "
                               "robust point-to-point (Alg. 1, m=5) or point-to-plane (Alg. 2, m=6) by "
                               "seeded coin, nu 3 x median -> 1e-3 diag; inputs resident in HBM; one step = "
                               "all pairs submitted (device pointers) to the last result",
                   "pairs": count, "sum_M": int(M.sum()), "sum_N": int(N.sum()),
                   "point_to_plane_pairs": int(sum(d["mode"] == 2 for d in pairs)),
                   "passes_per_replay": args.passes_per_replay},
        "nn_queries_per_s": queries * args.steps / wall,
        "nn_passes_per_registration": float(passes.mean()),
        "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99),
        "host_arrays": {"value": count / wall_h, "unit": "registrations/s",
                        "note": "the same batch submitted as host arrays (icp_batch_submit): validation, "
                                "copies into library-owned memory and PCIe uploads inside the timed region",
                        "bit_identical_to_device_inputs": f"{host_same}/{count}"},
        "plain_loop": None if args.no_plain else {
            "value": count / wall_p, "unit": "registrations/s", "p50_ms": _pct(lat_p, 50),
            "p99_ms": _pct(lat_p, 99), "nn_queries_per_s": queries / wall_p},
        "speedup_vs_plain": None if args.no_plain else value / (count / wall_p),
        "equal_rmse": None if args.no_plain else bool(np.array_equal(rm, rm_p)),
        "bit_identical_to_plain": None if args.no_plain else f"{same}/{count}",
        "rmse_over_diag": {"mean": float(rm.mean()), "median": float(np.median(rm)),
                           "p90": _pct(rm, 90), "max": float(rm.max()),
                           "pairs_below_1e-3": int((rm < 1e-3).sum()),
                           "pairs_rotated_over_10deg_from_truth": int(far.sum()),
                           "mean_excluding_those": float(rm[~far].mean()) if (~far).any() else None,
                           "far_pairs": far_pairs,
                           "note": "pairs start up to 45 deg from the truth; some settle in another "
                                   "local minimum of their energy: the bumpy sphere is symmetric under a "
                                   "90 deg turn about z (error rotation near 90 deg about z), and "
                                   "point-to-plane trajectories can wander into other minima; the oracle "
                                   "lands in such minima too (tests replay these trajectories step by step)"},
        "roofline": nn_roofline(prof, float(sum(r["nn_pairs"] for r in res_prof)), "batch-256",
                                "one profiled batch of the same 256 pairs; kernels timed per batch pass (the two slot branches of a pass one after the other, their intervals summed)"),
        "tuning": tuning,
    }
    return out, {"pairs": pairs, "passes": passes}


def cpu_baseline_batch(pairs, passes, budget_s):
    """The oracle as it stands on a bounded seeded sample of the batch: one
    full-size map evaluation at T0 per sampled pair (exhaustive FP32 closest
    point + FP64 reduction and update) on all host threads, pairs in a seeded
    order until budget_s seconds have been spent, and repeated evaluations of
    the smallest sampled pair on a single thread for about 2 s. Its cost is M x N pairs per evaluation, so the sample's pairs per
    second extrapolate to the whole batch: time = sum_i passes_i x M_i N_i /
    rate, with passes_i the closest-point passes the GPU run made for pair i."""
    import oracle
    gomp = _omp()
    cores = int(gomp.omp_get_max_threads()) if gomp else int(os.environ.get("OMP_NUM_THREADS", "1"))
    rng = np.random.default_rng(7)
    order = rng.permutation(len(pairs))
    used, times = [], []
    t_start = time.perf_counter()
    for i in order:
        d = pairs[i]
        t0 = time.perf_counter()
        oracle.eval_map(d["P"], d["Q"], d["Qn"] if d["mode"] == 2 else None, d["mode"], np.eye(4), d["nu_min"])
        times.append(time.perf_counter() - t0)
        used.append(int(i))
        if time.perf_counter() - t_start > budget_s and len(used) >= 3:
            break
    mn = np.array([len(pairs[i]["P"]) * float(len(pairs[i]["Q"])) for i in used])
    rate = mn.sum() / np.sum(times)
    all_mn = np.array([len(d["P"]) * float(len(d["Q"])) for d in pairs])
    t_batch = float((passes * all_mn).sum() / rate)
    out = {"value": len(pairs) / t_batch, "unit": "registrations/s", "cores": cores, "kind": "oracle",
           "cpu": _cpu_model(),
           "sample": f"{len(used)} of the {len(pairs)} pairs (seeded), one full-size map evaluation each "
                     f"at T0 ({mn.sum():.3g} source-target pairs in {np.sum(times):.1f} s = "
                     f"{rate:.3g} pairs/s); whole batch = sum over pairs of (GPU closest-point passes x "
                     f"M x N) / rate = {t_batch:.0f} s",
           "nn_queries_per_s": float(sum(len(pairs[i]["P"]) for i in used) / np.sum(times))}
    if gomp is not None:
        k = int(used[int(np.argmin(mn))])
        d = pairs[k]
        gomp.omp_set_num_threads(1)
        reps = 0
        t0 = time.perf_counter()
        while reps < 1 or time.perf_counter() - t0 < 2.0:
            oracle.eval_map(d["P"], d["Q"], d["Qn"] if d["mode"] == 2 else None, d["mode"], np.eye(4),
                            d["nu_min"])
            reps += 1
        t1 = time.perf_counter() - t0
        gomp.omp_set_num_threads(cores)
        rate1 = reps * len(d["P"]) * float(len(d["Q"])) / t1
        out["single_thread"] = {"value": len(pairs) / float((passes * all_mn).sum() / rate1),
                                "unit": "registrations/s", "cores": 1,
                                "sample": f"pair {k} ({len(d['P'])} x {len(d['Q'])}), {reps} map evaluations "
                                          f"in {t1:.1f} s = {rate1:.3g} pairs/s, same extrapolation"}
    return out


# ------------------------------------------------------------------ served stream

def serve_bench(args, B, pool):
    from paper_2007_07627_amd import metrics
    n_warm, n_req = args.serve_warmup, args.serve_requests
    reqs = [_request(B, d) for d in pool]
    ctx = B.icp_create(0, 64 << 30)
    B.icp_batch_config(ctx, args.passes_per_replay, 256)
    _wait_tickets(B, ctx, B.icp_batch_submit(ctx, reqs[:8]))
    t0 = time.perf_counter()
    res_pool = _wait_tickets(B, ctx, B.icp_batch_submit(ctx, reqs))
    capacity = len(pool) / (time.perf_counter() - t0)
    rate = 0.8 * capacity
    log(f"serve: closed-loop capacity {capacity:.1f} req/s -> Poisson arrivals at {rate:.1f} req/s, "
        f"{n_warm} + {n_req} requests drawn from a pool of {len(pool)}")
    rng = np.random.default_rng(5)
    total = n_warm + n_req
    picks = rng.integers(0, len(pool), total)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, total))
    tickets, sub_t = [None] * total, np.zeros(total)
    t0 = time.perf_counter()
    for i in range(total):
        delay = arrivals[i] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        sub_t[i] = time.perf_counter() - t0
        tickets[i] = B.icp_batch_submit(ctx, [reqs[picks[i]]])[0]
        if (i + 1) % 1000 == 0:
            log(f"serve: {i + 1}/{total} submitted")
    res = _wait_tickets(B, ctx, tickets)
    lat = np.array([r["latency_ms"] for r in res])
    done_t = sub_t + lat * 1e-3
    meas = slice(n_warm, total)
    window = float(done_t[meas].max() - sub_t[n_warm])
    same = all(np.array_equal(r["T"], res_pool[picks[i]]["T"]) for i, r in enumerate(res))
    log("serve: plain-loop service time of every pool request")
    svc, res_p = np.zeros(len(pool)), []
    for j, (P, Q, Qn, prm) in enumerate(reqs):
        prm.engine = B.ICP_ENGINE_PLAIN
        t = time.perf_counter()
        res_p.append(B.icp_register(ctx, P, Q, Qn, prm))
        svc[j] = time.perf_counter() - t
        prm.engine = B.ICP_ENGINE_GRAPH
    B.icp_destroy(ctx)
    finish, lat_f, fin_f = 0.0, np.zeros(total), np.zeros(total)
    for i in range(total):
        start = max(arrivals[i], finish)
        finish = start + svc[picks[i]]
        lat_f[i] = (finish - arrivals[i]) * 1e3
        fin_f[i] = finish
    drm = max(abs(metrics.rmse(d["T_gt"], a["T"], d["P"]) - metrics.rmse(d["T_gt"], b["T"], d["P"]))
              for d, a, b in zip(pool, res_pool, res_p))
    return {
        "workload": f"served stream: height-field requests (Alg. 2, m=6, 60% overlap, 5% outliers), "
                    f"M,N log-uniform in [1k,1M]; {n_warm} warm-up + {n_req} measured requests drawn "
                    f"(seeded) from a pool of {len(pool)} generated requests; Poisson arrivals at 0.8 x "
                    f"closed-loop capacity; latency from submission to result",
        "value": n_req / window, "unit": "registrations/s", "requests": n_req, "warmup_requests": n_warm,
        "pool": len(pool), "capacity_req_per_s": capacity, "arrival_rate": rate,
        "p50_ms": _pct(lat[meas], 50), "p99_ms": _pct(lat[meas], 99),
        "results_equal_to_alone": bool(same),
        "fifo_plain": {"value": n_req / float(fin_f[meas].max() - arrivals[n_warm]),
                       "p50_ms": _pct(lat_f[meas], 50), "p99_ms": _pct(lat_f[meas], 99),
                       "note": "the same arrival trace through a FIFO one-at-a-time plain loop, each "
                               "request taking its measured plain-loop time"},
        "max_abs_delta_rmse_vs_fifo": drm,
    }


# ------------------------------------------------------------------ single pairs

def single_pair_bench(args, B, torch, ds, prms, cfg, workload_name, steps, warmup):
    """One pair at a time with inputs resident in HBM: graph engine vs plain
    loop, a profiled run for the closest-point kernels' roofline."""
    from paper_2007_07627_amd import metrics
    dev = torch.device("cuda:0")
    npair = len(ds)
    Ps = [torch.from_numpy(d["P"]).to(dev) for d in ds]
    Qs = [torch.from_numpy(d["Q"]).to(dev) for d in ds]
    Qns = [torch.from_numpy(d["Qn"]).to(dev) if int(p.mode) == 2 else None for d, p in zip(ds, prms)]
    ctx = B.icp_create(0, 16 << 30)
    stream = torch.cuda.current_stream()
    tuning = tuning_used(B, ctx, [(len(d["P"]), len(d["Q"]), int(p.mode)) for d, p in zip(ds, prms)], 0)

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
            res.append(B.icp_register_dev(ctx, Ps[k], Qs[k], Qns[k], prms[k], stream))
            lat.append((time.perf_counter() - t) * 1e3)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = B.icp_profile_read(ctx) if profile else None
        if profile:
            B.icp_profile(ctx, False)
        return wall, lat, res, prof

    run(B.ICP_ENGINE_GRAPH, warmup)
    wall, lat, res, _ = run(B.ICP_ENGINE_GRAPH, steps)
    _, _, res_prof, prof = run(B.ICP_ENGINE_GRAPH, steps, profile=True)
    wall_p, lat_p, res_p, _ = run(B.ICP_ENGINE_PLAIN, steps)
    B.icp_destroy(ctx)
    log(f"{workload_name}: graph {steps} registrations in {wall:.3f} s, plain {wall_p:.3f} s")
    same = all(np.array_equal(r["T"], res[i % npair]["T"]) for i, r in enumerate(res_p))
    rm = [metrics.rmse(ds[i % npair]["T_gt"], r["T"], ds[i % npair]["P"]) / ds[i % npair]["diag"]
          for i, r in enumerate(res[:npair])]
    passes = float(np.mean([r["nn_passes"] for r in res]))
    M, N = len(ds[0]["P"]), len(ds[0]["Q"])
    return {
        "config": cfg, "value": steps / wall, "unit": "registrations/s", "steps": steps,
        "ms_per_step": wall / steps * 1e3, "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99),
        "plain_loop": {"value": steps / wall_p, "p50_ms": _pct(lat_p, 50), "p99_ms": _pct(lat_p, 99)},
        "speedup_vs_plain": wall_p / wall, "bit_identical_to_plain": bool(same),
        "rmse_over_diag_mean": float(np.mean(rm)),
        "nn_passes_per_registration": passes, "us_per_pass": wall / steps / passes * 1e6,
        "nn_queries_per_s": M * passes * steps / wall,
        "effective_pairs_per_s": M * float(N) * passes * steps / wall,
        "roofline": nn_roofline(prof, float(sum(r["nn_pairs"] for r in res_prof)), workload_name,
                                "a second run of the same registrations with per-pass kernel timing"),
        "tuning": tuning,
    }


def brute_roofline(B, torch, d):
    """Exhaustive closest-point kernel at M = N = 100k (1e10 pairs per launch)."""
    ctx = B.icp_create(0, 4 << 30)
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
    B.icp_destroy(ctx)
    pairs = float(len(d["P"])) * float(len(d["Q"]))
    ms = st["nn_ms"] / max(1, st["passes"])
    tf = pairs * FLOPS_PER_PAIR / (ms * 1e-3) / 1e12
    return {"kernel": "nn_brute_kernel (exhaustive)", "M": len(d["P"]), "N": len(d["Q"]), "ms_per_launch": ms,
            "pairs_per_s": pairs / (ms * 1e-3), "achieved_tflops": tf, "peak_tflops": FP32_PEAK_TFLOPS,
            "frac": tf / FP32_PEAK_TFLOPS}


def brute_batch_roofline(B, ds):
    """Exhaustive closest point over a batch of config-1 shapes: Fast ICP pairs
    of 4096 x 4096 (L2 + Anderson m = 5, exhaustive search) advanced together
    by the batch engine, each batch pass's closest-point kernels timed with HIP
    events on the library's stream; work = the pairs examined."""
    prm = lambda: B.icp_params_default(B.ICP_P2P_L2, eps=1e-6, iter_first=50, iter_cap=50, nn=B.ICP_NN_BRUTE)
    reqs = [(d["P"], d["Q"], None, prm()) for d in ds]
    ctx = B.icp_create(0, 8 << 30)
    B.icp_batch_config(ctx, 4, len(ds))
    _wait_tickets(B, ctx, B.icp_batch_submit(ctx, reqs[:8]))
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
    return {"kernel": "nn_slice_kernel, exhaustive items of the batch engine", "pairs": len(ds), "M": 4096,
            "N": 4096, "batch_passes": passes, "pairs_examined_per_pass": pairs / passes,
            "nn_ms_per_pass": st["nn_ms"] / passes, "achieved_tflops": tf, "peak_tflops": FP32_PEAK_TFLOPS,
            "frac": tf / FP32_PEAK_TFLOPS, "registrations_per_s_profiled": len(ds) / wall}


def single_workload(name, B, ds):
    if name == "robust-p2p-100k":
        prms = [B.icp_params_default(B.ICP_P2P_WELSCH, nu_min=d["nu_min"], nn=B.ICP_NN_CLUSTER) for d in ds]
        cfg = {"workload": "robust point-to-point (Alg. 1) + Anderson m=5, one 100k x 100k pair at a time "
                           "(bumpy sphere 70% overlap, 10% outliers, noise 2e-3 diag, rotation <= 45 deg), "
                           f"{len(ds)} seeded pairs in turn, inputs resident in HBM",
               "M": 100000, "N": 100000, "nn": "cluster", "anderson_m": 5}
        return prms, cfg
    if name == "fast-icp-4096":
        prms = [B.icp_params_default(B.ICP_P2P_L2, eps=1e-6, iter_first=50, iter_cap=50, nn=B.ICP_NN_BRUTE)
                for _ in ds]
        cfg = {"workload": "Fast ICP (L2 + Anderson m=5), 4096 points, bumpy sphere, same points, "
                           "noise 1e-3 diag", "M": 4096, "N": 4096, "nn": "brute"}
        return prms, cfg
    if name == "robust-p2pl-500k":
        prms = [B.icp_params_default(B.ICP_P2PL_WELSCH, anderson_m=6, nu_min=d["nu_min"], nn=B.ICP_NN_CLUSTER)
                for d in ds]
        cfg = {"workload": "robust point-to-plane (Alg. 2) + Anderson m=6, height field 200k x 500k, "
                           "60% overlap, 5% outliers, noise 1e-3", "M": 200000, "N": 500000, "nn": "cluster"}
        return prms, cfg
    raise SystemExit(f"unknown workload {name}")


# ------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch-256",
                    choices=["batch-256", "robust-p2p-100k", "fast-icp-4096", "robust-p2pl-500k",
                             "nn-brute"])
    ap.add_argument("--batch-pairs", type=int, default=256)
    ap.add_argument("--passes-per-replay", type=int, default=4)
    ap.add_argument("--serve-requests", type=int, default=5000)
    ap.add_argument("--serve-warmup", type=int, default=500)
    ap.add_argument("--serve-pool", type=int, default=256)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the batch's plain-loop comparator (counter runs: every dispatch is slow)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="headline only: no 100k x 100k pair, no exhaustive-kernel runs")
    ap.add_argument("--counter-run", action="store_true",
                    help="batch-256 only: one batch step from device inputs and nothing else (no timing "
                         "events, no comparators), for rocprofv3 --pmc runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain device copy of known size (for HBM counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the registration path runs on a single MI355X and no "
              f"multi-GPU path is built (--gpus {args.gpus} requested); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    # every input first, in forked workers, before this process touches the GPU
    if args.counter_run:
        args.workload, args.no_serve, args.no_secondary = "batch-256", True, True
    t0 = time.perf_counter()
    if args.workload == "batch-256":
        pairs = generate(_gen_batch_pair, args.batch_pairs, args.workers)
        pool = [] if args.no_serve else generate(_gen_served, args.serve_pool, args.workers)
        sphere = [] if args.no_secondary else generate(_gen_sphere, 4, args.workers)
        fast = [] if args.no_secondary else generate(_gen_fast, 256, args.workers)
    elif args.workload == "nn-brute":
        sphere = generate(_gen_sphere, 1, args.workers)
        fast = generate(_gen_fast, 256, args.workers)
    else:
        gen = {"robust-p2p-100k": (_gen_sphere, 8), "fast-icp-4096": (_gen_fast, 1)}
        if args.workload == "robust-p2pl-500k":
            from paper_2007_07627_amd import synth
            single = [synth.height_field_pair(synth.rng_for(3, 0))]
        else:
            fn, cnt = gen[args.workload]
            single = generate(fn, cnt, args.workers)
    log(f"inputs generated in {time.perf_counter() - t0:.1f} s")

    import torch

    from paper_2007_07627_amd import binding as B
    if args.copy_calibration:
        copy_calibration(torch)

    if args.workload == "nn-brute":
        # the exhaustive closest-point kernels alone (one-slot at 100k x 100k,
        # multi-slot over 256 pairs of 4096 x 4096)
        one = brute_roofline(B, torch, sphere[0])
        multi = brute_batch_roofline(B, fast)
        out = {"metric": "exhaustive closest-point pairs/s", "value": one["pairs_per_s"], "unit": "pairs/s",
               "n_gpus": 1, "steps": 5, "warmup": 1, "ms_per_step": one["ms_per_launch"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
               "data": DATA, "config": {"workload": "exhaustive closest point, 100k x 100k bumpy sphere "
                                                    "pair; then 256 Fast ICP pairs of 4096 x 4096"},
               "nn_brute_roofline": one, "nn_brute_batch_roofline": multi}
        print(json.dumps(out), flush=True)
        return

    if args.workload != "batch-256":
        prms, cfg = single_workload(args.workload, B, single)
        r = single_pair_bench(args, B, torch, single, prms, cfg, args.workload, args.steps, args.warmup)
        out = {"metric": METRIC, "value": r["value"], "unit": "registrations/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE,
               "data": DATA}
        out.update({k: v for k, v in r.items() if k not in ("value", "unit", "steps", "ms_per_step")})
        print(json.dumps(out), flush=True)
        return

    log(f"workload batch-256: {len(pairs)} pairs")
    if args.counter_run:
        counter_run(B, torch, pairs, args.passes_per_replay)
        return
    out, info = batch_bench(args, B, pairs)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a sample of the batch)")
        out["cpu_baseline"] = cpu_baseline_batch(pairs, info["passes"], args.cpu_budget)
    if not args.no_serve:
        out["serve"] = serve_bench(args, B, pool)
    if not args.no_secondary:
        log("robust-p2p-100k (one pair at a time)")
        prms, cfg = single_workload("robust-p2p-100k", B, sphere)
        out["robust_p2p_100k"] = single_pair_bench(args, B, torch, sphere, prms, cfg, "robust-p2p-100k",
                                                   8, 2)
        log("exhaustive kernel at 100k x 100k")
        out["nn_brute_roofline"] = brute_roofline(B, torch, sphere[0])
        log("exhaustive kernel over 256 pairs of 4096 x 4096")
        out["nn_brute_batch_roofline"] = brute_batch_roofline(B, fast)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

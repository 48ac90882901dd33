"""Tune the closest-point work partition for the size buckets of the
registration workloads on this GPU and write the cache that icp_create
loads (tuning_<arch>.json beside libicp.so).

    python -m paper_2007_07627_amd.autotune [--out PATH] [--only M:N:MODE:METHOD:BATCH ...]

--only tunes just the listed shapes (sizes, icp_mode, icp_nn_method, engine
kind) and merges them into the existing cache.

Buckets are (floor(log2 M), floor(log2 N)); the library's lookup takes the
nearest tuned bucket within two octaves. The batch engine's kind is tuned
over every other octave of the uneven batch's [2k, 200k] sizes (both mode
families) and of the served stream's [1k, 1M] sizes (point-to-plane); the
synchronous kind over a coarser grid plus the single-pair workloads' own
buckets.
"""
from __future__ import annotations

import argparse
import os
import time

from paper_2007_07627_amd import binding as B

P2P, P2PL = B.ICP_P2P_WELSCH, B.ICP_P2PL_WELSCH


def buckets():
    out = []
    for mb in (11, 13, 15, 17):
        for nb in (11, 13, 15, 17):
            out += [(mb, nb, P2P, 1), (mb, nb, P2PL, 1)]
    for mb in (10, 12, 14, 16, 18, 19):
        for nb in (10, 12, 14, 16, 18, 19):
            out.append((mb, nb, P2PL, 1))
    for mb in (11, 14, 17):
        for nb in (11, 14, 17):
            out += [(mb, nb, P2P, 0), (mb, nb, P2PL, 0)]
    out += [(12, 12, P2P, 0), (16, 16, P2P, 0), (17, 18, P2PL, 0)]
    # the exhaustive search at the 100k x 100k shape, requested explicitly
    out.append((16, 16, P2P, 0, B.ICP_NN_BRUTE))
    seen, res = set(), []
    for b in out:
        if b not in seen:
            seen.add(b)
            res.append(b)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--only", nargs="*", default=None)
    args = ap.parse_args()
    arch = B.icp_device_arch(0)
    out = args.out or os.path.join(os.path.dirname(B.LIB_PATH), f"tuning_{arch}.json")
    ctx = B.icp_create(0, 48 << 30)
    t0 = time.perf_counter()
    jobs = []
    if args.only:
        for spec in args.only:
            M, N, mode, method, batch = (int(x) for x in spec.split(":"))
            jobs.append((M, N, mode, method, batch))
    else:
        for b in buckets():
            mb, nb, mode, batch = b[:4]
            # a representative size inside the bucket
            M, N = int(1.41 * (1 << mb)), int(1.41 * (1 << nb))
            method = b[4] if len(b) > 4 else (B.ICP_NN_BRUTE if M * N <= 64e6 else B.ICP_NN_CLUSTER)
            jobs.append((M, N, mode, method, batch))
    entries = []
    for M, N, mode, method, batch in jobs:
        e = B.icp_autotune(ctx, M, N, mode, method, batch)
        entries.append(e)
        print(f"[autotune] {'batch' if batch else 'sync '} {M:8d} x {N:8d} mode {mode} method {method}: "
              f"{B.tuning_dict(e.tuning)} {e.ms:.2f} ms ({time.perf_counter() - t0:.0f} s)", flush=True)
    if args.only:
        # the tuned shapes replace their buckets in the existing cache
        key = lambda e: (e.m_bucket, e.n_bucket, e.mode, e.method, e.batch)
        new = {key(e) for e in entries}
        old = [e for e in B.icp_tuning_file_read(out, arch) if key(e) not in new] if os.path.exists(out) else []
        entries = old + entries
    B.icp_tuning_file_write(out, arch, entries)
    B.icp_destroy(ctx)
    print(f"[autotune] {len(entries)} buckets -> {out}", flush=True)


if __name__ == "__main__":
    main()

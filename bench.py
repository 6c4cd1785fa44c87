"""Benchmark of the LVQ similarity hot path on one MI355X.

Default workload (the headline configuration): an LVQ-4x8 store in the Turbo
layout, inner product, n = 10^6 vectors of d = 768 (unit-normalised
anisotropic Gaussian), 10^4 float queries each with a fixed list of 1,000
distinct uniform candidate ids; one step = query precompute + similarities of
all 10^7 (query, candidate) pairs at the full (two-level) level + fused
per-list top-10.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LVQ distances/s + HBM GB/s vs peak; QPS and p99 at 10-recall@10≥0.9"
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "k_cand_c2_full_traffic.md")
KERNEL_SOURCES = ["paper_2402_02044_amd/csrc/k_cand_impl.h", "paper_2402_02044_amd/csrc/k_common.h",
                  "paper_2402_02044_amd/csrc/k_cand_inst.h"]


def log(*a):
    print("[bench %.1fs]" % (time.time() - T0), *a, file=sys.stderr, flush=True)


T0 = time.time()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(launch_pairs: int, tile: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    vals = {}
    for line in open(PROFILE_TRAFFIC):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    try:
        if vals.get("kernel_source_sha") != kernel_source_hash():
            return None
        if int(vals["pairs_per_launch"]) != launch_pairs or int(vals["tile_shape"]) != tile:
            return None
        fetch = float(vals["fetch_kib_per_dispatch"]) * float(vals["fetch_scale"])
        write = float(vals["write_kib_per_dispatch"]) * float(vals["write_scale"])
        return (fetch + write) * 1024.0
    except (KeyError, ValueError):
        return None


def c2_inputs(n, nq, per):
    import synth
    log("generating %d x 768 base vectors, %d queries, %d candidates each" % (n, nq, per))
    X = synth.vectors("C2", synth.S_BASE, 0, n)
    Q = synth.vectors("C2", synth.S_QUERY, 0, nq)
    offs, ids = synth.candidate_lists(2, nq, n, length=per)
    mu = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    return X, Q, mu, offs, ids


def cpu_baseline_c2(X, Q, mu, offs, ids, level, budget_s=12.0):
    """The oracle (plain scalar C, binary64 distances) on a bounded sample of
    the same workload: the first queries' candidate lists, timed on one core."""
    import oracle
    fmt = oracle.Format(768, 4, 8, oracle.TURBO)
    lvl = oracle.FULL if level == 2 else oracle.PRIMARY

    def run(nq_s):
        e = int(offs[nq_s])
        sub_ids = ids[:e]
        uniq, inv = np.unique(sub_ids, return_inverse=True)
        rows, resid, _ = oracle.encode_rows(fmt, X[uniq], mu)
        t = time.perf_counter()
        oracle.distances(fmt, oracle.IP, lvl, Q[:nq_s], rows, resid, mu, offs[:nq_s + 1],
                         inv.astype(np.int32))
        return time.perf_counter() - t, e

    dt, e = run(4)
    nq_s = int(min(len(offs) - 1, max(4, 4 * budget_s / max(dt, 1e-6))))
    dt, e = run(nq_s)
    return {"value": e / dt, "unit": "distances/s", "cores": 1, "kind": "oracle",
            "sample": "%d queries x %d candidates (%d pairs) of the same workload, %s level, "
                      "binary64 scalar C on one host core, %.1f s" %
                      (nq_s, int(offs[1] - offs[0]), e, "full" if level == 2 else "primary", dt)}


def bench_c2(args):
    import torch

    import paper_2402_02044_amd as L
    n, nq, per = args.n, args.nq, 1000
    X, Q, mu, offs, ids = c2_inputs(n, nq, per)
    level = L.LVQ_FULL if args.level == "full" else L.LVQ_PRIMARY
    dev = torch.device("cuda:0")
    log("uploading and encoding the store")
    ix = L.Index(768, 4, 8, L.LVQ_IP, L.LVQ_TURBO, align=args.align, capacity=n, means=mu)
    xd = torch.from_numpy(X).to(dev)
    ix.insert(xd)
    del xd
    qd = torch.from_numpy(Q).to(dev)
    od = torch.from_numpy(offs).to(dev)
    idd = torch.from_numpy(ids).to(dev)
    dist = torch.empty(ids.shape[0], dtype=torch.float32, device=dev)
    ti = torch.empty((nq, 10), dtype=torch.int32, device=dev)
    td = torch.empty((nq, 10), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    s = int(stream.cuda_stream)

    def step():
        L.lvq_distances(ix.handle, qd.data_ptr(), nq, od.data_ptr(), idd.data_ptr(), ids.shape[0], level,
                        dist.data_ptr(), 10, ti.data_ptr(), td.data_ptr(), s)

    rc = ix.sync()
    assert rc == 0, L.lvq_strerror(rc)
    if args.tile >= 0:
        ix.set_tile(level, 1, args.tile)
        tile = args.tile
    else:
        tile = ix.use_tuned_tile(level, 10, qd, od, idd, retune=args.retune)
        log("tile shape %d (%s)" % (tile, "autotuned" if args.retune else "tuning cache or autotuner"))
    log("warmup %d steps" % args.warmup)
    for _ in range(args.warmup):
        step()
    assert ix.sync() == 0
    ix.set_timing(True)
    ix.kernel_time()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, launches = ix.kernel_time()
    ix.set_timing(False)
    assert ix.sync() == 0
    ms_step = wall * 1000.0 / args.steps
    pairs = int(ids.shape[0])
    value = pairs / (ms_step / 1000.0)
    k_avg_ms = kms / max(launches, 1)
    per_pair = (384 + 768 + 12 + 4 + 4) if level == L.LVQ_FULL else (384 + 8 + 4 + 4)
    alg_bytes = per_pair * pairs
    achieved = alg_bytes / (k_avg_ms / 1000.0) / 1e9
    traffic = read_traffic(pairs, tile) if level == L.LVQ_FULL and args.align == 32 else None
    log("step %.3f ms, kernel %.3f ms, %.1f GB/s algorithmic" % (ms_step, k_avg_ms, achieved))
    out = {
        "metric": METRIC, "value": value, "unit": "distances/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "LVQ-4x8 Turbo inner product, n=1,000,000, d=768, 10,000 queries x "
                               "1,000 candidates, %s level, distances + per-list top-10" % args.level,
                   "n": n, "dim": 768, "bits": "4x8", "layout": "turbo", "row_align": args.align,
                   "queries": nq, "candidates_per_query": per, "k": 10, "level": args.level,
                   "tile_shape": tile},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_cand (candidate-list similarity + fused top-k)",
                     "kernel_ms": k_avg_ms, "algorithmic_bytes_per_pair": per_pair},
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on a host-core sample")
        out["cpu_baseline"] = cpu_baseline_c2(X, Q, mu, offs, ids, level)
    ix.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=["c2"])
    ap.add_argument("--level", default="full", choices=["full", "primary"])
    ap.add_argument("--align", type=int, default=32)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--nq", type=int, default=10_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", type=int, default=-1, help="fixed tile shape (default: tuning cache, else autotune)")
    ap.add_argument("--retune", action="store_true", help="run the autotuner even when the cache has a shape")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each GPU would run the same "
              "kernels on its share of the queries); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        n = 1 << 28
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": n * 4, "copy_bytes_written_per_launch": n * 4,
                          "launches": 5}), flush=True)
        return
    out = bench_c2(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmarks of the LVQ hot path on one MI355X.

Default workload (the headline configuration, `--workload c2`): an LVQ-4x8
store in the Turbo layout, inner product, n = 10^6 vectors of d = 768
(unit-normalised anisotropic Gaussian), 10^4 float queries each with a fixed
list of 1,000 distinct uniform candidate ids; one step = query precompute +
similarities of all 10^7 (query, candidate) pairs at the full (two-level)
level + fused per-list top-10.  Inputs are resident in HBM before the timed
region.

Other workloads (each prints its own line): c1 (LVQ-8 encode + exhaustive L2
top-10, n = 10^4, d = 96), c3 (multi-means LVQ-8, L2, n = 10^7, d = 96, uneven
lists in one persistent launch replayed from a HIP graph), c4 (exhaustive
inner-product top-100 over n = 5 * 10^6, d = 512 LVQ-8 on the matrix cores with
bf16, fp16 and FP32 queries), c5scan (the serving store's exhaustive
both-level top-10 alone: 10^6 LVQ-4x8 rows of d = 768 with 16 means, a batch
of 2,048 queries in each precision).

Prints one JSON line per workload.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import glob
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
MFMA_BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["paper_2402_02044_amd/csrc/k_cand_impl.h", "paper_2402_02044_amd/csrc/k_common.h",
                  "paper_2402_02044_amd/csrc/k_cand_inst.h"]
T0 = time.time()


def log(*a):
    print("[bench %.1fs]" % (time.time() - T0), *a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(stem: str, launch_pairs: int, tile: int):
    """HBM bytes per launch from a committed rocprofv3 counter summary
    (profiles/<stem>*.md) taken on the current kernel source, this many pairs
    per launch and this tile shape (else None)."""
    for path in sorted(glob.glob(os.path.join(PROFILES, stem + "*.md"))):
        got = read_traffic_file(path, launch_pairs, tile)
        if got is not None:
            return got
    return None


def read_traffic_file(path, launch_pairs: int, tile: int):
    if not os.path.exists(path):
        return None
    vals = {}
    for ln in open(path):
        if ":" in ln and ln.strip().startswith("- "):
            k, v = ln.strip()[2:].split(":", 1)
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


def line(value, unit, steps, warmup, ms_step, dtype, config, roofline, higher=True, **extra):
    out = {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": ms_step, "higher_is_better": higher, "scaling": "weak", "vs_baseline": None,
           "dtype": dtype, "data": "synthetic", "config": config, "roofline": roofline}
    out.update(extra)
    return out


def exact_topk(metric, Q, X, k, live=None, chunk=1 << 20):
    """Exact top-k over the float vectors (the ground truth of the k-recall@k
    measure, Sec. 2.1): binary64 products on the GPU, chunk by chunk.  Returns
    nq x k slot indices, best first."""
    import torch
    dev = torch.device("cuda:0")
    q = torch.from_numpy(np.asarray(Q, np.float64)).to(dev)
    qq = (q * q).sum(1, keepdim=True)
    slots = np.arange(X.shape[0]) if live is None else np.flatnonzero(live)
    bv = bi = None
    for a in range(0, slots.shape[0], chunk):
        sl = slots[a:a + chunk]
        x = torch.from_numpy(np.asarray(X[sl], np.float64)).to(dev)
        ip = q @ x.T
        v = -ip if metric == 1 else qq - 2.0 * ip + (x * x).sum(1)[None, :]
        v, i = torch.topk(v, min(k, v.shape[1]), dim=1, largest=False)
        i = torch.from_numpy(sl).to(dev)[i]
        if bv is not None:
            v = torch.cat([bv, v], 1)
            i = torch.cat([bi, i], 1)
            v, o = torch.topk(v, k, dim=1, largest=False)
            i = torch.gather(i, 1, o)
        bv, bi = v, i
    return bi.cpu().numpy()


def recall_at_k(found, truth) -> float:
    """k-recall@k: |returned ∩ true top-k| / k, averaged over queries."""
    found, truth = np.asarray(found), np.asarray(truth)
    k = truth.shape[1]
    return sum(len(set(found[i].tolist()) & set(truth[i].tolist())) for i in range(truth.shape[0])) / float(
        k * truth.shape[0])


def read_ceilings(ix, ids_dev, n_ids, level, per_pair, kernel_ms, reps=10):
    """The library's bandwidth probes beside a candidate-kernel measurement:
    a coalesced streaming read of 4 GiB, and the kernel's own gather (the same
    slots in the same order, the same bytes per slot, no arithmetic); median
    of `reps` launches timed with HIP events on the current stream."""
    import torch

    import paper_2402_02044_amd as L
    dev = ids_dev.device
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    s = int(torch.cuda.current_stream().cuda_stream)

    def med(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    nbytes = 1 << 32
    buf = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    st_ms = med(lambda: L.lvq_bw_stream(buf.data_ptr(), nbytes, sink.data_ptr(), s))
    del buf
    g_ms = med(lambda: L.lvq_bw_gather(ix.handle, ids_dev.data_ptr(), n_ids, level, sink.data_ptr(), s))
    assert ix.sync() == 0
    return {"stream_read_GBs": nbytes / (st_ms / 1000.0) / 1e9,
            "gather_ms": g_ms, "gather_GBs_algorithmic": per_pair * n_ids / (g_ms / 1000.0) / 1e9,
            "kernel_frac_of_gather": g_ms / kernel_ms,
            "probes": "lvq_bw_stream over 4 GiB; lvq_bw_gather over the kernel's candidate slots"}


def timed(step, steps, warmup, ix):
    """Wall time per step (synchronised on both sides) and the average kernel
    time of the main similarity kernel (HIP events on its stream)."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ix.set_timing(True)
    ix.kernel_time()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, launches = ix.kernel_time()
    ix.set_timing(False)
    return wall * 1000.0 / steps, (kms / launches if launches else None)


def to_gpu_rows(ix, X, dev, chunk=1 << 20):
    """Insert X in chunks; returns the milliseconds of the encode-and-insert
    calls alone (HIP events on the current stream around each call, uploads
    excluded)."""
    import torch
    # the first launch of a kernel loads its code object: warm the encoder on
    # a few vectors (pure encode, same kernel) before timing
    w = torch.from_numpy(X[:64]).to(dev)
    ix.encode(w)
    torch.cuda.synchronize()
    ms = 0.0
    for a in range(0, X.shape[0], chunk):
        xd = torch.from_numpy(X[a:a + chunk]).to(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ix.insert(xd)
        e1.record()
        e1.synchronize()
        ms += e0.elapsed_time(e1)
    return ms


def warm_encode_ms(ix, X, dev, chunk=1 << 20):
    """Milliseconds to encode all of X in steady state: lvq_encode of the
    first chunk into output buffers already touched (one warm-up, best of
    three), scaled to len(X)."""
    import torch
    m = min(chunk, X.shape[0])
    xd = torch.from_numpy(X[:m]).to(dev)
    ix.encode(xd)
    best = float("inf")
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ix.encode(xd)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del xd
    return best * X.shape[0] / m


# FP32 vector lane-operations per second: 256 CUs x 64 lanes x 2.4 GHz (one
# operation per lane and cycle; FMA would count twice in the 78.6 TFLOP/s figure)
VALU_LANE_OPS = 256 * 64 * 2.4e9


def encode_roofline(ms, n, dim, row_bytes, resid_bytes, insert_ms=None, n_means=1):
    """k_encode against the HBM roofline: reads 4d bytes and writes a row and
    a residual row per vector.  ms: steady-state encode time of n vectors;
    insert_ms: the store build (lvq_insert into slots never written before).
    With several means the exact nearest-mean search (a subtraction, a
    product and a sum per mean and dimension, in order) bounds it as well."""
    per = 4 * dim + row_bytes + resid_bytes
    gbs = per * n / (ms / 1000.0) / 1e9
    out = {"kernel": "k_encode", "ms": ms, "vectors": n, "bytes_per_vector": per,
           "achieved_GBs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
    if n_means > 1:
        ops = 3.0 * n_means * dim
        alu_ms = ops * n / VALU_LANE_OPS * 1000.0
        out.update({"nearest_mean_lane_ops_per_vector": ops, "alu_bound_ms": alu_ms,
                    "frac_of_alu_bound": alu_ms / ms})
    if insert_ms is not None:
        out["insert_ms_cold"] = insert_ms
    return out


def host_kmeans(S, k, iters, seed_workload, seed_chunk=1):
    """Lloyd's k-means in binary64 on a sample (harness input for M-LVQ):
    k distinct sample points as the start, `iters` rounds of nearest-centre
    assignment and centroid update (an empty cluster keeps its centre)."""
    import synth
    g = synth.rng(seed_workload, synth.S_SAMPLE, seed_chunk)
    Sd = S.astype(np.float64)
    C = Sd[g.choice(S.shape[0], k, replace=False)]
    sq = (Sd * Sd).sum(1)
    for _ in range(iters):
        d2 = sq[:, None] - 2.0 * Sd @ C.T + (C * C).sum(1)[None, :]
        a = d2.argmin(1)
        onehot = np.zeros((S.shape[0], k))
        onehot[np.arange(S.shape[0]), a] = 1.0
        cnt = onehot.sum(0)
        sums = onehot.T @ Sd
        nz = cnt > 0
        C[nz] = sums[nz] / cnt[nz, None]
    return C.astype(np.float32)


# ---------------------------------------------------------------------------
# C2: candidate lists, LVQ-4x8 Turbo, inner product (the headline)
# ---------------------------------------------------------------------------

def c2_inputs(n, nq, per):
    import synth
    log("generating %d x 768 base vectors, %d queries, %d candidates each" % (n, nq, per))
    X = synth.vectors("C2", synth.S_BASE, 0, n)
    Q = synth.vectors("C2", synth.S_QUERY, 0, nq)
    offs, ids = synth.candidate_lists(2, nq, n, length=per)
    mu = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    return X, Q, mu, offs, ids


def cpu_baseline_lists(fmt, metric, level, X, Q, means, offs, ids, budget_s=12.0):
    """The oracle (plain scalar C, binary64 similarities) on a bounded sample of
    the same workload: the first queries' candidate lists, on one host core."""
    import oracle

    def run(nq_s):
        e = int(offs[nq_s])
        uniq, inv = np.unique(ids[:e], return_inverse=True)
        rows, resid, _ = oracle.encode_rows(fmt, X[uniq], means)
        inv = inv.astype(np.int32)
        t = time.perf_counter()
        ref = oracle.distances(fmt, metric, level, Q[:nq_s], rows, resid, means, offs[:nq_s + 1], inv)
        return time.perf_counter() - t, e, (rows, resid, inv), ref

    dt, e, _, _ = run(4)
    # as many leading lists as fit the time budget at the measured rate per pair
    want = min(budget_s * max(e, 1) / max(dt, 1e-6), 4e6)
    nq_s = int(min(len(offs) - 1, max(4, np.searchsorted(offs, want) - 1)))
    dt, e, enc, ref = run(nq_s)
    out = {"value": e / dt, "unit": "distances/s", "cores": 1, "kind": "oracle",
           "sample": "first %d queries' candidate lists (%d pairs) of the same workload, %s level, "
                     "binary64 scalar C on one host core, %.1f s" %
                     (nq_s, e, "full" if level == 2 else "primary", dt)}
    out["all_cores"] = cpu_baseline_threads(fmt, metric, level, Q, means, offs, nq_s, enc)
    return out, (nq_s, enc, ref)


def sample_parity(fmt, metric, level, Q, means, offs, ids, sample, dist, topk_ids, topk_dist, k):
    """The timed launch's outputs on the oracle's sample (the first queries'
    lists, values the CPU baseline computed): every value within the test
    suite's tolerance of the oracle's, every top-k list equal to the oracle's
    up to near-ties."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle
    from lvq_check import check_topk, pair_tolerance
    nq_s, (rows, resid, inv), ref = sample
    e = int(offs[nq_s])
    xh = oracle.reconstruct(fmt, rows, resid, means, level)
    mrow = np.asarray(means, np.float64)[oracle.unpack(fmt, rows)[3]]
    qi = np.repeat(np.arange(nq_s), np.diff(offs[:nq_s + 1]))
    tol = np.empty(e)
    for a in range(0, e, 1 << 16):
        c = slice(a, a + (1 << 16))
        tol[c] = pair_tolerance(metric, Q, xh[inv[c]], mrow[inv[c]], qi[c])
    got = np.asarray(dist[:e], np.float64)
    ratio = np.abs(got - ref) / np.maximum(tol, 1e-300)
    bad_topk = 0
    for i in range(nq_s):
        a, b = int(offs[i]), int(offs[i + 1])
        try:
            check_topk(metric, topk_ids[i], topk_dist[i], ids[a:b], ref[a:b], tol[a:b], k)
        except AssertionError:
            bad_topk += 1
    ok = bool(np.all(np.abs(got - ref) <= tol)) and bad_topk == 0
    return {"pairs_checked": e, "lists_checked": nq_s, "max_err_over_tolerance": float(ratio.max()),
            "topk_lists_failed": bad_topk, "ok": ok,
            "note": "the timed launch's values and top-%d lists on the oracle's sample, tolerance of "
                    "tests/lvq_check.py" % k}


def host_cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_threads(fmt, metric, level, Q, means, offs, nq_s, enc):
    """The same oracle sample (its encoded rows in `enc`) split over host
    threads: one query range per thread; the C calls run without the
    interpreter lock."""
    import threading

    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    e = int(offs[nq_s])
    rows, resid, inv = enc
    bounds = np.linspace(0, nq_s, threads + 1).astype(int)

    def work(a, b):
        o = offs[a:b + 1] - offs[a]
        oracle.distances(fmt, metric, level, Q[a:b], rows, resid, means, o, inv[offs[a]:offs[b]])

    ts = [threading.Thread(target=work, args=(int(bounds[t]), int(bounds[t + 1]))) for t in range(threads)
          if bounds[t + 1] > bounds[t]]
    t0 = time.perf_counter()
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    dt = time.perf_counter() - t0
    return {"value": e / dt, "unit": "distances/s", "cores": len(ts), "cpu_model": host_cpu_model(),
            "sample": "the same %d queries split over %d host threads, %.2f s" % (nq_s, len(ts), dt)}


def bench_c2(args):
    import torch

    import paper_2402_02044_amd as L
    n, nq, per = args.n or 1_000_000, args.nq or 10_000, 1000
    X, Q, mu, offs, ids = c2_inputs(n, nq, per)
    level = L.LVQ_FULL if args.level == "full" else L.LVQ_PRIMARY
    dev = torch.device("cuda:0")
    log("uploading and encoding the store")
    ix = L.Index(768, 4, 8, L.LVQ_IP, L.LVQ_TURBO, align=args.align, capacity=n, means=mu)
    enc_ms = to_gpu_rows(ix, X, dev)
    qd = torch.from_numpy(Q).to(dev)
    od = torch.from_numpy(offs).to(dev)
    idd = torch.from_numpy(ids).to(dev)
    dist = torch.empty(ids.shape[0], dtype=torch.float32, device=dev)
    ti = torch.empty((nq, 10), dtype=torch.int32, device=dev)
    td = torch.empty((nq, 10), dtype=torch.float32, device=dev)
    s = int(torch.cuda.current_stream().cuda_stream)

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
    log("tile shape %d; warmup %d, timing %d steps" % (tile, args.warmup, args.steps))
    ms_step, k_ms = timed(step, args.steps, args.warmup, ix)
    assert ix.sync() == 0
    pairs = int(ids.shape[0])
    # codes (+ residual codes) + l, Delta + slot id read + value written
    per_pair = (384 + 768 + 8 + 4 + 4) if level == L.LVQ_FULL else (384 + 8 + 4 + 4)
    achieved = per_pair * pairs / (k_ms / 1000.0) / 1e9
    traffic = read_traffic("k_cand_c2_%s_traffic" % args.level, pairs, tile) if args.align == 32 else None
    log("step %.3f ms, kernel %.3f ms, %.1f GB/s algorithmic" % (ms_step, k_ms, achieved))
    ceil = read_ceilings(ix, idd, pairs, level, per_pair, k_ms)
    log("streaming read %.0f GB/s; the same gather without arithmetic %.3f ms (kernel at %.0f%% of it)" %
        (ceil["stream_read_GBs"], ceil["gather_ms"], 100.0 * ceil["kernel_frac_of_gather"]))
    out = line(pairs / (ms_step / 1000.0), "distances/s", args.steps, args.warmup, ms_step, "f32",
               {"workload": "LVQ-4x8 Turbo inner product, n=1,000,000, d=768, 10,000 queries x 1,000 "
                            "candidates, %s level, distances + per-list top-10" % args.level,
                "n": n, "dim": 768, "bits": "4x8", "layout": "turbo", "row_align": args.align, "queries": nq,
                "candidates_per_query": per, "k": 10, "level": args.level, "tile_shape": tile},
               {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "k_cand (candidate-list similarity + fused top-k)", "kernel_ms": k_ms,
                "algorithmic_bytes_per_pair": per_pair, "ceilings": ceil},
               encode=encode_roofline(warm_encode_ms(ix, X, dev), n, 768, ix.row_bytes, ix.resid_bytes, enc_ms))
    dist_h, ti_h, td_h = dist.cpu().numpy(), ti.cpu().numpy(), td.cpu().numpy()
    ix.close()
    del qd, od, idd, dist, ti, td
    if not args.no_cpu_baseline:
        import oracle
        log("timing the oracle on a host-core sample")
        fmt = oracle.Format(768, 4, 8, oracle.TURBO)
        out["cpu_baseline"], sample = cpu_baseline_lists(fmt, oracle.IP, level, X, Q, mu, offs, ids)
        out["parity"] = sample_parity(fmt, oracle.IP, level, Q, mu, offs, ids, sample, dist_h, ti_h, td_h, 10)
        log("parity on the oracle sample: %s" % json.dumps(out["parity"]))
    del X
    if args.serving:
        out["serving"] = serving_summary(args)
    return out


# ---------------------------------------------------------------------------
# C1: LVQ-8 encode + exhaustive L2 top-10, n = 10^4, d = 96
# ---------------------------------------------------------------------------

def bench_c1(args):
    import torch

    import paper_2402_02044_amd as L
    import synth
    n, nq, d = 10_000, 100, 96
    X = synth.vectors("C1", synth.S_BASE, 0, n)
    Q = synth.vectors("C1", synth.S_QUERY, 0, nq)
    mu = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    dev = torch.device("cuda:0")
    ix = L.Index(d, 8, 0, L.LVQ_L2, L.LVQ_SEQUENTIAL, capacity=n, means=mu)
    xd = torch.from_numpy(X).to(dev)
    ix.insert(xd)
    qd = torch.from_numpy(Q).to(dev)
    rows = torch.empty((n, ix.row_bytes), dtype=torch.uint8, device=dev)
    ids = torch.empty((nq, 10), dtype=torch.int32, device=dev)
    dist = torch.empty((nq, 10), dtype=torch.float32, device=dev)
    s = int(torch.cuda.current_stream().cuda_stream)

    def step():
        L.lvq_encode(ix.handle, xd.data_ptr(), n, rows.data_ptr(), 0, s)
        L.lvq_topk(ix.handle, qd.data_ptr(), L.LVQ_FP32, nq, 10, L.LVQ_PRIMARY, ids.data_ptr(), dist.data_ptr(), s)

    ms_step, k_ms = timed(step, args.steps * 10, args.warmup, ix)
    assert ix.sync() == 0
    rec = recall_at_k(ids.cpu().numpy(), exact_topk(0, Q, X, 10))
    flops = 3.0 * d * n * nq          # subtract, multiply, add per (pair, dim)
    achieved = flops / (k_ms / 1000.0) / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        fmt = oracle.Format(d, 8, 0)
        orows, _, _ = oracle.encode_rows(fmt, X, mu)
        t = time.perf_counter()
        oracle.topk_exhaustive(fmt, oracle.L2, oracle.PRIMARY, Q, orows, None, mu, 10)
        ct = time.perf_counter() - t
        cpu = {"value": n * nq / ct, "unit": "distances/s", "cores": 1, "kind": "oracle",
               "sample": "all 100 queries x 10,000 rows, binary64 scalar C, %.2f s" % ct}
    out = line(n * nq / (ms_step / 1000.0), "distances/s", args.steps * 10, args.warmup, ms_step, "f32",
               {"workload": "LVQ-8 encode of 10,000 x 96 vectors (32 Gaussian clusters) + exhaustive L2 top-10 "
                            "of 100 queries", "n": n, "dim": d, "queries": nq, "k": 10},
               {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None, "kernel": "k_scan (FP32 exhaustive top-k)",
                "kernel_ms": k_ms, "note": "store of 1.28 MB is cache resident: latency-bound, not a roofline claim"},
               recall_at_10=rec)
    if cpu:
        out["cpu_baseline"] = cpu
    ix.close()
    return out


# ---------------------------------------------------------------------------
# C3: multi-means LVQ-8, L2, n = 10^7, d = 96, uneven lists, one persistent
# launch replayed from a HIP graph
# ---------------------------------------------------------------------------

def bench_c3(args):
    import torch

    import paper_2402_02044_amd as L
    import synth
    n, nq, d, M = args.n or 10_000_000, args.nq or 10_000, 96, 16
    log("generating %d x %d base vectors (256 clusters), %d queries" % (n, d, nq))
    X = synth.vectors("C3", synth.S_BASE, 0, n)
    Q = synth.vectors("C3", synth.S_QUERY, 0, nq)
    sample = X[synth.sample_indices(3, n, 100_000)]
    log("k-means (M = %d) on a 100k sample" % M)
    means = host_kmeans(sample, M, 25, 3)
    offs, ids = synth.candidate_lists(3, nq, n, lmin=64, lmax=4096)
    dev = torch.device("cuda:0")
    log("uploading and encoding the store (%d lists, %d pairs)" % (nq, ids.shape[0]))
    ix = L.Index(d, 8, 0, L.LVQ_L2, L.LVQ_SEQUENTIAL, capacity=n, means=means)
    enc_ms = to_gpu_rows(ix, X, dev)
    qd = torch.from_numpy(Q).to(dev)
    od = torch.from_numpy(offs).to(dev)
    idd = torch.from_numpy(ids).to(dev)
    dist = torch.empty(ids.shape[0], dtype=torch.float32, device=dev)
    ti = torch.empty((nq, 10), dtype=torch.int32, device=dev)
    td = torch.empty((nq, 10), dtype=torch.float32, device=dev)
    assert ix.sync() == 0
    if args.tile >= 0:
        ix.set_tile(L.LVQ_PRIMARY, 1, args.tile)
        tile = args.tile
    else:
        tile = ix.use_tuned_tile(L.LVQ_PRIMARY, 10, qd, od, idd, retune=args.retune)
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())

    def call(stream):
        L.lvq_distances(ix.handle, qd.data_ptr(), nq, od.data_ptr(), idd.data_ptr(), ids.shape[0], L.LVQ_PRIMARY,
                        dist.data_ptr(), 10, ti.data_ptr(), td.data_ptr(), int(stream.cuda_stream))

    with torch.cuda.stream(cs):
        call(cs)
    torch.cuda.synchronize()
    ms_eager, k_ms = timed(lambda: call(torch.cuda.current_stream()), args.steps, args.warmup, ix)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=cs):
        call(cs)
    ms_graph, _ = timed(graph.replay, args.steps, args.warmup, ix)
    assert ix.sync() == 0
    pairs = int(ids.shape[0])
    per_pair = 96 + 8 + 1 + 4 + 4
    achieved = per_pair * pairs / (k_ms / 1000.0) / 1e9
    log("eager step %.3f ms, graph step %.3f ms, kernel %.3f ms" % (ms_eager, ms_graph, k_ms))
    ceil = read_ceilings(ix, idd, pairs, L.LVQ_PRIMARY, per_pair, k_ms)
    log("streaming read %.0f GB/s; the same gather without arithmetic %.3f ms (kernel at %.0f%% of it)" %
        (ceil["stream_read_GBs"], ceil["gather_ms"], 100.0 * ceil["kernel_frac_of_gather"]))
    out = line(pairs / (ms_graph / 1000.0), "distances/s", args.steps, args.warmup, ms_graph, "f32",
               {"workload": "multi-means LVQ-8 L2, n=10,000,000, d=96 (256 clusters), 16 means (k-means on a "
                            "100k sample), 10,000 queries with log-uniform 64..4096 candidate lists, top-10, one "
                            "persistent launch per step, steps replayed from a HIP graph",
                "n": n, "dim": d, "means": M, "queries": nq, "pairs": pairs, "k": 10, "tile_shape": tile},
               {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel": "k_cand (persistent, longest lists first)", "kernel_ms": k_ms,
                "algorithmic_bytes_per_pair": per_pair, "ceilings": ceil},
               ms_per_step_eager=ms_eager)
    out["encode"] = encode_roofline(warm_encode_ms(ix, X, dev), n, d, ix.row_bytes, ix.resid_bytes, enc_ms, n_means=M)
    out["roofline"]["traffic"] = read_traffic("k_cand_c3_traffic", pairs, tile)
    # load balance inside a list: a workgroup scores blocks of 256 / lanes
    # candidates (lanes per candidate of the tile shape); the last block of a
    # list leaves the lanes past its end idle
    lanes = L.lvq_tile_shape(tile)[0]
    blk = 256 // lanes
    lens = np.diff(offs)
    out["load_balance"] = {"busy_lane_fraction": pairs / float((np.ceil(lens / blk) * blk).sum()),
                           "candidates_per_block": blk, "lists": nq,
                           "note": "listed pairs / lane slots of the blocks the lists occupy; lists are taken "
                                   "longest first from one work counter by the persistent workgroups"}
    dist_h, ti_h, td_h = dist.cpu().numpy(), ti.cpu().numpy(), td.cpu().numpy()
    if not args.no_cpu_baseline:
        import oracle
        fmt = oracle.Format(d, 8, 0)
        out["cpu_baseline"], sample = cpu_baseline_lists(fmt, oracle.L2, oracle.PRIMARY, X, Q, means, offs, ids)
        out["parity"] = sample_parity(fmt, oracle.L2, oracle.PRIMARY, Q, means, offs, ids, sample, dist_h, ti_h,
                                      td_h, 10)
        log("parity on the oracle sample: %s" % json.dumps(out["parity"]))
    ix.close()
    return out


# ---------------------------------------------------------------------------
# C4: exhaustive inner-product top-100, n = 5 * 10^6, d = 512, LVQ-8, MFMA
# ---------------------------------------------------------------------------

def bench_c4(args):
    import torch

    import paper_2402_02044_amd as L
    import synth
    n, nq, d, k = args.n or 5_000_000, args.nq or 10_000, 512, 100
    log("generating %d x %d base vectors, %d queries" % (n, d, nq))
    X = synth.vectors("C4", synth.S_BASE, 0, n)
    Q = synth.vectors("C4", synth.S_QUERY, 0, nq)
    mu = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    dev = torch.device("cuda:0")
    log("uploading and encoding the store")
    ix = L.Index(d, 8, 0, L.LVQ_IP, L.LVQ_SEQUENTIAL, capacity=n, means=mu)
    enc_ms = to_gpu_rows(ix, X, dev)
    assert ix.sync() == 0
    qf = torch.from_numpy(Q).to(dev)
    res = {}
    # fp32: FP32 on the matrix cores; fp32_plain: the plain FP32 vector kernel
    forms = [f for f in (("bf16", torch.bfloat16), ("fp16", torch.float16), ("fp32", torch.float32),
                         ("fp32_plain", torch.float32))
             if f[0] in args.forms.split(",")]
    for name, tdt in forms:
        q = qf.to(tdt)
        ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
        dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
        prec = {"bf16": L.LVQ_BF16, "fp16": L.LVQ_FP16, "fp32": L.LVQ_FP32, "fp32_plain": L.LVQ_FP32_VALU}[name]
        s = int(torch.cuda.current_stream().cuda_stream)

        def step():
            L.lvq_topk(ix.handle, q.data_ptr(), prec, nq, k, L.LVQ_PRIMARY, ids.data_ptr(), dist.data_ptr(), s)

        steps = {"fp32": max(1, args.steps // 4), "fp32_plain": max(1, args.steps // 15)}.get(name, args.steps)
        ms, k_ms = timed(step, steps, 1, ix)
        assert ix.sync() == 0
        res[name] = (ms, k_ms, ids.cpu().numpy(), dist.cpu().numpy())
        log("%s: step %.2f ms, kernel %.2f ms" % (name, ms, k_ms))
    # recall@100 of every form on a query sample against the exact float top-100
    ns = 100
    Qd = Q[:ns]
    gt = exact_topk(1, Qd, X, k)
    acc = {}
    for name, (ms, k_ms, ids, dist) in res.items():
        tf = 2.0 * d * n * nq / (k_ms / 1000.0) / 1e12
        peak = FP32_PEAK_TFLOPS if name.startswith("fp32") else MFMA_BF16_PEAK_TFLOPS
        acc[name] = {"recall_at_100": recall_at_k(ids[:ns], gt), "ms_per_step": ms, "kernel_ms": k_ms,
                     "distances_per_s": n * nq / (ms / 1000.0), "kernel_tflops": tf,
                     "frac_of_dense_peak": tf / peak, "peak_tflops": peak}
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on the host: returned values of every form against its
        # binary64 similarities (float32 queries), and its own rate on a slice
        import oracle
        fmt = oracle.Format(d, 8, 0)
        offs = np.arange(ns + 1, dtype=np.int64) * k
        for name, (ms, k_ms, ids, dist) in res.items():
            uniq, inv = np.unique(ids[:ns].ravel(), return_inverse=True)
            rows, _, _ = oracle.encode_rows(fmt, X[uniq], mu)
            ref = oracle.distances(fmt, oracle.IP, oracle.PRIMARY, Qd, rows, None, mu, offs, inv.astype(np.int32))
            xh = oracle.reconstruct(fmt, rows, None, mu)[inv]
            S = np.abs(np.repeat(Qd.astype(np.float64), k, 0) * xh).sum(1)
            err = np.abs(dist[:ns].ravel().astype(np.float64) - ref) / S
            acc[name]["max_err_over_S"] = float(err.max())
            acc[name]["mean_err_over_S"] = float(err.mean())
        # a sample of about ten seconds of the oracle on one host core
        m, nqs = 500_000, 8
        rows, _, _ = oracle.encode_rows(fmt, X[:m], mu)
        t = time.perf_counter()
        oracle.topk_exhaustive(fmt, oracle.IP, oracle.PRIMARY, Q[:nqs], rows, None, mu, k)
        ct = time.perf_counter() - t
        cpu = {"value": nqs * m / ct, "unit": "distances/s", "cores": 1, "kind": "oracle",
               "sample": "exhaustive top-100 of %d queries over the first %d rows, binary64 scalar C, %.2f s"
                         % (nqs, m, ct)}
    # the line's form: bf16 when it ran, else the first one that did
    main_form = "bf16" if "bf16" in res else next(iter(res))
    ms, k_ms = res[main_form][0], res[main_form][1]
    flops = 2.0 * d * n * nq
    achieved = flops / (k_ms / 1000.0) / 1e12
    peak = FP32_PEAK_TFLOPS if main_form.startswith("fp32") else MFMA_BF16_PEAK_TFLOPS
    out = line(n * nq / (ms / 1000.0), "distances/s", args.steps, 1, ms, main_form,
               {"workload": "exhaustive inner-product top-100 over n=5,000,000 d=512 LVQ-8 codes (anisotropic "
                            "unit vectors), 10,000 queries in bf16 on MFMA with FP32 accumulation; fp16, "
                            "FP32 queries on the FP32 MFMA, and the plain FP32 vector kernel on the same store",
                "n": n, "dim": d, "queries": nq, "k": k},
               {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None,
                "kernel": "k_scan_mfma_wide (%s, fused top-100)" % main_form, "kernel_ms": k_ms},
               precision=acc, accuracy_sample="%d queries: recall@100 vs the exact float top-100; errors "
                                              "|gpu - binary64 oracle (float32 query)| / sum_j |q_j x_hat_j| "
                                              "(with the CPU baseline)" % ns)
    out["encode"] = encode_roofline(warm_encode_ms(ix, X, dev), n, d, ix.row_bytes, ix.resid_bytes, enc_ms)
    if cpu:
        out["cpu_baseline"] = cpu
    ix.close()
    return out


# ---------------------------------------------------------------------------
# The both-level exhaustive scan at the serving store's shape, alone: 10^6
# LVQ-4x8 Turbo rows of d = 768 with 16 means, a batch of queries in each
# precision, top-10 (the kernel the C5 server runs per batch)
# ---------------------------------------------------------------------------

def bench_c5scan(args):
    import torch

    import paper_2402_02044_amd as L
    import synth
    n, nq, d, k = args.n or 1_000_000, args.nq or 2048, 768, 10
    dev = torch.device("cuda:0")
    log("generating %d x %d C5 vectors, 16 means" % (n, d))
    X = synth.vectors("C5", synth.S_BASE, 0, n)
    means = host_kmeans(X[synth.sample_indices(5, n, 100_000)], 16, 25, 5)
    ix = L.Index(d, 4, 8, L.LVQ_IP, L.LVQ_TURBO, capacity=n, means=means)
    to_gpu_rows(ix, X, dev)
    assert ix.sync() == 0
    Q = synth.c5_points(synth.S_QUERY, 1, nq, part=1)
    qf = torch.from_numpy(Q).to(dev)
    forms = [f for f in (("bf16", torch.bfloat16), ("fp16", torch.float16), ("fp32", torch.float32),
                         ("fp32_plain", torch.float32)) if f[0] in args.forms.split(",")]
    # flops the matrix cores execute per (query, row): the 16-bit forms take
    # <q, c1> and <q, c2> (two chains, 4d), the FP32 form <q, y> on decoded y
    # (2d); the plain vector kernel 2d FMAs on decoded y
    per_pair = {"bf16": 4 * d, "fp16": 4 * d, "fp32": 2 * d, "fp32_plain": 2 * d}
    res = {}
    for name, tdt in forms:
        q = qf.to(tdt)
        ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
        dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
        prec = {"bf16": L.LVQ_BF16, "fp16": L.LVQ_FP16, "fp32": L.LVQ_FP32, "fp32_plain": L.LVQ_FP32_VALU}[name]
        s = int(torch.cuda.current_stream().cuda_stream)

        def step():
            L.lvq_topk(ix.handle, q.data_ptr(), prec, nq, k, L.LVQ_FULL, ids.data_ptr(), dist.data_ptr(), s)

        steps = args.steps if name != "fp32_plain" else max(1, args.steps // 4)
        ms, k_ms = timed(step, steps, 1, ix)
        assert ix.sync() == 0
        tf = per_pair[name] * float(n) * nq / (k_ms / 1000.0) / 1e12
        peak = MFMA_BF16_PEAK_TFLOPS if name in ("bf16", "fp16") else FP32_PEAK_TFLOPS
        res[name] = {"ms_per_step": ms, "kernel_ms": k_ms, "queries_per_s": nq / (ms / 1000.0),
                     "kernel_tflops": tf, "frac_of_peak": tf / peak, "peak_tflops": peak,
                     "flops_per_pair": per_pair[name]}
        log("%s: step %.2f ms, kernel %.2f ms, %.1f TFLOP/s (%.3f of %.1f)" % (name, ms, k_ms, tf, tf / peak, peak))
    main_form = "bf16" if "bf16" in res else next(iter(res))
    r = res[main_form]
    out = line(r["queries_per_s"], "queries/s", args.steps, 1, r["ms_per_step"], main_form,
               {"workload": "exhaustive both-level inner-product top-%d of %d queries over n=%d d=%d LVQ-4x8 Turbo "
                            "rows with 16 means (the serving store), bf16 on MFMA; fp16, FP32 on the FP32 MFMA and "
                            "the plain FP32 vector kernel on the same store" % (k, nq, n, d),
                "n": n, "dim": d, "queries": nq, "k": k},
               {"bound": "mfma", "achieved": r["kernel_tflops"], "peak": r["peak_tflops"], "unit": "TFLOP/s",
                "frac": r["frac_of_peak"], "traffic": None,
                "kernel": "k_scan_mfma_wide (%s, both levels, fused top-%d)" % (main_form, k),
                "kernel_ms": r["kernel_ms"]},
               forms=res)
    ix.close()
    return out


# ---------------------------------------------------------------------------
# Mean re-estimation on the C5 stream (Sec. 3.2): the periodic re-fit (new
# means appended every 10 rounds, rows never re-encoded) against online
# updates (every round, each moved centre replaced and its rows re-encoded)
# ---------------------------------------------------------------------------

def bench_means(args):
    import torch

    import paper_2402_02044_amd as L
    import synth
    n0 = args.n or 1_000_000
    rounds = args.rounds
    ins = max(100, n0 // 100)
    dev = torch.device("cuda:0")
    X0 = synth.vectors("C5", synth.S_BASE, 0, n0)
    samp = synth.sample_indices(5, n0, 100_000)
    means = host_kmeans(X0[samp], 16, 25, 5)
    cap = 2 * n0 + 5 * ins + 4096
    thr = 0.05
    res = {}
    scan = []
    for policy in ("periodic", "online"):
        log("policy %s: encoding the store" % policy)
        st = C5Store(L, X0, means, cap, dev)
        torch.cuda.synchronize()
        rec = {"recall_at_10": [], "update_ms": [], "reencoded": [], "means_moved": [], "ids_in_use": []}
        for r in range(rounds):
            t = time.perf_counter()
            cand = np.flatnonzero(st.live)
            dead = np.sort(synth.rng(5, synth.S_DELETE, r).choice(cand, cand.size // 10, replace=False))
            st.delete(dead)
            st.insert(synth.c5_points(synth.S_INSERT, r + 1, ins))
            moved = reenc = 0
            if policy == "periodic":
                if (r + 1) % 10 == 0:
                    st.refit_means(r)
            else:
                moved, reenc = st.online_update(thr)
            st.consolidate()
            st.stream.synchronize()
            rec["update_ms"].append((time.perf_counter() - t) * 1000.0)
            rec["reencoded"].append(reenc)
            rec["means_moved"].append(moved)
            rec["ids_in_use"].append(st.n_ids if policy == "online" else st.n_means)
            Qr = synth.c5_points(synth.S_QUERY, r + 1, 200, part=0)
            q = torch.from_numpy(Qr).to(dev).to(torch.bfloat16)
            with torch.cuda.stream(st.stream):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                ids, _ = st.ix.topk(q, 10, level=L.LVQ_FULL, stream=st.stream)
                e1.record()
            st.stream.synchronize()
            scan.append(int(st.live.sum()) * Qr.shape[0] / (e0.elapsed_time(e1) / 1000.0))
            rec["recall_at_10"].append(recall_at_k(ids.cpu().numpy(), st.groundtruth(Qr)))
            log("%s round %d: recall %.3f, update %.0f ms, means moved %d, rows re-encoded %d" %
                (policy, r, rec["recall_at_10"][-1], rec["update_ms"][-1], moved, reenc))
        assert st.ix.sync() == 0
        r_ = np.array(rec["recall_at_10"])
        res[policy] = {"recall_at_10_mean": float(r_.mean()), "recall_at_10_min": float(r_.min()),
                       "recall_at_10_last10_mean": float(r_[-10:].mean()),
                       "update_ms_mean": float(np.mean(rec["update_ms"])),
                       "update_ms_max": float(np.max(rec["update_ms"])),
                       "rows_reencoded": int(np.sum(rec["reencoded"])), "ids_in_use_last": rec["ids_in_use"][-1],
                       "per_round": rec}
        st.ix.close()
        del st
        torch.cuda.empty_cache()
    out = line(float(np.mean(scan)), "distances/s", rounds, 0, res["online"]["update_ms_mean"], "bf16",
               {"workload": "C5 stream (n=1,000,000 d=768 LVQ-4x8 Turbo IP, 30 rounds of 10%% deletes, %d drifted "
                            "inserts and consolidation) under two mean policies; per round the exhaustive bf16 "
                            "both-level top-10 of 200 queries of the round's distribution" % ins,
                "n": n0, "dim": 768, "rounds": rounds, "online_threshold": thr},
               {"bound": "mfma", "achieved": None, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": None,
                "traffic": None, "kernel": "k_scan_mfma_wide (both levels); value: scan rate during the rounds"},
               policies=res)
    return out


# ---------------------------------------------------------------------------
# Soft inverted index (M-LVQ means as lists, Sec. 3.2): C3's data law with 256
# means; each query scores the members of its nprobe nearest means
# ---------------------------------------------------------------------------

def bench_probe(args):
    import torch

    import paper_2402_02044_amd as L
    import synth
    n, nq, d, M, k = args.n or 10_000_000, args.nq or 10_000, 96, 256, 10
    log("generating %d x %d base vectors (256 clusters), %d queries" % (n, d, nq))
    X = synth.vectors("C3", synth.S_BASE, 0, n)
    Q = synth.vectors("C3", synth.S_QUERY, 0, nq)
    sample = X[synth.sample_indices(3, n, 100_000)]
    log("k-means (M = %d) on a 100k sample" % M)
    means = host_kmeans(sample, M, 10, 3)
    dev = torch.device("cuda:0")
    log("uploading and encoding the store")
    ix = L.Index(d, 8, 0, L.LVQ_L2, L.LVQ_SEQUENTIAL, capacity=n, means=means)
    enc_ms = to_gpu_rows(ix, X, dev)
    tile = args.tile if args.tile >= 0 else 28
    ix.set_tile(L.LVQ_PRIMARY, 1, tile)
    # members per mean (header byte 12 of every row), for the pairs scanned
    sizes = torch.zeros(M, dtype=torch.int64, device=dev)
    for a in range(0, n, 1 << 20):
        sl = torch.arange(a, min(n, a + (1 << 20)), dtype=torch.int32, device=dev)
        rows, _ = ix.read_rows(sl)
        sizes += torch.bincount(rows[:, 12].long(), minlength=M)
    sizes = sizes.cpu().numpy()
    ns = 1000
    log("exact float top-%d of %d queries" % (k, ns))
    gt = exact_topk(0, Q[:ns], X, k)
    qd = torch.from_numpy(Q).to(dev)
    probe_buf = {}
    ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
    s = int(torch.cuda.current_stream().cuda_stream)
    points = []
    for nprobe in (1, 2, 4, 8):
        probe = probe_buf.setdefault(nprobe, torch.empty((nq, nprobe), dtype=torch.int32, device=dev))

        def step():
            L.lvq_probe_topk(ix.handle, qd.data_ptr(), nq, nprobe, k, L.LVQ_PRIMARY, probe.data_ptr(),
                             ids.data_ptr(), dist.data_ptr(), s)

        ms, k_ms = timed(step, args.steps, args.warmup, ix)
        assert ix.sync() == 0
        pairs = int(sizes[probe.cpu().numpy()].sum())
        rec = recall_at_k(ids[:ns].cpu().numpy(), gt)
        points.append({"nprobe": nprobe, "ms_per_batch": ms, "kernel_ms": k_ms, "qps": nq / (ms / 1000.0),
                       "pairs_per_query": pairs / nq, "distances_per_s": pairs / (ms / 1000.0),
                       "recall_at_10": rec})
        log("nprobe %2d: batch %.3f ms (k_cand %.3f ms), %.0f q/s, %.0f pairs/query, recall@10 %.3f" %
            (nprobe, ms, k_ms, nq / (ms / 1000.0), pairs / nq, rec))
    head = next((p for p in points if p["recall_at_10"] >= 0.9), points[-1])
    per_pair = 96 + 8 + 1 + 4 + 4
    pairs = head["pairs_per_query"] * nq
    achieved = per_pair * pairs / (head["kernel_ms"] / 1000.0) / 1e9
    out = line(head["distances_per_s"], "distances/s", args.steps, args.warmup, head["ms_per_batch"], "f32",
               {"workload": "soft inverted index: n=10,000,000 d=96 (256 clusters) LVQ-8 L2 with 256 means "
                            "(k-means on a 100k sample); 10,000 queries, each scoring the rows of its nprobe "
                            "nearest means, top-10; value at the smallest nprobe reaching recall@10 >= 0.9",
                "n": n, "dim": d, "means": M, "queries": nq, "k": k, "nprobe": head["nprobe"], "tile_shape": tile},
               {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel": "k_cand over the probed members (fused top-10)", "kernel_ms": head["kernel_ms"],
                "algorithmic_bytes_per_pair": per_pair},
               qps=head["qps"], recall_at_10=head["recall_at_10"], operating_points=points,
               recall_sample="%d queries against the exact float top-10" % ns)
    out["encode"] = encode_roofline(warm_encode_ms(ix, X, dev), n, d, ix.row_bytes, ix.resid_bytes, enc_ms, n_means=M)
    if not args.no_cpu_baseline:
        import oracle
        log("timing the oracle on a host-core sample")
        # a 200k-row slice of the store, encoded by the oracle; its queries
        # routed and scored by the oracle, timed
        m = 200_000
        fmt = oracle.Format(d, 8, 0)
        rows, _, _ = oracle.encode_rows(fmt, X[:m], means)
        nqs = 2000
        t = time.perf_counter()
        pr = oracle.probe_means(Q[:nqs], means, head["nprobe"])
        offs, lid = oracle.probe_lists(pr, rows[:, 12])
        dd = oracle.distances(fmt, oracle.L2, oracle.PRIMARY, Q[:nqs], rows, None, means, offs, lid)
        oracle.topk_lists(oracle.L2, dd, offs, lid, k)
        ct = time.perf_counter() - t
        out["cpu_baseline"] = {"value": int(offs[-1]) / ct, "unit": "distances/s", "cores": 1, "kind": "oracle",
                               "sample": "%d queries routed (nprobe %d) over a %d-row slice of the store, %d pairs, "
                                         "binary64 scalar C, %.2f s" % (nqs, head["nprobe"], m, int(offs[-1]), ct)}
    ix.close()
    return out


# ---------------------------------------------------------------------------
# Greedy graph search (Alg. 1) over LVQ-8 codes: queries/s against recall
# ---------------------------------------------------------------------------

GRAPH_TRAFFIC = os.path.join(ROOT, "profiles", "k_graph_search_g1_stats.md")
GRAPH_SOURCES = ["paper_2402_02044_amd/csrc/k_graph.hip", "paper_2402_02044_amd/csrc/k_common.h"]


def read_graph_traffic(nq: int, window: int):
    """HBM bytes per search launch from the committed counter summary, if it
    was taken on the current kernel source, batch and window (else None)."""
    if not os.path.exists(GRAPH_TRAFFIC):
        return None
    vals = {}
    for ln in open(GRAPH_TRAFFIC):
        if ":" in ln and ln.strip().startswith("- "):
            k, v = ln.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    h = hashlib.sha256()
    for p in GRAPH_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    try:
        if vals.get("kernel_source_sha") != h.hexdigest()[:16]:
            return None
        if int(vals["queries_per_launch"]) != nq or int(vals["window"]) != window:
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def bench_graph(args):
    import torch

    import paper_2402_02044_amd as L
    import synth
    n, nq, d, k = args.n or 1_000_000, args.nq or 10_000, 96, 10
    # the paper's graph parameters at 10^6 vectors: out-degree 64, build
    # window 200, alpha 1.2 (L2), two passes
    R, build_w, alpha = 64, 200, 1.2
    log("generating %d x %d base vectors (G1), %d queries" % (n, d, nq))
    X = synth.vectors("G1", synth.S_BASE, 0, n)
    Q = synth.vectors("G1", synth.S_QUERY, 0, nq)
    dev = torch.device("cuda:0")
    mu = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    log("uploading and encoding the store")
    ix = L.Index(d, 8, 0, L.LVQ_L2, L.LVQ_SEQUENTIAL, capacity=n, means=mu)
    enc_ms = to_gpu_rows(ix, X, dev)
    # one entry node: the row nearest to the data mean (the medoid's stand-in)
    xd = torch.from_numpy(X).to(dev)
    entry = torch.argmin(((xd - torch.from_numpy(mu).to(dev)) ** 2).sum(1)).to(torch.int32).reshape(1)
    log("graph construction: R %d, window %d, alpha %.2f, two passes" % (R, build_w, alpha))
    torch.cuda.synchronize()
    t = time.perf_counter()
    graph = L.graph_build(xd, R, build_w, alpha, L.LVQ_L2, int(entry.item()), passes=2, max_batch=16384)
    torch.cuda.synchronize()
    graph_s = time.perf_counter() - t
    deg = (graph >= 0).sum(1).float()
    log("built in %.1f s; mean out-degree %.1f" % (graph_s, deg.mean().item()))
    del xd
    ns = 1000
    log("exact float top-%d of %d queries" % (k, ns))
    gt = exact_topk(0, Q[:ns], X, k)
    qd = torch.from_numpy(Q).to(dev)
    ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
    cnt = torch.empty((nq, 2), dtype=torch.int32, device=dev)
    s = int(torch.cuda.current_stream().cuda_stream)
    row_bytes = ix.row_bytes
    points = []
    for W in ((args.window,) if args.window else (16, 24, 32, 48, 64, 96, 128)):

        def step():
            L.lvq_graph_search(ix.handle, qd.data_ptr(), nq, graph.data_ptr(), R, entry.data_ptr(), 1, W, k,
                               ids.data_ptr(), dist.data_ptr(), cnt.data_ptr(), s)

        ms, k_ms = timed(step, args.steps, args.warmup, ix)
        assert ix.sync() == 0
        c = cnt.cpu().numpy().astype(np.int64)
        rec = recall_at_k(ids[:ns].cpu().numpy(), gt)
        # algorithmic bytes: the query (kernel order), each explored node's
        # graph row, each scored node's code row
        nbytes = int(nq * d * 4 + c[:, 0].sum() * R * 4 + c[:, 1].sum() * row_bytes)
        points.append({"window": W, "ms_per_batch": ms, "kernel_ms": k_ms, "qps": nq / (ms / 1000.0),
                       "explored_per_query": float(c[:, 0].mean()), "scored_per_query": float(c[:, 1].mean()),
                       "distances_per_s": float(c[:, 1].sum()) / (ms / 1000.0), "recall_at_10": rec,
                       "bytes_per_launch": nbytes})
        log("W %3d: batch %.3f ms (kernel %.3f ms), %.0f q/s, explored %.0f, scored %.0f, recall@10 %.3f" %
            (W, ms, k_ms, nq / (ms / 1000.0), c[:, 0].mean(), c[:, 1].mean(), rec))
    # two levels (Sec. 2.3): an LVQ-4x8 store of the same vectors; the 4-bit
    # first level traverses, both levels re-rank the walk's final set
    two = []
    if not args.window:
        log("LVQ-4x8 store: walk on the first level, re-rank the final set at both levels")
        ix2 = L.Index(d, 4, 8, L.LVQ_L2, L.LVQ_TURBO, capacity=n, means=mu)
        to_gpu_rows(ix2, X, dev)
        for W in (32, 48, 64, 96):
            wid = torch.empty((nq, W), dtype=torch.int32, device=dev)
            wd = torch.empty((nq, W), dtype=torch.float32, device=dev)
            offs = torch.arange(nq + 1, dtype=torch.int64, device=dev) * W

            def step2():
                L.lvq_graph_search(ix2.handle, qd.data_ptr(), nq, graph.data_ptr(), R, entry.data_ptr(), 1, W, W,
                                   wid.data_ptr(), wd.data_ptr(), 0, s)
                L.lvq_distances(ix2.handle, qd.data_ptr(), nq, offs.data_ptr(), wid.data_ptr(), nq * W, L.LVQ_FULL,
                                0, k, ids.data_ptr(), dist.data_ptr(), s)

            ms2, _ = timed(step2, args.steps, args.warmup, ix2)
            assert ix2.sync() == 0
            rec2 = recall_at_k(ids[:ns].cpu().numpy(), gt)
            rec1 = recall_at_k(wid[:ns, :k].cpu().numpy(), gt)
            two.append({"window": W, "ms_per_batch": ms2, "qps": nq / (ms2 / 1000.0), "recall_at_10": rec2,
                        "recall_at_10_first_level_only": rec1})
            log("4x8 W %3d: walk + re-rank %.3f ms, %.0f q/s, recall@10 %.3f (first level alone %.3f)" %
                (W, ms2, nq / (ms2 / 1000.0), rec2, rec1))
        ix2.close()
    # graph updates (App. A): consolidate the deletion of 1% of the nodes out of
    # the graph, then insert their vectors again into the freed slots
    updates = None
    if not args.window:
        g = synth.rng(6, synth.S_DELETE)
        cand = np.setdiff1d(np.arange(n), [int(entry.item())])
        dead = np.sort(g.choice(cand, n // 100, replace=False)).astype(np.int32)
        ix.delete(torch.from_numpy(dead).to(dev))
        flags = torch.zeros(n, dtype=torch.uint8, device=dev)
        flags[torch.from_numpy(dead).long().to(dev)] = 1
        xg = torch.from_numpy(X).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.graph_delete(xg, graph, flags, alpha, L.LVQ_L2)
        torch.cuda.synchronize()
        del_s = time.perf_counter() - t0
        ix.consolidate()
        slots = ix.insert(torch.from_numpy(X[dead]).to(dev))
        assert ix.sync() == 0
        xg[slots.long()] = torch.from_numpy(X[dead]).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.graph_insert(xg, graph, slots.cpu().numpy(), build_w, alpha, L.LVQ_L2, int(entry.item()))
        torch.cuda.synchronize()
        ins_s = time.perf_counter() - t0
        Xnow = xg.cpu().numpy()
        gt2 = exact_topk(0, Q[:ns], Xnow, k)
        W = head_w = next((p["window"] for p in points if p["recall_at_10"] >= 0.9), points[-1]["window"])
        L.lvq_graph_search(ix.handle, qd.data_ptr(), nq, graph.data_ptr(), R, entry.data_ptr(), 1, W, k,
                           ids.data_ptr(), dist.data_ptr(), cnt.data_ptr(), s)
        assert ix.sync() == 0
        rec_after = recall_at_k(ids[:ns].cpu().numpy(), gt2)
        updates = {"deleted": int(dead.size), "delete_consolidation_s": del_s, "reinserted": int(dead.size),
                   "insert_s": ins_s, "insert_nodes_per_s": dead.size / ins_s, "window": head_w,
                   "recall_at_10_after": rec_after}
        log("graph updates: delete consolidation of %d nodes %.3f s; insert of %d nodes %.3f s; recall@10 at "
            "W %d afterwards %.3f" % (dead.size, del_s, dead.size, ins_s, head_w, rec_after))
        del xg
    head = next((p for p in points if p["recall_at_10"] >= 0.9), points[-1])
    achieved = head["bytes_per_launch"] / (head["kernel_ms"] / 1000.0) / 1e9
    out = line(head["qps"], "queries/s", args.steps, args.warmup, head["ms_per_batch"], "f32",
               {"workload": "greedy graph search: n=1,000,000 d=96 (anisotropic, unit norm) LVQ-8 L2, graph "
                            "built on the GPU (out-degree 64, build window 200, alpha 1.2, two passes), one entry "
                            "node; 10,000 queries, top-10; value at the smallest window W reaching recall@10 >= 0.9",
                "n": n, "dim": d, "degree": R, "queries": nq, "k": k, "window": head["window"]},
               {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": read_graph_traffic(nq, head["window"]),
                "kernel": "k_graph_search (one 64-lane workgroup per query; a chain of dependent steps per query)",
                "kernel_ms": head["kernel_ms"],
                "algorithmic_bytes": "d*4 per query + degree*4 per explored node + %d per scored node" % row_bytes},
               distances_per_s=head["distances_per_s"], recall_at_10=head["recall_at_10"], operating_points=points,
               recall_sample="%d queries against the exact float top-10" % ns, two_level_lvq4x8=two,
               graph_updates=updates,
               graph_build={"seconds": graph_s, "nodes_per_s": n / graph_s, "degree": R, "window": build_w,
                            "alpha": alpha, "passes": 2, "mean_out_degree": deg.mean().item()})
    out["encode"] = encode_roofline(warm_encode_ms(ix, X, dev), n, d, ix.row_bytes, ix.resid_bytes, enc_ms)
    if not args.no_cpu_baseline:
        import oracle
        log("timing the oracle on a host-core sample")
        fmt = oracle.Format(d, 8, 0)
        rows, _, _ = oracle.encode_rows(fmt, X, mu)
        g_host = graph.cpu().numpy()
        e_host = entry.cpu().numpy()
        # queries in order until 15 s of host time (at most 2000)
        nqs = 0
        t = time.perf_counter()
        while nqs < 2000 and time.perf_counter() - t < 15.0:
            oracle.greedy_search(fmt, oracle.L2, oracle.PRIMARY, Q[nqs], rows, None, mu, g_host, e_host,
                                 head["window"], k)
            nqs += 1
        ct = time.perf_counter() - t
        out["cpu_baseline"] = {"value": nqs / ct, "unit": "queries/s", "cores": 1, "kind": "oracle",
                               "sample": "%d queries, window %d, over the whole store and graph; binary64 "
                                         "similarities (scalar C) in a Python walk, %.2f s" %
                                         (nqs, head["window"], ct)}
    ix.close()
    return out


def bench_graph_stream(args):
    """Streaming graph search (App. A): the G1 store and its graph, then
    rounds of: tombstone 5% of the live nodes, consolidate them out of the
    graph (lvq_graph_delete) and the store, insert 50,000 fresh vectors into
    the freed slots (store, then lvq_graph_insert); after each round the
    search (W = 96, top-10) over the live set: queries/s and recall@10."""
    import torch

    import paper_2402_02044_amd as L
    import synth
    n, nq, d, k, W = args.n or 1_000_000, args.nq or 10_000, 96, 10, 96
    R, build_w, alpha = 64, 200, 1.2
    rounds = min(args.rounds, 10)
    per_round_new, frac_del = n // 20, 0.05
    dev = torch.device("cuda:0")
    log("generating %d x %d base vectors (G1), %d queries" % (n, d, nq))
    X = synth.vectors("G1", synth.S_BASE, 0, n)
    Q = synth.vectors("G1", synth.S_QUERY, 0, nq)
    mu = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    ix = L.Index(d, 8, 0, L.LVQ_L2, L.LVQ_SEQUENTIAL, capacity=n, means=mu)
    to_gpu_rows(ix, X, dev)
    xg = torch.from_numpy(X).to(dev)
    entry = int(torch.argmin(((xg - torch.from_numpy(mu).to(dev)) ** 2).sum(1)).item())
    t = time.perf_counter()
    graph = L.graph_build(xg, R, build_w, alpha, L.LVQ_L2, entry, passes=2, max_batch=16384)
    torch.cuda.synchronize()
    log("graph built in %.1f s" % (time.perf_counter() - t))
    live = np.ones(n, bool)
    qd = torch.from_numpy(Q).to(dev)
    ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
    cnt = torch.empty((nq, 2), dtype=torch.int32, device=dev)
    ed = torch.tensor([entry], dtype=torch.int32, device=dev)
    s = int(torch.cuda.current_stream().cuda_stream)
    ns = 1000

    def search_round(r, upd):
        def step():
            L.lvq_graph_search(ix.handle, qd.data_ptr(), nq, graph.data_ptr(), R, ed.data_ptr(), 1, W, k,
                               ids.data_ptr(), dist.data_ptr(), cnt.data_ptr(), s)
        ms, k_ms = timed(step, args.steps, args.warmup, ix)
        assert ix.sync() == 0
        c = cnt.cpu().numpy().astype(np.int64)
        xs = xg.cpu().numpy()
        gt = exact_topk(0, Q[:ns], xs, k, live=live)
        rec = recall_at_k(ids[:ns].cpu().numpy(), gt)
        row = {"round": r, "live": int(live.sum()), "ms_per_batch": ms, "kernel_ms": k_ms, "qps": nq / (ms / 1000.0),
               "recall_at_10": rec,
               "bytes_per_launch": int(nq * d * 4 + c[:, 0].sum() * R * 4 + c[:, 1].sum() * ix.row_bytes)}
        row.update(upd)
        log("round %2d: live %d, %.0f q/s, recall@10 %.3f %s" %
            (r, live.sum(), nq / (ms / 1000.0), rec,
             " ".join(("%s %d" if isinstance(v, (int, np.integer)) else "%s %.3f") % (kk, v) for kk, v in upd.items())))
        return row

    hist = [search_round(0, {})]
    for r in range(1, rounds + 1):
        g = synth.rng(6, synth.S_DELETE, r)
        cand = np.flatnonzero(live & (np.arange(n) != entry))
        dead = np.sort(g.choice(cand, int(frac_del * live.sum()), replace=False)).astype(np.int32)
        ix.delete(torch.from_numpy(dead).to(dev))
        flags = torch.zeros(n, dtype=torch.uint8, device=dev)
        flags[torch.from_numpy(dead).long().to(dev)] = 1
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.graph_delete(xg, graph, flags, alpha, L.LVQ_L2)
        torch.cuda.synchronize()
        del_s = time.perf_counter() - t0
        ix.consolidate()
        live[dead] = False
        Xn = synth.vectors("G1", synth.S_INSERT, (r - 1) * per_round_new, min(per_round_new, dead.size))
        slots = ix.insert(torch.from_numpy(Xn).to(dev))
        assert ix.sync() == 0
        sl = slots.cpu().numpy()
        xg[slots.long()] = torch.from_numpy(Xn).to(dev)
        live[sl] = True
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.graph_insert(xg, graph, sl, build_w, alpha, L.LVQ_L2, entry)
        torch.cuda.synchronize()
        ins_s = time.perf_counter() - t0
        hist.append(search_round(r, {"deleted": int(dead.size), "delete_s": del_s, "inserted": int(sl.size),
                                     "insert_s": ins_s}))
    last = hist[-1]
    achieved = last["bytes_per_launch"] / (last["kernel_ms"] / 1000.0) / 1e9
    out = line(last["qps"], "queries/s", args.steps, args.warmup, last["ms_per_batch"], "f32",
               {"workload": "streaming graph search: G1 n=1,000,000 d=96 LVQ-8 L2, graph out-degree 64 (build "
                            "window 200, alpha 1.2); %d rounds of 5%% deletes consolidated out of the graph and "
                            "50,000 inserts into the freed slots; search W=96, top-10, 10,000 queries; value "
                            "after the last round" % rounds,
                "n": n, "dim": d, "degree": R, "window": W, "rounds": rounds, "queries": nq, "k": k},
               {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel": "k_graph_search after the last round (one 64-lane workgroup per query)",
                "kernel_ms": last["kernel_ms"],
                "algorithmic_bytes": "d*4 per query + degree*4 per explored node + %d per scored node" % ix.row_bytes},
               rounds=hist, recall_sample="%d queries against the exact float top-10 of the live set" % ns)
    if not args.no_cpu_baseline:
        import oracle
        log("timing the oracle on a host-core sample")
        fmt = oracle.Format(d, 8, 0)
        xs = xg.cpu().numpy()
        rows, _, _ = oracle.encode_rows(fmt, xs, mu)
        g_host = graph.cpu().numpy()
        nqs = 0
        t = time.perf_counter()
        while nqs < 2000 and time.perf_counter() - t < 15.0:
            oracle.greedy_search(fmt, oracle.L2, oracle.PRIMARY, Q[nqs], rows, None, mu, g_host, [entry], W, k, live)
            nqs += 1
        ct = time.perf_counter() - t
        out["cpu_baseline"] = {"value": nqs / ct, "unit": "queries/s", "cores": 1, "kind": "oracle",
                               "sample": "%d queries, window %d, over the store and graph after the last round; "
                                         "binary64 similarities (scalar C) in a Python walk, %.2f s" % (nqs, W, ct)}
    ix.close()
    return out


# ---------------------------------------------------------------------------
# Turbo vs sequential 4-bit layout (the GPU analogue of the paper's Turbo
# table, Sec. 3.1): first-level inner products over candidate lists
# ---------------------------------------------------------------------------

def bench_layouts(args):
    import torch

    import paper_2402_02044_amd as L
    import synth
    n, nq, per = args.n or 1_000_000, args.nq or 2_000, 1000
    dev = torch.device("cuda:0")
    rows = []
    for d in (64, 128, 256, 512, 768, 1024):
        X = synth.anisotropic(2, synth.S_BASE, 0, n, d)
        Q = synth.anisotropic(2, synth.S_QUERY, 0, nq, d)
        mu = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
        offs, ids = synth.candidate_lists(2, nq, n, length=per)
        qd = torch.from_numpy(Q).to(dev)
        od = torch.from_numpy(offs).to(dev)
        idd = torch.from_numpy(ids).to(dev)
        ent = {"dim": d}
        for name, layout in (("turbo", L.LVQ_TURBO), ("sequential", L.LVQ_SEQUENTIAL)):
            ix = L.Index(d, 4, 0, L.LVQ_IP, layout, capacity=n, means=mu)
            to_gpu_rows(ix, X, dev)
            shape, _ = ix.autotune(qd, od, idd, level=L.LVQ_PRIMARY, k=0)
            dist = torch.empty(ids.shape[0], dtype=torch.float32, device=dev)
            s = int(torch.cuda.current_stream().cuda_stream)

            def step():
                L.lvq_distances(ix.handle, qd.data_ptr(), nq, od.data_ptr(), idd.data_ptr(), ids.shape[0],
                                L.LVQ_PRIMARY, dist.data_ptr(), 0, 0, 0, s)

            _, k_ms = timed(step, args.steps, args.warmup, ix)
            assert ix.sync() == 0
            ent[name] = {"kernel_ms": k_ms, "ns_per_distance": k_ms * 1e6 / ids.shape[0], "tile_shape": shape,
                         "row_bytes": ix.row_bytes}
            ix.close()
        ent["time_reduction"] = 1.0 - ent["turbo"]["kernel_ms"] / ent["sequential"]["kernel_ms"]
        log("d=%d: turbo %.4f ns, sequential %.4f ns per distance (reduction %.1f%%)" %
            (d, ent["turbo"]["ns_per_distance"], ent["sequential"]["ns_per_distance"], 100 * ent["time_reduction"]))
        rows.append(ent)
    t768 = [r for r in rows if r["dim"] == 768][0]["turbo"]
    return line(1e9 / t768["ns_per_distance"], "distances/s", args.steps, args.warmup, None, "f32",
                {"workload": "first-level LVQ-4 inner products, Turbo vs sequential 4-bit layout, n=%d, %d queries x "
                             "%d candidates, d in 64..1024 (value: Turbo at d=768)" % (n, nq, per)},
                None, layouts=rows)


# ---------------------------------------------------------------------------
# C5: streaming serving (request server beside inserts, deletes, drift)
# ---------------------------------------------------------------------------

class C5Store:
    """The served index plus what the harness needs to judge it: the float
    vectors by slot (device copy for the ground truth, host copy for spot
    checks) and which slots are live."""

    def __init__(self, L, X0, means, cap, dev):
        import torch
        self.L, self.dev, self.cap = L, dev, cap
        self.ix = L.Index(768, 4, 8, L.LVQ_IP, L.LVQ_TURBO, capacity=cap, means=means)
        self.stream = torch.cuda.Stream()
        self.Xd = torch.zeros((cap, 768), dtype=torch.float32, device=dev)
        self.Xh = np.zeros((cap, 768), np.float32)
        self.live = np.zeros(cap, bool)
        self.n_means = means.shape[0]
        self.n_ids = means.shape[0]                  # ids in use (online policy)
        self.means_by_id = np.zeros((256, 768), np.float64)
        self.means_by_id[:self.n_ids] = means
        self.retired = np.zeros(256, bool)
        for a in range(0, X0.shape[0], 1 << 18):
            self.insert(X0[a:a + (1 << 18)])

    def insert(self, X):
        import torch
        with torch.cuda.stream(self.stream):
            xd = torch.from_numpy(X).to(self.dev)
            slots_d = self.ix.insert(xd)
            self.Xd[slots_d.long()] = xd
            slots = slots_d.cpu().numpy()
        self.Xh[slots] = X
        self.live[slots] = True
        return slots

    def delete(self, slots):
        import torch
        with torch.cuda.stream(self.stream):
            self.ix.delete(torch.from_numpy(slots.astype(np.int32)).to(self.dev))
        self.live[slots] = False

    def consolidate(self):
        return self.ix.consolidate(stream=self.stream)

    def refit_means(self, round_, k=16, sample=100_000, iters=25):
        """k-means (host, binary64) over a uniform sample of live vectors,
        appended to the index's means."""
        import synth
        g = synth.rng(5, synth.S_SAMPLE, 100 + round_)
        cand = np.flatnonzero(self.live)
        pick = np.sort(g.choice(cand, min(sample, cand.size), replace=False))
        C = host_kmeans(self.Xh[pick], k, iters, 5, 200 + round_)
        self.ix.set_means(C, stream=self.stream)
        self.n_means += k

    def online_update(self, thr):
        """Online M-LVQ re-estimation: the centroid of every active mean's live
        members (binary64, on the GPU); each mean whose centroid moved by more
        than thr becomes a new mean at the centroid (lvq_add_means, reusing
        freed ids), the old id is retired, and its live rows are re-encoded
        (deleted and inserted again from their float vectors).  Returns (means
        moved, rows re-encoded)."""
        import torch
        act = np.array([m for m in range(self.n_ids) if not self.retired[m]], np.int32)
        offs, mem = self.ix.mean_members(act, cap=int(self.live.sum()), stream=self.stream)
        with torch.cuda.stream(self.stream):
            # members come grouped by mean: one reduction per contiguous range
            sums = torch.zeros((act.size, 768), dtype=torch.float64, device=self.dev)
            for i in range(act.size):
                if offs[i + 1] > offs[i]:
                    sums[i] = self.Xd[mem[offs[i]:offs[i + 1]].long()].double().sum(0)
            cnt = torch.from_numpy(np.maximum(np.diff(offs), 1)).to(self.dev)
            cen = (sums / cnt[:, None]).cpu().numpy()
        self.stream.synchronize()
        old = self.means_by_id[act].astype(np.float64)
        shift = np.linalg.norm(cen - old, axis=1)
        moved = np.flatnonzero((np.diff(offs) > 0) & (shift > thr))
        if moved.size == 0:
            return 0, 0
        new_ids = self.ix.add_means(cen[moved].astype(np.float32), stream=self.stream)
        self.ix.retire_means(act[moved], stream=self.stream)
        for i, m in zip(moved, new_ids):
            self.means_by_id[m] = cen[i]
            self.retired[m] = False
            self.n_ids = max(self.n_ids, int(m) + 1)
        self.retired[act[moved]] = True
        mem_h = mem.cpu().numpy()
        slots = np.concatenate([mem_h[offs[i]:offs[i + 1]] for i in moved]).astype(np.int32)
        self.delete(slots)
        for a in range(0, slots.size, 1 << 18):
            self.insert(self.Xh[slots[a:a + (1 << 18)]].copy())
        return int(moved.size), int(slots.size)

    def groundtruth(self, Q, k=10, chunk=65536):
        """Exact top-k by inner product over the live float vectors, binary64
        products and sums (torch float64 on the GPU)."""
        import torch
        live = torch.from_numpy(np.flatnonzero(self.live)).to(self.dev)
        with torch.cuda.stream(self.stream):
            q = torch.from_numpy(Q).to(self.dev, torch.float64)
            bv = bi = None
            for a in range(0, live.numel(), chunk):
                idx = live[a:a + chunk]
                sc = q @ self.Xd[idx].double().T
                v, i = sc.topk(k, dim=1)
                i = idx[i]
                if bv is not None:
                    v = torch.cat([bv, v], 1)
                    i = torch.cat([bi, i], 1)
                    v, o = v.topk(k, dim=1)
                    i = torch.gather(i, 1, o)
                bv, bi = v, i
            out = bi.cpu().numpy()
        return out


def c5_host_groundtruth(store, Q, k=10):
    """Exact inner-product top-k over the live float vectors on the host
    (numpy binary64), to spot-check the GPU ground truth."""
    live = np.flatnonzero(store.live)
    sc = np.asarray(Q, np.float64) @ store.Xh[live].astype(np.float64).T
    return live[np.argsort(-sc, axis=1, kind="stable")[:, :k]]


def c5_load(sv, batches, arrivals, waiter_out):
    """Submit `batches` (host arrays) at the given arrival offsets in seconds
    (None: all at once) and collect (nq, record) per batch, in order."""
    import threading
    tickets = []
    lock = threading.Condition()

    def waiter():
        got = 0
        while got < len(batches):
            with lock:
                while len(tickets) <= got:
                    lock.wait()
                t, nq = tickets[got]
            _, _, info = sv.wait(t, nq)
            waiter_out.append((nq, info))
            got += 1

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    lag = []
    for b, q in enumerate(batches):
        if arrivals is not None:
            due = t0 + arrivals[b]
            while True:
                dt = due - time.perf_counter()
                if dt <= 0:
                    break
                time.sleep(min(dt, 0.002) if dt > 0.0003 else 0)
            lag.append(time.perf_counter() - due)
        t = sv.submit(q)
        with lock:
            tickets.append((t, q.shape[0]))
            lock.notify()
    th.join()
    return float(np.mean(lag)) if lag else 0.0


def serving_summary(args, n0=1_000_000, load=0.8, n_sat=60, n_lat=120):
    """A bounded run of the serving workload for the default line: the C5
    store (10^6 LVQ-4x8 Turbo vectors of d = 768 from 64 unit clusters, 16
    means from k-means on a 100k sample) served in batches of U{1..512}
    queries by the request server in two forms -- exhaustive two-level top-10
    on the FP32 vector path and on the matrix cores (bf16) -- while a thread
    runs update rounds at a constant store size (delete 10^4 live vectors,
    insert 10^4 drifted ones, consolidate; the paper's constant-size streaming
    protocol, so that both forms are measured over the same row count).  Per form: the saturation rate of a burst
    of batches, p50 / p99 latency under Poisson arrivals at `load` times that
    rate, and recall@10 of 200 queries against the exact float top-10 of the
    live vectors; beside them the two-stage form (first-level bf16 top-K'
    re-ranked with both levels) for K' in {64, 256, 1024}."""
    import threading

    import torch

    import paper_2402_02044_amd as L
    import synth
    K, MAXB, SLOTS, ins = 10, 512, 8, 10_000
    dev = torch.device("cuda:0")
    t_start = time.perf_counter()
    log("serving: generating %d x 768 C5 vectors, 16 means" % n0)
    X0 = synth.vectors("C5", synth.S_BASE, 0, n0)
    means = host_kmeans(X0[synth.sample_indices(5, n0, 100_000)], 16, 25, 5)
    st = C5Store(L, X0, means, n0 + 8 * ins + 4096, dev)
    del X0
    torch.cuda.synchronize()
    forms = {"fp32": L.LVQ_FP32, "bf16": L.LVQ_BF16}
    servers = {f: L.Server(st.ix, slots=SLOTS, max_batch=MAXB, k=K, k_first=64, precision=p,
                           scan_level=L.LVQ_FULL) for f, p in forms.items()}
    qpool = synth.c5_points(synth.S_QUERY, 1, 4096, part=1)
    g = synth.rng(5, synth.S_ARRIVAL, 1)

    def make_batches(nb):
        sizes = g.integers(1, MAXB + 1, nb)
        starts = g.integers(0, qpool.shape[0] - MAXB, nb)
        return [qpool[a:a + s] for a, s in zip(starts, sizes)]

    stop = threading.Event()
    rounds = []

    def updates():
        r = 0
        while not stop.is_set() and r < 20:
            t = time.perf_counter()
            cand = np.flatnonzero(st.live)
            st.delete(np.sort(synth.rng(5, synth.S_DELETE, 1000 + r).choice(cand, ins, replace=False)))
            st.insert(synth.c5_points(synth.S_INSERT, r + 1, ins))
            freed = st.consolidate()
            rounds.append({"round": r, "live": int(st.live.sum()), "freed": int(freed),
                           "update_ms": (time.perf_counter() - t) * 1000.0})
            r += 1
            stop.wait(0.3)

    for f in forms:   # warm-up
        c5_load(servers[f], make_batches(8), None, [])
    upd = threading.Thread(target=updates)
    upd.start()
    out = {}
    try:
        for f in forms:
            sv = servers[f]
            rows0 = st.ix.stats().live_estimate
            got = []
            c5_load(sv, make_batches(n_sat), None, got)
            qps = sum(nq for nq, _ in got) / (max(i.t_done for _, i in got) - min(i.t_submit for _, i in got))
            arr = np.cumsum(g.exponential((MAXB + 1) / 2.0 / (load * qps), n_lat))
            got = []
            c5_load(sv, make_batches(n_lat), arr, got)
            lat = np.array([(i.t_done - i.t_submit) * 1000.0 for _, i in got])
            span = max(i.t_done for _, i in got) - min(i.t_submit for _, i in got)
            out[f] = {"qps_saturation": qps, "rows_at_saturation": int(rows0),
                      "load": load, "achieved_qps": sum(nq for nq, _ in got) / span,
                      "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                      "peak_in_flight": sv.stats().peak_in_flight}
            log("serving %s: saturation %.0f q/s over %d rows; at %d%% load p50 %.2f ms, p99 %.2f ms" %
                (f, qps, rows0, load * 100, out[f]["p50_ms"], out[f]["p99_ms"]))
    finally:
        stop.set()
        upd.join()
    # recall at the final state
    Qr = synth.c5_points(synth.S_QUERY, 1, 200, part=0)
    gt = st.groundtruth(Qr)
    for f in forms:
        t = servers[f].submit(Qr)
        ids, _, _ = servers[f].wait(t, Qr.shape[0])
        out[f]["recall_at_10"] = recall_at_k(ids, gt)
    for sv in servers.values():
        sv.close()
    qd = torch.from_numpy(Qr).to(dev)
    rerank = {}
    for kf in (64, 256, 1024):
        # the matrix-core scan's per-query buffers hold up to a few hundred
        # keys; larger K' take the first-level FP32 scan
        cid = None
        for prec, tdt in (("bf16", torch.bfloat16), ("fp32", torch.float32)):
            try:
                cid, _ = st.ix.topk(qd.to(tdt), kf, level=L.LVQ_PRIMARY)
                break
            except L.LVQError as e:
                if e.code != L.LVQ_ERR_UNSUPPORTED:
                    raise
        if cid is None:
            rerank[str(kf)] = None
            continue
        offs = torch.arange(0, (Qr.shape[0] + 1) * kf, kf, dtype=torch.int64, device=dev)
        _, ti, _ = st.ix.distances(qd, offs, cid.reshape(-1), level=L.LVQ_FULL, k=K, want_dist=False)
        rerank[str(kf)] = {"first_level_scan": prec, "recall_at_10": recall_at_k(ti.cpu().numpy(), gt)}
    assert st.ix.sync() == 0
    st.ix.close()
    log("serving: recall@10 fp32 %.3f, bf16 %.3f; first-level top-K' re-ranked: %s" %
        (out["fp32"]["recall_at_10"], out["bf16"]["recall_at_10"], rerank))
    out["rerank_first_level_top_kprime"] = rerank
    out["update_rounds"] = rounds
    out["workload"] = ("C5 store: LVQ-4x8 Turbo inner product, d=768, %d vectors from 64 unit clusters, 16 means; "
                       "request server, %d slots, batches of U{1..%d} queries, exhaustive two-level top-%d; "
                       "update rounds (delete %d live, insert as many, consolidate) beside the load; recall@10 of "
                       "200 queries against the exact float top-10 of the live vectors" % (n0, SLOTS, MAXB, K, ins))
    out["seconds"] = time.perf_counter() - t_start
    return out


def bench_c5(args):
    import threading

    import torch

    import paper_2402_02044_amd as L
    import synth
    n0 = args.n or 1_000_000
    rounds = args.rounds
    ins = max(100, n0 // 100)
    K, KF, MAXB, SLOTS = 10, 64, 512, 8
    dev = torch.device("cuda:0")
    log("generating %d x 768 C5 base vectors" % n0)
    X0 = synth.vectors("C5", synth.S_BASE, 0, n0)
    log("M-LVQ means: k-means (16) on a 100k sample")
    samp = synth.sample_indices(5, n0, 100_000)
    means = host_kmeans(X0[samp], 16, 25, 5)
    cap = n0 + 5 * ins + 4096
    log("encoding the store (capacity %d)" % cap)
    st = C5Store(L, X0, means, cap, dev)
    del X0
    torch.cuda.synchronize()
    assert st.ix.sync() == 0
    # plain (FP32 vector) and matrix-core (bf16 MFMA) exhaustive scans at both
    # levels, and the two-stage form: first-level MFMA top-K' re-ranked with
    # both levels
    forms = {"fp32": (L.LVQ_FP32, L.LVQ_FULL), "bf16": (L.LVQ_BF16, L.LVQ_FULL),
             "bf16_rerank%d" % KF: (L.LVQ_BF16, L.LVQ_PRIMARY)}
    servers = {f: L.Server(st.ix, slots=SLOTS, max_batch=MAXB, k=K, k_first=KF, precision=p, scan_level=lv)
               for f, (p, lv) in forms.items()}
    qpool = synth.c5_points(synth.S_QUERY, rounds // 2, 4096, part=1)
    g = synth.rng(5, synth.S_ARRIVAL, 0)

    def make_batches(nb):
        sizes = g.integers(1, MAXB + 1, nb)
        starts = g.integers(0, qpool.shape[0] - MAXB, nb)
        return [qpool[a:a + s] for a, s in zip(starts, sizes)]

    # ---- the update stream: rounds of delete / insert / consolidate / drift
    progress = {"done": 0.0}
    rec = {"live": [], "freed": [], "n_means": [], "update_ms": [], "epoch": [],
           "recall": {f: [] for f in forms}, "gt_spot_checks": 0}
    err = []

    def updates():
        try:
            for r in range(rounds):
                while progress["done"] < r / rounds:
                    time.sleep(0.005)
                t = time.perf_counter()
                cand = np.flatnonzero(st.live)
                dead = np.sort(synth.rng(5, synth.S_DELETE, r).choice(cand, cand.size // 10, replace=False))
                st.delete(dead)
                st.insert(synth.c5_points(synth.S_INSERT, r + 1, ins))
                freed = st.consolidate()
                if (r + 1) % 10 == 0:
                    st.refit_means(r)
                rec["update_ms"].append((time.perf_counter() - t) * 1000.0)
                rec["live"].append(int(st.live.sum()))
                rec["freed"].append(int(freed))
                rec["n_means"].append(st.n_means)
                # served recall at this round's state: 200 queries of the drifted mixture
                Qr = synth.c5_points(synth.S_QUERY, r + 1, 200, part=0)
                tk = {f: servers[f].submit(Qr) for f in forms}
                res = {f: servers[f].wait(tk[f], Qr.shape[0]) for f in forms}
                epoch = st.ix.stats().epoch
                gt = st.groundtruth(Qr)
                if r % 10 == 0:   # the GPU ground truth against the host definition on a few queries
                    cpu = c5_host_groundtruth(st, Qr[:3])
                    assert np.array_equal(np.sort(cpu, 1), np.sort(gt[:3], 1)), "ground truth mismatch"
                    rec["gt_spot_checks"] += 1
                for f in forms:
                    ids, _, info = res[f]
                    assert info.epoch == epoch
                    rec["recall"][f].append(recall_at_k(ids, gt))
                rec["epoch"].append(int(epoch))
                log("round %d: live %d, freed %d, means %d, update %.0f ms, recall %s" %
                    (r, rec["live"][-1], freed, st.n_means, rec["update_ms"][-1],
                     " ".join("%s %.3f" % (f, rec["recall"][f][-1]) for f in forms)))
        except BaseException as e:   # surfaced by the main thread
            err.append(e)

    upd = threading.Thread(target=updates)
    upd.start()

    # ---- the query load.  The store shrinks round by round (10% deleted,
    # 10k inserted), so the scans get cheaper as the run goes on; each load
    # level is therefore measured for every form back to back, right after a
    # saturation burst of that form: offered load = fraction x that burst's
    # rate.  Rows scanned (occupied slots) are recorded with every phase.
    n_sat, n_lat = args.sat_batches, args.lat_batches
    levels = (0.5, 0.8, 0.95)
    total = len(levels) * len(forms) * (n_sat + n_lat)
    served = 0
    serving = {f: {"phases": []} for f in forms}
    mean_nq = (MAXB + 1) / 2.0

    def burst(sv):
        out = []
        c5_load(sv, make_batches(n_sat), None, out)
        q = sum(nq for nq, _ in out)
        return q / (max(i.t_done for _, i in out) - min(i.t_submit for _, i in out))

    for f in forms:   # warm-up
        c5_load(servers[f], make_batches(8), None, [])
    for frac in levels:
        for f in forms:
            sv = servers[f]
            rows0 = st.ix.stats().live_estimate
            qps = burst(sv)
            served += n_sat
            progress["done"] = served / total
            arr = np.cumsum(g.exponential(mean_nq / (frac * qps), n_lat))
            out = []
            lag = c5_load(sv, make_batches(n_lat), arr, out)
            served += n_lat
            progress["done"] = served / total
            rows1 = st.ix.stats().live_estimate
            lat = np.array([(i.t_done - i.t_submit) * 1000.0 for _, i in out])
            q = sum(nq for nq, _ in out)
            span = max(i.t_done for _, i in out) - min(i.t_submit for _, i in out)
            ph = {"load": frac, "qps_saturation": qps, "offered_qps": frac * qps, "achieved_qps": q / span,
                  "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                  "mean_ms": float(lat.mean()), "rows_scanned": [int(rows0), int(rows1)],
                  "batches": [n_sat, n_lat], "mean_submit_lag_ms": lag * 1000.0}
            serving[f]["phases"].append(ph)
            log("%s: saturation %.0f q/s over %d rows; at %d%%: p50 %.2f ms, p99 %.2f ms" %
                (f, qps, rows0, frac * 100, ph["p50_ms"], ph["p99_ms"]))
    for f in forms:
        ph = serving[f]["phases"]
        serving[f]["qps_saturation"] = ph[0]["qps_saturation"]
        serving[f]["latency_ms"] = {"%d%%" % round(p["load"] * 100): {"p50": p["p50_ms"], "p99": p["p99_ms"]}
                                    for p in ph}
        serving[f]["peak_in_flight"] = servers[f].stats().peak_in_flight
    progress["done"] = 1.0
    upd.join()
    if err:
        raise err[0]
    for f in forms:
        r = np.array(rec["recall"][f])
        serving[f]["recall_at_10"] = {"mean": float(r.mean()), "min": float(r.min()),
                                      "per_round": [round(float(v), 4) for v in r]}
    assert st.ix.sync() == 0

    # cpu baseline: the oracle serving queries on a bounded slice of the store
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("timing the oracle on a host-core sample")
        fmt = oracle.Format(768, 4, 8, oracle.TURBO)
        live = np.flatnonzero(st.live)
        sl = live[:100_000]
        rows, resid, _ = oracle.encode_rows(fmt, st.Xh[sl], means)
        Qs = synth.c5_points(synth.S_QUERY, rounds, 64, part=2)
        t = time.perf_counter()
        nq_s = 0
        while nq_s < Qs.shape[0] and time.perf_counter() - t < 15.0:
            oracle.topk_exhaustive(fmt, oracle.IP, oracle.FULL, Qs[nq_s:nq_s + 1], rows, resid, means, K)
            nq_s += 1
        dt = time.perf_counter() - t
        per_q = dt / nq_s * (live.size / sl.size)
        cpu = {"value": 1.0 / per_q, "unit": "queries/s", "cores": 1, "kind": "oracle",
               "sample": "%d queries, each an exhaustive two-level top-%d over a 100,000-row slice of the live "
                         "store (binary64 scalar C, one host core, %.1f s), scaled to the %d live rows"
                         % (nq_s, K, dt, live.size)}
    for sv in servers.values():
        sv.close()
    st.ix.close()
    bf = serving["bf16"]
    rows_scanned = int(np.mean(bf["phases"][0]["rows_scanned"]))
    out = line(bf["qps_saturation"], "queries/s", n_sat, 8, 1000.0 / bf["qps_saturation"], "bf16",
               {"workload": "C5 streaming serving: LVQ-4x8 Turbo inner product, d=768, start 1,000,000 vectors "
                            "(64 drifting unit clusters), M-LVQ 16 means re-fitted every 10 rounds; each round "
                            "deletes 10%% of live, inserts %d, consolidates; batches of U{1..512} queries; "
                            "exhaustive two-level top-%d on the FP32 vector path and on MFMA (bf16), and "
                            "first-level MFMA top-%d re-ranked with both levels" % (ins, K, KF),
                "n0": n0, "dim": 768, "rounds": rounds, "inserts_per_round": ins, "slots": SLOTS,
                "max_batch": MAXB, "k": K, "k_first": KF},
               {"bound": "mfma", "achieved": None, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": None,
                "traffic": None, "kernel": "k_scan_mfma_wide (two-level exhaustive scan of every batch)"},
               serving=serving, rounds_record=rec)
    flops = 2.0 * 2 * 768 * rows_scanned * bf["qps_saturation"] / 1e12
    out["roofline"]["achieved"] = flops
    out["roofline"]["frac"] = flops / MFMA_BF16_PEAK_TFLOPS
    out["roofline"]["note"] = ("whole-server rate of the first bf16 saturation burst: 2 levels x 2*d flops "
                               "per (query, occupied row) x %d rows x served queries/s; kernels of concurrent "
                               "batches overlap" % rows_scanned)
    if cpu:
        out["cpu_baseline"] = cpu
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "c5scan", "layouts", "probe",
                                                         "means", "graph", "graph_stream"])
    ap.add_argument("--rounds", type=int, default=30, help="c5: update rounds")
    ap.add_argument("--sat-batches", type=int, default=60, help="c5: batches of each saturation burst")
    ap.add_argument("--lat-batches", type=int, default=120, help="c5: batches of each latency phase")
    ap.add_argument("--level", default="full", choices=["full", "primary"])
    ap.add_argument("--forms", default="bf16,fp16,fp32,fp32_plain",
                    help="c4: query precisions to run (comma list; fp32_plain = the FP32 vector kernel)")
    ap.add_argument("--align", type=int, default=32)
    ap.add_argument("--n", type=int, default=0, help="override the store size (testing)")
    ap.add_argument("--nq", type=int, default=0, help="override the query count (testing)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--window", type=int, default=0, help="graph: one search window instead of the sweep")
    ap.add_argument("--tile", type=int, default=-1, help="fixed tile shape (default: tuning cache, else autotune)")
    ap.add_argument("--retune", action=argparse.BooleanOptionalAction, default=True,
                    help="c2, c3: run the library's autotuner on this box before timing (default); --no-retune "
                         "takes the shape recorded in the tuning cache")
    ap.add_argument("--serving", action=argparse.BooleanOptionalAction, default=True,
                    help="c2: add a bounded serving run (the C5 store, fp32 and bf16 two-level forms) to the line")
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
    fn = {"c1": bench_c1, "c2": bench_c2, "c3": bench_c3, "c4": bench_c4, "c5": bench_c5, "c5scan": bench_c5scan,
          "layouts": bench_layouts, "probe": bench_probe, "means": bench_means,
          "graph": bench_graph, "graph_stream": bench_graph_stream}[args.workload]
    out = fn(args)
    print(json.dumps(out), flush=True)
    if not out.get("parity", {}).get("ok", True):
        log("the timed launch's outputs disagree with the oracle on its sample")
        sys.exit(3)


if __name__ == "__main__":
    main()

"""Parity on the launch paths the full-size workloads take, through the C ABI.

The small parity tests launch fewer lists than the chip holds workgroups,
and exhaustive scans over stores too small to be split.  Here:

* lvq_distances with at least four times as many lists as the persistent
  grid has workgroups (read back from lvq_get_stats), so every workgroup
  pops several lists from the device counter and resets its per-list state
  (query tables, top-k buffers and bounds) between them: the 10^6 x 768
  LVQ-4x8 Turbo inner-product format at both levels, the 96-d LVQ-8 L2
  format with 16 means, and the soft inverted index's segmented lists;
* lvq_topk over stores of 2^17 rows and more, so that the matrix-core scan
  splits the rows into several parts that share a per-query bound and the
  FP32 scan's merge takes hundreds of parts, for 1, 70 and 600 queries
  (the last query tile partly empty), checked against the oracle on a
  sample of queries.

Values are held to the tolerance of tests/lvq_check.py, top-k sets to the
oracle's up to near-ties.
"""
import numpy as np
import pytest

import oracle
import synth
from lvq_check import ExhaustiveReference, check_topk, check_values, pair_reference

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2402_02044_amd as lib
    return lib


def _persistent_grid(L, ix, d, levels):
    """Largest workgroup count of the persistent candidate launch over every
    tile shape, level and top-k mode: a call with more (empty) lists than the
    chip holds workgroups launches the full grid of its shape."""
    nq = 1 << 16
    q = torch.zeros((nq, d), device="cuda")
    offs = torch.zeros(nq + 1, dtype=torch.int64, device="cuda")
    ids = torch.zeros(1, dtype=torch.int32, device="cuda")
    dist = torch.empty(1, device="cuda")
    ti = torch.empty((nq, 10), dtype=torch.int32, device="cuda")
    td = torch.empty((nq, 10), device="cuda")
    grid = 0
    for level in levels:
        for shape in range(-1, L.lvq_num_tile_shapes()):
            for k in (0, 10):
                try:
                    ix.set_tile(level, k > 0, shape)
                    L.lvq_distances(ix.handle, q.data_ptr(), nq, offs.data_ptr(), ids.data_ptr(), 0, level,
                                    dist.data_ptr(), k, ti.data_ptr(), td.data_ptr(), 0)
                except L.LVQError as e:
                    assert e.code == L.LVQ_ERR_UNSUPPORTED and shape >= 0
                    continue
                assert ix.sync() == 0
                g = ix.stats().last_workgroups
                assert 0 < g < nq
                grid = max(grid, g)
        ix.set_tile(level, 0, -1)
        ix.set_tile(level, 1, -1)
    return grid


def _ragged_lengths(g, nq, lmax):
    """Log-uniform lengths in [1, lmax] with every 29th list empty."""
    lens = np.floor(np.exp(g.uniform(0.0, np.log(lmax + 1), nq))).astype(np.int64)
    lens = np.clip(lens, 1, lmax)
    lens[::29] = 0
    return lens


def _lists(g, n, lens):
    offs = np.zeros(len(lens) + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    ids = np.concatenate([g.choice(n, int(x), replace=False) for x in lens]).astype(np.int32)
    return offs, ids


def _check_lists(L, ix, fmt, metric, Q, rows, resid, means, offs, ids, live, levels, grid, shapes):
    shapes, topk_shapes = shapes
    qd = torch.from_numpy(Q).cuda()
    od, idd = torch.from_numpy(offs).cuda(), torch.from_numpy(ids).cuda()
    nq = Q.shape[0]
    for level in levels:
        ref, tol = pair_reference(fmt, metric, level, Q, rows, resid, means, offs, ids)
        for shape in shapes:
            for k in (0, 10):
                try:
                    ix.set_tile(level, k > 0, shape)
                    dist, ti, td = ix.distances(qd, od, idd, level=level, k=k)
                except L.LVQError as e:
                    assert e.code == L.LVQ_ERR_UNSUPPORTED and shape >= 0
                    continue
                assert ix.sync() == 0
                st = ix.stats()
                assert st.last_lists == nq
                assert nq >= 4 * st.last_workgroups, (nq, st.last_workgroups)
                check_values(dist.cpu().numpy(), ref, tol, "shape %d level %d k %d" % (shape, level, k))
                if k == 0 or shape not in topk_shapes:
                    continue
                ti, td = ti.cpu().numpy(), td.cpu().numpy()
                for i in range(nq):
                    a, b = offs[i], offs[i + 1]
                    check_topk(metric, ti[i], td[i], ids[a:b], ref[a:b], tol[a:b], k, live[ids[a:b]])
            ix.set_tile(level, 0, -1)
            ix.set_tile(level, 1, -1)
    assert grid > 0


def _tuned_shapes(ix, levels):
    """Every shape: the default (-1), the shapes the tuning cache holds for
    this device and format (the ones the benchmark times), then the others;
    and the first two kinds, whose top-k lists are checked too."""
    import paper_2402_02044_amd as lib
    tuned = []
    for level in levels:
        s = ix.use_tuned_tile(level, 10)
        if s >= 0:
            tuned.append(s)
        ix.set_tile(level, 1, -1)
    rest = [s for s in range(lib.lvq_num_tile_shapes()) if s not in tuned]
    return [-1] + tuned + rest, [-1] + tuned


def test_persistent_lists_768d_turbo_ip(L):
    """The 10^6 x 768 LVQ-4x8 Turbo inner-product format (one global mean),
    first level and both levels, over 20,000 rows."""
    d, n = 768, 20000
    g = synth.rng(9100, 0)
    X = synth.anisotropic(2, synth.S_BASE, 0, n, d)
    mu = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    fmt = oracle.Format(d, 4, 8, oracle.TURBO)
    rows, resid, _ = oracle.encode_rows(fmt, X, mu)
    ix = L.Index(d, 4, 8, L.LVQ_IP, L.LVQ_TURBO, capacity=n, means=mu)
    ix.insert(torch.from_numpy(X).cuda())
    dead = np.sort(g.choice(n, 1000, replace=False)).astype(np.int32)
    ix.delete(torch.from_numpy(dead).cuda())
    assert ix.sync() == 0
    live = np.ones(n, bool)
    live[dead] = False
    grid = _persistent_grid(L, ix, d, (L.LVQ_PRIMARY, L.LVQ_FULL))
    nq = 4 * grid + 37
    Q = synth.anisotropic(2, synth.S_QUERY, 0, nq, d)
    offs, ids = _lists(g, n, _ragged_lengths(g, nq, 400))
    levels = [oracle.PRIMARY, oracle.FULL]
    _check_lists(L, ix, fmt, oracle.IP, Q, rows, resid, mu, offs, ids, live, levels, grid,
                 _tuned_shapes(ix, levels))
    ix.close()


def test_persistent_lists_96d_lvq8_l2_16_means(L):
    """The 96-d LVQ-8 Euclidean format with 16 means (per-list query tables
    q - mu_m rebuilt from the means kept in LDS for every list a workgroup
    pops), list lengths up to 1,500."""
    d, n, M = 96, 20000, 16
    g = synth.rng(9101, 0)
    cent = synth.centres(3, 256, d)
    X = synth.mixture(3, synth.S_BASE, 0, n, cent, 0.3)
    means = X[g.choice(n, M, replace=False)]
    fmt = oracle.Format(d, 8, 0, oracle.SEQUENTIAL)
    rows, resid, _ = oracle.encode_rows(fmt, X, means)
    ix = L.Index(d, 8, 0, L.LVQ_L2, L.LVQ_SEQUENTIAL, capacity=n, means=means)
    ix.insert(torch.from_numpy(X).cuda())
    dead = np.sort(g.choice(n, 1000, replace=False)).astype(np.int32)
    ix.delete(torch.from_numpy(dead).cuda())
    assert ix.sync() == 0
    live = np.ones(n, bool)
    live[dead] = False
    grid = _persistent_grid(L, ix, d, (L.LVQ_PRIMARY,))
    nq = 4 * grid + 37
    Q = synth.mixture(3, synth.S_QUERY, 0, nq, cent, 0.3)
    offs, ids = _lists(g, n, _ragged_lengths(g, nq, 1500))
    levels = [oracle.PRIMARY]
    _check_lists(L, ix, fmt, oracle.L2, Q, rows, resid, means, offs, ids, live, levels, grid,
                 _tuned_shapes(ix, levels))
    ix.close()


def test_persistent_probe_lists(L):
    """Soft inverted index with more queries than the persistent grid has
    workgroups: every workgroup walks several queries' segmented member
    ranges, with the probed means' tables rebuilt per list."""
    d, n, M, nprobe, k = 96, 20000, 64, 2, 10
    g = synth.rng(9102, 0)
    cent = synth.centres(3, 256, d)
    X = synth.mixture(3, synth.S_BASE, 0, n, cent, 0.3)
    means = X[g.choice(n, M, replace=False)]
    fmt = oracle.Format(d, 8, 0, oracle.SEQUENTIAL)
    rows, resid, _ = oracle.encode_rows(fmt, X, means)
    ix = L.Index(d, 8, 0, L.LVQ_L2, L.LVQ_SEQUENTIAL, capacity=n, means=means)
    ix.insert(torch.from_numpy(X).cuda())
    dead = np.sort(g.choice(n, 1000, replace=False)).astype(np.int32)
    ix.delete(torch.from_numpy(dead).cuda())
    assert ix.sync() == 0
    live = np.ones(n, bool)
    live[dead] = False
    nq = 1 << 15
    probe, ti, td = ix.probe_topk(torch.zeros((nq, d), device="cuda"), nprobe, k)
    assert ix.sync() == 0
    grid = ix.stats().last_workgroups
    nq = 4 * grid + 37
    Q = synth.mixture(3, synth.S_QUERY, 0, nq, cent, 0.3)
    probe, ti, td = ix.probe_topk(torch.from_numpy(Q).cuda(), nprobe, k)
    assert ix.sync() == 0
    st = ix.stats()
    assert st.last_lists == nq and nq >= 4 * st.last_workgroups
    probe, ti, td = probe.cpu().numpy(), ti.cpu().numpy(), td.cpu().numpy()
    want = oracle.probe_means(Q, means, nprobe)
    np.testing.assert_array_equal(probe, want)
    offs, ids = oracle.probe_lists(want, rows[:, 12], live)
    ref, tol = pair_reference(fmt, oracle.L2, oracle.PRIMARY, Q, rows, resid, means, offs, ids)
    for i in range(nq):
        a, b = offs[i], offs[i + 1]
        check_topk(oracle.L2, ti[i], td[i], ids[a:b], ref[a:b], tol[a:b], k)
    ix.close()


SAMPLE = {1: [0], 70: [0, 37, 69], 600: [0, 311, 599]}
SAMPLED = sorted(set(sum(SAMPLE.values(), [])))


def _scan_case(L, ix, fmt, metric, Q, rows, resid, means, live, levels, precs, ks, min_parts):
    n = rows.shape[0]
    allids = np.arange(n, dtype=np.int32)
    exh = ExhaustiveReference(fmt, rows, resid, means)
    row_of = {qi: r for r, qi in enumerate(SAMPLED)}
    for prec in precs:
        if prec == "fp32":
            Qd, Qr = torch.from_numpy(Q).cuda(), Q
        else:
            tdt = torch.bfloat16 if prec == "bf16" else torch.float16
            Qh = torch.from_numpy(Q).to(tdt)
            Qd, Qr = Qh.cuda(), Qh.float().numpy()
        for olev, glev in levels:
            ref, tol = exh(metric, olev, Qr[SAMPLED])
            for nq, sample in SAMPLE.items():
                for k in ks:
                    ti, td = ix.topk(Qd[:nq], k, level=glev)
                    assert ix.sync() == 0
                    parts = ix.stats().last_parts
                    assert parts >= min_parts, (prec, nq, k, parts)
                    ti, td = ti.cpu().numpy(), td.cpu().numpy()
                    for qi in sample:
                        r = row_of[qi]
                        try:
                            check_topk(metric, ti[qi], td[qi], allids, ref[r], tol[r], k, live)
                        except AssertionError as e:
                            raise AssertionError("%s level %d nq %d k %d query %d parts %d: %s"
                                                 % (prec, olev, nq, k, qi, parts, e))


def test_multipart_scan_512d_lvq8(L):
    """The 512-d LVQ-8 inner-product format over 2^17 + 3,001 rows with 5%
    tombstoned: bf16 and fp16 on the matrix cores (several row parts that
    share each query's bound) and the FP32 scan (131 parts for one query)."""
    d, n = 512, (1 << 17) + 3001
    g = synth.rng(9200, 0)
    X = synth.anisotropic(4, synth.S_BASE, 0, n, d)
    Q = synth.anisotropic(4, synth.S_QUERY, 0, 600, d)
    mu = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    fmt = oracle.Format(d, 8, 0, oracle.SEQUENTIAL)
    rows, resid, _ = oracle.encode_rows(fmt, X, mu)
    ix = L.Index(d, 8, 0, L.LVQ_IP, L.LVQ_SEQUENTIAL, capacity=n, means=mu)
    ix.insert(torch.from_numpy(X).cuda())
    dead = np.sort(g.choice(n, n // 20, replace=False)).astype(np.int32)
    ix.delete(torch.from_numpy(dead).cuda())
    assert ix.sync() == 0
    live = np.ones(n, bool)
    live[dead] = False
    _scan_case(L, ix, fmt, oracle.IP, Q, rows, resid, mu, live, [(oracle.PRIMARY, L.LVQ_PRIMARY)],
               ["bf16", "fp16", "fp32"], (10, 100), 2)
    ix.close()


def test_multipart_scan_768d_turbo_both_levels(L):
    """The 768-d LVQ-4x8 Turbo inner-product format with 16 means (the
    serving store's), first level and both levels, bf16 / fp16 / fp32."""
    d, n, M = 768, (1 << 17) + 1234, 16
    g = synth.rng(9201, 0)
    X = synth.mixture(5, synth.S_BASE, 0, n, synth.centres(5, 64, d), 0.3, unit=True)
    Q = synth.mixture(5, synth.S_QUERY, 0, 600, synth.centres(5, 64, d), 0.3, unit=True)
    means = X[g.choice(n, M, replace=False)]
    fmt = oracle.Format(d, 4, 8, oracle.TURBO)
    rows, resid, _ = oracle.encode_rows(fmt, X, means)
    ix = L.Index(d, 4, 8, L.LVQ_IP, L.LVQ_TURBO, capacity=n, means=means)
    ix.insert(torch.from_numpy(X).cuda())
    dead = np.sort(g.choice(n, n // 20, replace=False)).astype(np.int32)
    ix.delete(torch.from_numpy(dead).cuda())
    assert ix.sync() == 0
    live = np.ones(n, bool)
    live[dead] = False
    _scan_case(L, ix, fmt, oracle.IP, Q, rows, resid, means, live,
               [(oracle.PRIMARY, L.LVQ_PRIMARY), (oracle.FULL, L.LVQ_FULL)], ["bf16", "fp16", "fp32"], (10,), 2)
    ix.close()


def test_fp32_scan_merges_hundreds_of_parts(L):
    """The FP32 scan over 300,000 rows of the 96-d LVQ-8 Euclidean format:
    one query is split into 292 row parts whose top-k lists one merge
    combines."""
    d, n = 96, 300000
    g = synth.rng(9202, 0)
    cent = synth.centres(1, 32, d)
    X = synth.mixture(1, synth.S_BASE, 0, n, cent, 0.3)
    Q = synth.mixture(1, synth.S_QUERY, 0, 600, cent, 0.3)
    mu = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    fmt = oracle.Format(d, 8, 0, oracle.SEQUENTIAL)
    rows, resid, _ = oracle.encode_rows(fmt, X, mu)
    ix = L.Index(d, 8, 0, L.LVQ_L2, L.LVQ_SEQUENTIAL, capacity=n, means=mu)
    ix.insert(torch.from_numpy(X).cuda())
    dead = np.sort(g.choice(n, n // 20, replace=False)).astype(np.int32)
    ix.delete(torch.from_numpy(dead).cuda())
    assert ix.sync() == 0
    live = np.ones(n, bool)
    live[dead] = False
    ti, td = ix.topk(torch.from_numpy(Q[:1]).cuda(), 10)
    assert ix.sync() == 0
    assert ix.stats().last_parts >= 200
    _scan_case(L, ix, fmt, oracle.L2, Q, rows, resid, mu, live, [(oracle.PRIMARY, L.LVQ_PRIMARY)], ["fp32"],
               (10, 100), 2)
    ix.close()

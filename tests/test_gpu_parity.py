"""GPU parity through the C ABI: encoded rows bit-exact with the oracle,
similarities within the stated tolerance (tests/lvq_check.py), top-k sets
equal up to near-ties."""
import numpy as np
import pytest

import oracle
import synth
from lvq_check import check_topk, check_values, pair_reference

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2402_02044_amd as lib
    return lib


def _special_rows(d, g):
    rows = [np.full(d, 0.75, np.float32),                                   # u == l
            (g.standard_normal(d) * 1e-38).astype(np.float32),              # subnormal spread
            (1000.0 + 0.9 * 255 * 6.1e-5 * g.uniform(-1, 1, d)).astype(np.float32),  # far from mean
            (g.standard_normal(d) * 3e37).astype(np.float32)]               # near overflow
    return np.stack(rows)


ENC_FORMATS = [(96, 8, 0, oracle.SEQUENTIAL), (96, 4, 8, oracle.TURBO), (768, 4, 8, oracle.TURBO),
               (130, 4, 8, oracle.TURBO), (7, 8, 4, oracle.SEQUENTIAL), (200, 4, 4, oracle.SEQUENTIAL),
               (64, 8, 8, oracle.TURBO), (1, 4, 0, oracle.SEQUENTIAL), (512, 8, 0, oracle.SEQUENTIAL),
               (300, 8, 8, oracle.SEQUENTIAL),
               # the largest row whose packing units fit four per lane, and a
               # longer one encoded through the staged (LDS) path
               (2048, 4, 8, oracle.TURBO), (1100, 8, 0, oracle.SEQUENTIAL)]


@pytest.mark.parametrize("d,b1,b2,layout", ENC_FORMATS)
@pytest.mark.parametrize("M", [1, 3, 16])
def test_encode_bit_exact(L, d, b1, b2, layout, M):
    g = synth.rng(1000 + d, b1 * 16 + b2 + M)
    n = 301
    X = np.concatenate([synth.small_vectors(d + M, n - 4, d, ["normal", "uniform", "wide", "lowcard"][d % 4]),
                        _special_rows(d, g)])
    means = (g.standard_normal((M, d)) * 0.5).astype(np.float32)
    if M == 1:
        means = X[:n - 4].astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    fmt = oracle.Format(d, b1, b2, layout)
    ref_rows, ref_res, rej = oracle.encode_rows(fmt, X, means)
    assert rej == 0
    ix = L.Index(d, b1, b2, L.LVQ_L2, layout, means=means)
    rows, res = ix.encode(torch.from_numpy(X).cuda())
    assert ix.sync() == 0
    np.testing.assert_array_equal(rows.cpu().numpy(), ref_rows)
    if b2:
        np.testing.assert_array_equal(res.cpu().numpy(), ref_res)
    ix.close()


def test_encode_nonfinite(L):
    d = 40
    X = synth.small_vectors(5, 9, d)
    X[2, 5] = np.nan
    X[7, 0] = -np.inf
    mu = np.zeros((1, d), np.float32)
    fmt = oracle.Format(d, 4, 8, oracle.TURBO)
    ref_rows, ref_res, rej = oracle.encode_rows(fmt, X, mu)
    assert rej == 2
    ix = L.Index(d, 4, 8, L.LVQ_IP, L.LVQ_TURBO, means=mu)
    rows, res = ix.encode(torch.from_numpy(X).cuda())
    assert ix.sync() == L.LVQ_ERR_NONFINITE
    assert ix.sync() == 0          # the sticky error is cleared by reading it
    got = rows.cpu().numpy()
    np.testing.assert_array_equal(got[:, 4:], ref_rows[:, 4:])
    np.testing.assert_array_equal(np.isnan(got[:, :4].copy().view(np.float32)),
                                  np.isnan(ref_rows[:, :4].copy().view(np.float32)))
    np.testing.assert_array_equal(res.cpu().numpy(), ref_res)
    ix.close()


def _lists(g, nq, n, lens):
    offs = np.zeros(nq + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    ids = np.concatenate([g.choice(n, L_, replace=False) for L_ in lens]).astype(np.int32) \
        if offs[-1] else np.zeros(0, np.int32)
    return offs, ids


DIST_CASES = [
    # d, b1, b2, layout, metric, M
    (96, 8, 0, oracle.SEQUENTIAL, oracle.L2, 1),
    (96, 8, 0, oracle.SEQUENTIAL, oracle.L2, 16),
    (768, 4, 8, oracle.TURBO, oracle.IP, 1),
    (768, 4, 8, oracle.TURBO, oracle.IP, 16),
    (130, 4, 8, oracle.TURBO, oracle.L2, 1),
    (130, 4, 8, oracle.TURBO, oracle.L2, 3),
    (200, 4, 4, oracle.SEQUENTIAL, oracle.IP, 2),
    (512, 8, 0, oracle.SEQUENTIAL, oracle.IP, 1),
    (100, 8, 4, oracle.SEQUENTIAL, oracle.L2, 1),
    (64, 8, 8, oracle.TURBO, oracle.IP, 1),
]


@pytest.mark.parametrize("d,b1,b2,layout,metric,M", DIST_CASES)
def test_candidate_distances_and_topk(L, d, b1, b2, layout, metric, M):
    g = synth.rng(2000 + d, b1 * 16 + b2 + M * 3 + metric)
    n = 2600
    cent = g.standard_normal((8, d)).astype(np.float32)
    X = (cent[g.integers(0, 8, n)] + 0.4 * g.standard_normal((n, d))).astype(np.float32)
    Q = (cent[g.integers(0, 8, 23)] + 0.4 * g.standard_normal((23, d))).astype(np.float32)
    if metric == oracle.IP:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    means = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32) if M == 1 \
        else X[g.choice(n, M, replace=False)]
    fmt = oracle.Format(d, b1, b2, layout)
    rows, resid, _ = oracle.encode_rows(fmt, X, means)
    # ragged lists: empty, single, short, longer than one LDS buffer of keys
    lens = [0, 1, 5, 64, 2500, 37, 1000, 3, 0, 129] + list(g.integers(1, 400, 13))
    offs, ids = _lists(g, 23, n, lens)

    ix = L.Index(d, b1, b2, metric, layout, capacity=n, means=means)
    slots = ix.insert(torch.from_numpy(X).cuda())
    assert ix.sync() == 0
    np.testing.assert_array_equal(slots.cpu().numpy(), np.arange(n))
    dead = np.sort(g.choice(n, 300, replace=False)).astype(np.int32)
    ix.delete(torch.from_numpy(dead).cuda())
    assert ix.sync() == 0
    keep_slot = np.ones(n, bool)
    keep_slot[dead] = False
    qd = torch.from_numpy(Q).cuda()
    od, idd = torch.from_numpy(offs).cuda(), torch.from_numpy(ids).cuda()
    for level in ([oracle.PRIMARY, oracle.FULL] if b2 else [oracle.PRIMARY]):
        ref, tol = pair_reference(fmt, metric, level, Q, rows, resid, means, offs, ids)
        for k in (0, 10, 100):
            dist, ti, td = ix.distances(qd, od, idd, level=level, k=k)
            assert ix.sync() == 0
            check_values(dist.cpu().numpy(), ref, tol)
            if k == 0:
                continue
            ti, td = ti.cpu().numpy(), td.cpu().numpy()
            for i in range(23):
                a, b = offs[i], offs[i + 1]
                check_topk(metric, ti[i], td[i], ids[a:b], ref[a:b], tol[a:b], k, keep_slot[ids[a:b]])
    ix.close()


SHAPE_CASES = [
    (768, 4, 8, oracle.TURBO, oracle.IP, 1),
    (96, 8, 0, oracle.SEQUENTIAL, oracle.L2, 16),
    (512, 8, 0, oracle.SEQUENTIAL, oracle.IP, 1),
]


@pytest.mark.parametrize("d,b1,b2,layout,metric,M", SHAPE_CASES)
def test_every_tile_shape(L, d, b1, b2, layout, metric, M):
    """Every tile shape the format admits (forced with lvq_set_tile) gives the
    oracle's values and top-k on ragged lists."""
    g = synth.rng(2100 + d, b1 + b2 + M)
    n = 1500
    X = g.standard_normal((n, d)).astype(np.float32)
    Q = g.standard_normal((9, d)).astype(np.float32)
    if metric == oracle.IP:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    means = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32) if M == 1 \
        else X[g.choice(n, M, replace=False)]
    fmt = oracle.Format(d, b1, b2, layout)
    rows, resid, _ = oracle.encode_rows(fmt, X, means)
    lens = [0, 1, 3, 64, 65, 130, 700, 1500, 31]
    offs, ids = _lists(g, 9, n, lens)
    ix = L.Index(d, b1, b2, metric, layout, capacity=n, means=means)
    ix.insert(torch.from_numpy(X).cuda())
    assert ix.sync() == 0
    qd = torch.from_numpy(Q).cuda()
    od, idd = torch.from_numpy(offs).cuda(), torch.from_numpy(ids).cuda()
    tested = 0
    for level in ([oracle.PRIMARY, oracle.FULL] if b2 else [oracle.PRIMARY]):
        ref, tol = pair_reference(fmt, metric, level, Q, rows, resid, means, offs, ids)
        for shape in range(L.lvq_num_tile_shapes()):
            for k in (0, 10):
                try:
                    ix.set_tile(level, k > 0, shape)
                    dist, ti, td = ix.distances(qd, od, idd, level=level, k=k)
                except L.LVQError as e:
                    assert e.code == L.LVQ_ERR_UNSUPPORTED
                    continue
                assert ix.sync() == 0
                check_values(dist.cpu().numpy(), ref, tol, "shape %d" % shape)
                tested += 1
                if k:
                    ti, td = ti.cpu().numpy(), td.cpu().numpy()
                    for i in range(9):
                        a, b = offs[i], offs[i + 1]
                        check_topk(metric, ti[i], td[i], ids[a:b], ref[a:b], tol[a:b], k)
        ix.set_tile(level, 0, -1)
        ix.set_tile(level, 1, -1)
    assert tested >= 10
    ix.close()


def _exact_selection(metric, dist, ids, live, k):
    """The k best live entries of one list, ranked by score then slot, with
    repeated ids kept as separate entries: the selection the fused top-k makes
    over the same call's own values (the ranking order of the C ABI)."""
    d = np.asarray(dist, np.float32)
    bits = (-d if metric == oracle.IP else d).view(np.uint32).astype(np.uint64)
    hi = np.where(bits & 0x80000000, ~bits & 0xFFFFFFFF, bits | 0x80000000)
    hi = np.where(np.isnan(d), 0xFFFFFFFF, hi)
    m = live[ids]
    order = np.lexsort((ids[m].astype(np.int64), hi[m]))[:k]
    out_i = np.full(k, -1, np.int32)
    out_d = np.full(k, np.inf if metric == oracle.L2 else -np.inf, np.float32)
    out_i[:len(order)] = ids[m][order]
    out_d[:len(order)] = d[m][order]
    return out_i, out_d


@pytest.mark.parametrize("d,b1,b2,layout,metric", [
    (96, 8, 0, oracle.SEQUENTIAL, oracle.L2),
    (256, 4, 8, oracle.TURBO, oracle.IP),
])
def test_candidate_topk_selection(L, d, b1, b2, layout, metric):
    """Fused per-list top-k on long lists (many times one wave's key buffer),
    lists with repeated ids, deleted entries, and k from 1 to the maximum
    1024: the oracle's ranking within tolerance, and exactly the selection of
    the k best over the values the same call returns."""
    g = synth.rng(2200 + d, b1 + b2)
    n = 5000
    X = g.standard_normal((n, d)).astype(np.float32)
    Q = g.standard_normal((7, d)).astype(np.float32)
    if metric == oracle.IP:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    means = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    fmt = oracle.Format(d, b1, b2, layout)
    rows, resid, _ = oracle.encode_rows(fmt, X, means)
    lens = [4096, 3000, 1030, 0, 700, 2049, 5]
    offs = np.zeros(8, np.int64)
    offs[1:] = np.cumsum(lens)
    parts = []
    for i, L_ in enumerate(lens):
        if i == 4:   # repeated ids: 350 slots listed twice
            base = g.choice(n, 350, replace=False)
            parts.append(g.permutation(np.concatenate([base, base])))
        else:
            parts.append(g.choice(n, L_, replace=False))
    ids = np.concatenate(parts).astype(np.int32)
    ix = L.Index(d, b1, b2, metric, layout, capacity=n, means=means)
    ix.insert(torch.from_numpy(X).cuda())
    dead = np.sort(g.choice(n, 800, replace=False)).astype(np.int32)
    ix.delete(torch.from_numpy(dead).cuda())
    assert ix.sync() == 0
    live = np.ones(n, bool)
    live[dead] = False
    qd = torch.from_numpy(Q).cuda()
    od, idd = torch.from_numpy(offs).cuda(), torch.from_numpy(ids).cuda()
    for level in ([oracle.PRIMARY, oracle.FULL] if b2 else [oracle.PRIMARY]):
        ref, tol = pair_reference(fmt, metric, level, Q, rows, resid, means, offs, ids)
        for k in (1, 10, 100, 300, 1000, 1024):
            dist, ti, td = ix.distances(qd, od, idd, level=level, k=k)
            assert ix.sync() == 0
            dist, ti, td = dist.cpu().numpy(), ti.cpu().numpy(), td.cpu().numpy()
            check_values(dist, ref, tol)
            for i in range(7):
                a, b = offs[i], offs[i + 1]
                check_topk(metric, ti[i], td[i], ids[a:b], ref[a:b], tol[a:b], k, live[ids[a:b]])
                ei, ed = _exact_selection(metric, dist[a:b], ids[a:b], live, k)
                np.testing.assert_array_equal(ti[i], ei, err_msg="list %d k %d ids" % (i, k))
                np.testing.assert_array_equal(td[i], ed, err_msg="list %d k %d values" % (i, k))
    ix.close()


def test_duplicate_ids_and_bad_slots(L):
    d, n = 96, 500
    X = synth.small_vectors(11, n, d)
    mu = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    fmt = oracle.Format(d, 8, 0)
    rows, _, _ = oracle.encode_rows(fmt, X, mu)
    ix = L.Index(d, 8, 0, L.LVQ_L2, L.LVQ_SEQUENTIAL, capacity=n, means=mu)
    ix.insert(torch.from_numpy(X).cuda())
    offs = np.array([0, 6], np.int64)
    ids = np.array([4, 4, 9, 4, 0, 9], np.int32)
    Q = synth.small_vectors(12, 1, d)
    ref, tol = pair_reference(fmt, oracle.L2, oracle.PRIMARY, Q, rows, None, mu, offs, ids)
    dist, ti, td = ix.distances(torch.from_numpy(Q).cuda(), torch.from_numpy(offs).cuda(),
                                torch.from_numpy(ids).cuda(), k=4)
    assert ix.sync() == 0
    check_values(dist.cpu().numpy(), ref, tol)
    # duplicates are scored once per entry
    assert sorted(ti.cpu().numpy()[0].tolist()) == sorted(ids[np.lexsort((ids, ref))][:4].tolist())
    bad = np.array([1, -3, n + 5], np.int32)
    dist, _, _ = ix.distances(torch.from_numpy(Q).cuda(), torch.tensor([0, 3], dtype=torch.int64).cuda(),
                              torch.from_numpy(bad).cuda())
    assert ix.sync() == L.LVQ_ERR_BAD_SLOT
    got = dist.cpu().numpy()
    assert not np.isnan(got[0]) and np.isnan(got[1]) and np.isnan(got[2])
    ix.close()


EXH_CASES = [
    (96, 8, 0, oracle.SEQUENTIAL, oracle.L2, 1),
    (768, 4, 8, oracle.TURBO, oracle.IP, 16),
    (512, 8, 0, oracle.SEQUENTIAL, oracle.IP, 1),
    (130, 4, 8, oracle.TURBO, oracle.L2, 1),
    (100, 8, 0, oracle.SEQUENTIAL, oracle.L2, 1),
]


@pytest.mark.parametrize("d,b1,b2,layout,metric,M", EXH_CASES)
def test_exhaustive_topk(L, d, b1, b2, layout, metric, M):
    g = synth.rng(3000 + d, M + metric)
    n, nq = 3000, 21
    cent = g.standard_normal((8, d)).astype(np.float32)
    X = (cent[g.integers(0, 8, n)] + 0.4 * g.standard_normal((n, d))).astype(np.float32)
    Q = (cent[g.integers(0, 8, nq)] + 0.4 * g.standard_normal((nq, d))).astype(np.float32)
    means = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32) if M == 1 \
        else X[g.choice(n, M, replace=False)]
    fmt = oracle.Format(d, b1, b2, layout)
    rows, resid, _ = oracle.encode_rows(fmt, X, means)
    ix = L.Index(d, b1, b2, metric, layout, capacity=n + 100, means=means)
    ix.insert(torch.from_numpy(X).cuda())
    dead = np.sort(g.choice(n, 250, replace=False)).astype(np.int32)
    ix.delete(torch.from_numpy(dead).cuda())
    assert ix.sync() == 0
    live = np.ones(n, bool)
    live[dead] = False
    offs = np.arange(nq + 1, dtype=np.int64) * n
    allids = np.tile(np.arange(n, dtype=np.int32), nq)
    # inner product: the FP32 matrix cores and the plain vector kernel
    for plain in ((False, True) if metric == oracle.IP else (False,)):
        for level in ([oracle.PRIMARY, oracle.FULL] if b2 else [oracle.PRIMARY]):
            ref, tol = pair_reference(fmt, metric, level, Q, rows, resid, means, offs, allids)
            for k in (1, 10, 100):
                ti, td = ix.topk(torch.from_numpy(Q).cuda(), k, level=level, plain=plain)
                assert ix.sync() == 0
                ti, td = ti.cpu().numpy(), td.cpu().numpy()
                for i in range(nq):
                    a, b = offs[i], offs[i + 1]
                    check_topk(metric, ti[i], td[i], allids[a:b], ref[a:b], tol[a:b], k, live)
    ix.close()


def test_store_sequence_matches_model(L):
    """Insert / delete / consolidate: slots follow the free-stack order (pops
    ascend from 0; consolidation pushes freed slots so they pop ascending),
    stored rows equal the oracle's, tombstoned slots leave the top-k."""
    d, cap = 64, 300
    g = synth.rng(4000, 0)
    mu = np.zeros((1, d), np.float32)
    fmt = oracle.Format(d, 4, 8, oracle.TURBO)
    ix = L.Index(d, 4, 8, L.LVQ_IP, L.LVQ_TURBO, capacity=cap, means=mu)
    X1 = g.standard_normal((200, d)).astype(np.float32)
    s1 = ix.insert(torch.from_numpy(X1).cuda()).cpu().numpy()
    np.testing.assert_array_equal(s1, np.arange(200))
    dead = np.array([3, 50, 199, 120], np.int32)
    ix.delete(torch.from_numpy(dead).cuda())
    assert ix.consolidate() == 4
    X2 = g.standard_normal((7, d)).astype(np.float32)
    s2 = ix.insert(torch.from_numpy(X2).cuda()).cpu().numpy()
    np.testing.assert_array_equal(s2, [3, 50, 120, 199, 200, 201, 202])
    assert ix.sync() == 0
    rows, resid = ix.read_rows(torch.from_numpy(s2).cuda())
    ref_rows, ref_res, _ = oracle.encode_rows(fmt, X2, mu)
    got = rows.cpu().numpy()
    np.testing.assert_array_equal(got[:, :13], ref_rows[:, :13])   # l, Delta, Delta2, mean id
    np.testing.assert_array_equal(got[:, 32:], ref_rows[:, 32:])
    np.testing.assert_array_equal(resid.cpu().numpy(), ref_res)
    assert np.all(got[:, 13] == 1)                                  # occupied
    assert np.all(got[:, 20:24].copy().view(np.uint32) == 0xFFFFFFFF)
    # capacity: 300 - 203 = 97 free
    with pytest.raises(L.LVQError) as e:
        ix.insert(torch.from_numpy(g.standard_normal((98, d)).astype(np.float32)).cuda())
    assert e.value.code == L.LVQ_ERR_CAPACITY
    # deleting a dead slot is reported
    ix.delete(torch.tensor([5, 5000], dtype=torch.int32).cuda())
    ix.delete(torch.tensor([5], dtype=torch.int32).cuda())
    assert ix.sync() == L.LVQ_ERR_BAD_SLOT
    st = ix.stats()
    assert st.free_slots == 97 and st.capacity == cap
    ix.close()


def test_invalid_arguments(L):
    import ctypes
    cfg = L.lvq_config(96, 5, 0, 0, 0, 32, 0, 0)
    with pytest.raises(L.LVQError) as e:
        L.lvq_row_format(cfg)
    assert e.value.code == L.LVQ_ERR_INVALID_ARG
    ix = L.Index(16, 8, 0, L.LVQ_L2, L.LVQ_SEQUENTIAL, capacity=10, means=np.zeros(16, np.float32))
    q = torch.zeros((1, 16), device="cuda")
    offs = torch.tensor([0, 1], dtype=torch.int64, device="cuda")
    ids = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(L.LVQError) as e:      # FULL needs a residual level
        ix.distances(q, offs, ids, level=L.LVQ_FULL)
    assert e.value.code == L.LVQ_ERR_INVALID_ARG
    with pytest.raises(L.LVQError):
        ix.distances(q, offs, ids, k=5000)
    with pytest.raises(L.LVQError) as e:
        L.lvq_create(L.lvq_config(16, 8, 0, 0, 0, 32, 0, 0), np.zeros(16, np.float32).ctypes.data, 0)
    assert e.value.code == L.LVQ_ERR_INVALID_ARG
    bad = np.full(16, np.nan, np.float32)
    with pytest.raises(L.LVQError) as e:
        L.lvq_create(L.lvq_config(16, 8, 0, 0, 0, 32, 0, 0), bad.ctypes.data, 1)
    assert e.value.code == L.LVQ_ERR_NONFINITE
    with pytest.raises(L.LVQError) as e:       # memory budget below the store
        L.Index(768, 4, 8, L.LVQ_IP, L.LVQ_TURBO, capacity=100000, mem_budget_bytes=1 << 20)
    assert e.value.code == L.LVQ_ERR_OOM
    assert ctypes is not None
    ix.close()


def test_mean_and_kmeans(L):
    g = synth.rng(5000, 0)
    X = (g.standard_normal((20000, 24)) + 3.0).astype(np.float32)
    m = L.mean(torch.from_numpy(X).cuda()).cpu().numpy()
    np.testing.assert_allclose(m, X.astype(np.float64).mean(0), rtol=0, atol=1e-6)
    cent = (g.standard_normal((5, 24)) * 4).astype(np.float32)
    lab = g.integers(0, 5, 5000)
    Y = (cent[lab] + 0.2 * g.standard_normal((5000, 24))).astype(np.float32)
    init = [int(np.flatnonzero(lab == c)[0]) for c in range(5)]
    C = L.kmeans(torch.from_numpy(Y).cuda(), 5, init, iters=10).cpu().numpy()
    np.testing.assert_allclose(C, cent, atol=0.05)
    # a fixed point of Lloyd: every centre is the mean of its members
    d2 = ((Y[:, None, :].astype(np.float64) - C[None]) ** 2).sum(-1)
    a = d2.argmin(1)
    for c in range(5):
        np.testing.assert_allclose(C[c], Y[a == c].astype(np.float64).mean(0), atol=1e-5)


MFMA_CASES = [
    (512, 8, 0, oracle.SEQUENTIAL, 1),
    (768, 4, 8, oracle.TURBO, 16),
    (96, 8, 0, oracle.SEQUENTIAL, 1),
    (256, 4, 0, oracle.TURBO, 2),
    (256, 8, 8, oracle.SEQUENTIAL, 3),
    (512, 4, 8, oracle.TURBO, 1),
    (128, 4, 4, oracle.TURBO, 1),
    (384, 4, 0, oracle.TURBO, 1),   # six chunks of 64 positions: a three-chunk ring
]


@pytest.mark.parametrize("d,b1,b2,layout,M", MFMA_CASES)
@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp32"])
def test_exhaustive_topk_mfma(L, d, b1, b2, layout, M, prec):
    """Matrix-core form: 16-bit queries x exactly converted codes, FP32
    accumulation, at the first level and (8-bit residual codes) at both
    levels.  The oracle runs on the same 16-bit query values (upcast exactly),
    so the only difference left is FP32 accumulation order.  FP32 queries:
    the first level with one mean runs on the FP32 matrix cores (codes
    converted exactly, FP32 products), the rest on the vector path."""
    g = synth.rng(3100 + d, M + {"bf16": 0, "fp16": 1, "fp32": 2}[prec])
    n, nq = 3000, 70
    cent = g.standard_normal((8, d)).astype(np.float32)
    X = (cent[g.integers(0, 8, n)] + 0.4 * g.standard_normal((n, d))).astype(np.float32)
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    Q = (cent[g.integers(0, 8, nq)] + 0.4 * g.standard_normal((nq, d))).astype(np.float32)
    Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    tdt = {"bf16": torch.bfloat16, "fp16": torch.float16, "fp32": torch.float32}[prec]
    Qh = torch.from_numpy(Q).to(tdt)
    Qr = Qh.float().numpy()
    means = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32) if M == 1 \
        else X[g.choice(n, M, replace=False)]
    fmt = oracle.Format(d, b1, b2, layout)
    rows, resid, _ = oracle.encode_rows(fmt, X, means)
    ix = L.Index(d, b1, b2, L.LVQ_IP, layout, capacity=n + 50, means=means)
    ix.insert(torch.from_numpy(X).cuda())
    dead = np.sort(g.choice(n, 200, replace=False)).astype(np.int32)
    ix.delete(torch.from_numpy(dead).cuda())
    assert ix.sync() == 0
    live = np.ones(n, bool)
    live[dead] = False
    offs = np.arange(nq + 1, dtype=np.int64) * n
    allids = np.tile(np.arange(n, dtype=np.int32), nq)
    levels = [(oracle.PRIMARY, L.LVQ_PRIMARY)] + ([(oracle.FULL, L.LVQ_FULL)] if b2 == 8 else [])
    for olev, glev in levels:
        ref, tol = pair_reference(fmt, oracle.IP, olev, Qr, rows, resid, means, offs, allids)
        # k = 300 and 512: 512 sorted keys per query in the queries-in-LDS
        # kernel, which takes the first level and both levels with 8-bit
        # residual codes, any of these mean counts
        wide = (olev == oracle.FULL and b2 == 8) or (olev == oracle.PRIMARY and (M == 1 or prec == "fp32"))
        big = (300,) + ((512,) if (M == 1 and olev == oracle.PRIMARY and prec == "bf16") or
                        (M > 1 and olev == oracle.FULL and prec == "fp32") else ())
        for k in (1, 10, 100) + (big if wide else ()):
            ti, td = ix.topk(Qh.cuda(), k, level=glev)
            assert ix.sync() == 0
            ti, td = ti.cpu().numpy(), td.cpu().numpy()
            for i in range(nq):
                a, b = offs[i], offs[i + 1]
                check_topk(oracle.IP, ti[i], td[i], allids[a:b], ref[a:b], tol[a:b], k, live)
    if b2 == 4 and prec != "fp32":   # both levels on the matrix cores need 8-bit residual codes
        with pytest.raises(L.LVQError) as e:
            ix.topk(Qh.cuda(), 10, level=L.LVQ_FULL)
        assert e.value.code == L.LVQ_ERR_UNSUPPORTED
    ix.close()


@pytest.mark.parametrize("b2", [0, 8])
def test_exhaustive_topk_many_means(L, b2):
    """Two hundred means: the queries-in-LDS kernel's c_m table at the size
    a large M-LVQ store reaches (FP32 at either level, bf16 at both levels),
    the rows' mean ids spread over all of them, nq past one query tile."""
    d, n, nq, M = 96, 4000, 150, 200
    g = synth.rng(3400 + b2, M)
    cent = g.standard_normal((M, d)).astype(np.float32)
    X = (cent[g.integers(0, M, n)] + 0.3 * g.standard_normal((n, d))).astype(np.float32)
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    Q = (cent[g.integers(0, M, nq)] + 0.3 * g.standard_normal((nq, d))).astype(np.float32)
    Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    means = X[g.choice(n, M, replace=False)]
    fmt = oracle.Format(d, 8, b2, oracle.SEQUENTIAL)
    rows, resid, _ = oracle.encode_rows(fmt, X, means)
    assert len(np.unique(rows[:, 12])) > M // 2   # the rows use many of the means
    ix = L.Index(d, 8, b2, L.LVQ_IP, L.LVQ_SEQUENTIAL, capacity=n, means=means)
    ix.insert(torch.from_numpy(X).cuda())
    dead = np.sort(g.choice(n, 300, replace=False)).astype(np.int32)
    ix.delete(torch.from_numpy(dead).cuda())
    assert ix.sync() == 0
    live = np.ones(n, bool)
    live[dead] = False
    offs = np.arange(nq + 1, dtype=np.int64) * n
    allids = np.tile(np.arange(n, dtype=np.int32), nq)
    levels = [(oracle.PRIMARY, L.LVQ_PRIMARY)] + ([(oracle.FULL, L.LVQ_FULL)] if b2 else [])
    for prec, tdt in (("fp32", torch.float32), ("bf16", torch.bfloat16)):
        Qh = torch.from_numpy(Q).to(tdt)
        Qr = Qh.float().numpy()
        for olev, glev in levels:
            if prec == "bf16" and olev == oracle.PRIMARY:
                continue   # the register-resident kernel; its per-query buffers cap the mean count
            ref, tol = pair_reference(fmt, oracle.IP, olev, Qr, rows, resid, means, offs, allids)
            for k in (10, 100):
                ti, td = ix.topk(Qh.cuda(), k, level=glev)
                assert ix.sync() == 0
                ti, td = ti.cpu().numpy(), td.cpu().numpy()
                for i in range(nq):
                    a, b = offs[i], offs[i + 1]
                    check_topk(oracle.IP, ti[i], td[i], allids[a:b], ref[a:b], tol[a:b], k, live)
    ix.close()


def test_mfma_rejects_l2(L):
    ix = L.Index(96, 8, 0, L.LVQ_L2, L.LVQ_SEQUENTIAL, capacity=100, means=np.zeros(96, np.float32))
    ix.insert(torch.zeros((10, 96), device="cuda"))
    with pytest.raises(L.LVQError) as e:
        ix.topk(torch.zeros((4, 96), dtype=torch.bfloat16, device="cuda"), 5)
    assert e.value.code == L.LVQ_ERR_UNSUPPORTED
    ix.close()


def test_graph_capture_replays_match_eager(L):
    """A captured lvq_distances (query prep, list ordering, persistent
    candidate kernel) replays to the eager result, several times, with eager
    work and synchronisation between replays."""
    d, n, nq = 96, 4000, 40
    g = synth.rng(6000, 0)
    X = g.standard_normal((n, d)).astype(np.float32)
    Q = g.standard_normal((nq, d)).astype(np.float32)
    means = X[g.choice(n, 4, replace=False)]
    ix = L.Index(d, 8, 0, L.LVQ_L2, L.LVQ_SEQUENTIAL, capacity=n, means=means)
    ix.insert(torch.from_numpy(X).cuda())
    offs, ids = synth.candidate_lists(7, nq, n, lmin=5, lmax=900)
    qd = torch.from_numpy(Q).cuda()
    od, idd = torch.from_numpy(offs).cuda(), torch.from_numpy(ids).cuda()
    assert ix.sync() == 0
    dist0, ti0, td0 = ix.distances(qd, od, idd, k=10)
    assert ix.sync() == 0
    dist = torch.empty_like(dist0)
    ti = torch.empty_like(ti0)
    td = torch.empty_like(td0)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())

    def call(stream):
        L.lvq_distances(ix.handle, qd.data_ptr(), nq, od.data_ptr(), idd.data_ptr(), ids.shape[0], L.LVQ_PRIMARY,
                        dist.data_ptr(), 10, ti.data_ptr(), td.data_ptr(), int(stream.cuda_stream))

    with torch.cuda.stream(s):
        call(s)                               # sizes this stream's workspace
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        call(s)
    torch.cuda.synchronize()
    for r in range(4):
        dist.fill_(-1.0)
        ti.fill_(-7)
        td.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(dist, dist0), r
        assert torch.equal(ti, ti0) and torch.equal(td, td0), r
    # the captured stream's workspace is fixed now: a larger batch on that
    # stream is refused (the graph still reads the buffers it would grow), a
    # smaller one runs in them, and replays still match
    q3 = torch.cat([qd, qd, qd])
    o3 = torch.from_numpy(np.concatenate([offs[:-1], offs[:-1] + offs[-1], offs + 2 * offs[-1]])).cuda()
    i3 = torch.cat([idd, idd, idd])
    d3 = torch.empty(3 * ids.shape[0], device="cuda")
    t3 = torch.empty((3 * nq, 10), dtype=torch.int32, device="cuda")
    v3 = torch.empty((3 * nq, 10), device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(L.LVQError) as e:
        L.lvq_distances(ix.handle, q3.data_ptr(), 3 * nq, o3.data_ptr(), i3.data_ptr(), 3 * ids.shape[0],
                        L.LVQ_PRIMARY, d3.data_ptr(), 10, t3.data_ptr(), v3.data_ptr(), int(s.cuda_stream))
    assert e.value.code == L.LVQ_ERR_INVALID_ARG
    L.lvq_distances(ix.handle, q3.data_ptr(), 3 * nq, o3.data_ptr(), i3.data_ptr(), 3 * ids.shape[0],
                    L.LVQ_PRIMARY, d3.data_ptr(), 10, t3.data_ptr(), v3.data_ptr(), 0)   # another stream
    h = nq // 2
    tot = int(offs[h])
    L.lvq_distances(ix.handle, qd.data_ptr(), h, od.data_ptr(), idd.data_ptr(), tot, L.LVQ_PRIMARY,
                    d3.data_ptr(), 10, t3.data_ptr(), v3.data_ptr(), int(s.cuda_stream))
    torch.cuda.synchronize()
    assert torch.equal(d3[:tot], dist0[:tot]) and torch.equal(t3[:h], ti0[:h]) and torch.equal(v3[:h], td0[:h])
    dist.fill_(-1.0)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    assert torch.equal(dist, dist0) and torch.equal(ti, ti0) and torch.equal(td, td0)
    assert ix.sync() == 0
    ix.close()

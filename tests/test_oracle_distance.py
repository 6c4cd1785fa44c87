"""Pins of the oracle's similarities and top-k (Sec. 2.1, Sec. 3.2).

The reference values here come from an independent numpy decoder of the row
bytes (header read with frombuffer, codes placed with the paper's worked
example read as a dim -> (word, nibble) rule) and binary64 brute force, plus
the algebraic decompositions the GPU kernels rely on."""
import numpy as np
import pytest

import oracle
import synth


def _np_decode(fmt, rows, resid):
    """Independent decoder: (l, Delta, Delta2, mean id, c1, c2) per row."""
    n = rows.shape[0]
    hdr = rows[:, :12].copy().view(np.float32)
    mid = rows[:, 12].astype(np.int64)
    d = fmt.dim
    c1 = np.zeros((n, d), np.int64)
    c2 = np.zeros((n, d), np.int64)
    codes = rows[:, 32:]
    for j in range(d):
        if fmt.layout == oracle.TURBO:
            blk = 128 if fmt.bits1 == 4 else 64
            per = 32 // fmt.bits1
            b, r = divmod(j, blk)
            w, k = r % 16, r // 16
            pos = b * blk + per * w + k
        else:
            pos = j
        if fmt.bits1 == 4:
            c1[:, j] = (codes[:, pos // 2] >> (4 * (pos % 2))) & 0xF
        else:
            c1[:, j] = codes[:, pos]
        if fmt.bits2 == 8:
            c2[:, j] = resid[:, pos]
        elif fmt.bits2 == 4:
            c2[:, j] = (resid[:, pos // 2] >> (4 * (pos % 2))) & 0xF
    return hdr[:, 0], hdr[:, 1], hdr[:, 2], mid, c1, c2


def _setup(d, b1, b2, layout, M, n=40, nq=5, seed=1):
    g = synth.rng(555, seed)
    means = g.standard_normal((M, d)).astype(np.float32)
    X = (means[g.integers(0, M, n)] + 0.5 * g.standard_normal((n, d))).astype(np.float32)
    Q = g.standard_normal((nq, d)).astype(np.float32)
    fmt = oracle.Format(d, b1, b2, layout)
    rows, resid, rej = oracle.encode_rows(fmt, X, means)
    assert rej == 0
    return fmt, means, X, Q, rows, resid


CASES = [(96, 8, 0, oracle.SEQUENTIAL, 1), (130, 4, 8, oracle.TURBO, 3),
         (200, 4, 4, oracle.SEQUENTIAL, 1), (64, 8, 8, oracle.TURBO, 2), (7, 4, 8, oracle.TURBO, 1)]


@pytest.mark.parametrize("d,b1,b2,layout,M", CASES)
@pytest.mark.parametrize("level", [oracle.PRIMARY, oracle.FULL])
def test_distances_match_bruteforce(d, b1, b2, layout, M, level):
    fmt, means, X, Q, rows, resid = _setup(d, b1, b2, layout, M)
    l, dl, dl2, mid, c1, c2 = _np_decode(fmt, rows, resid)
    xh = means[mid].astype(np.float64) + l[:, None].astype(np.float64) + dl[:, None] * c1
    if level == oracle.FULL and b2:
        xh = xh - dl[:, None].astype(np.float64) / 2 + dl2[:, None].astype(np.float64) * c2
    np.testing.assert_allclose(oracle.reconstruct(fmt, rows, resid, means, level), xh,
                               rtol=0, atol=1e-12)
    n = X.shape[0]
    offsets = np.arange(0, Q.shape[0] + 1, dtype=np.int64) * n
    ids = np.tile(np.arange(n, dtype=np.int32), Q.shape[0])
    Qd = Q.astype(np.float64)
    ip = (Qd @ xh.T).ravel()
    l2 = ((Qd[:, None, :] - xh[None]) ** 2).sum(-1).ravel()
    got_ip = oracle.distances(fmt, oracle.IP, level, Q, rows, resid, means, offsets, ids)
    got_l2 = oracle.distances(fmt, oracle.L2, level, Q, rows, resid, means, offsets, ids)
    np.testing.assert_allclose(got_ip, ip, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(got_l2, l2, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d,b1,b2,layout,M", CASES)
def test_decomposition_identities(d, b1, b2, layout, M):
    """Sec. 3.2: with per-query constants c_m = <q, mu_m>, the inner product is
    c_m + (l [- Delta/2]) sum(q) + Delta <q, c1> [+ Delta2 <q, c2>]; the squared
    distance is ||(q - mu_m) - x'||^2 with x' = l + Delta c1 [- Delta/2 + Delta2 c2]."""
    fmt, means, X, Q, rows, resid = _setup(d, b1, b2, layout, M, seed=2)
    l, dl, dl2, mid, c1, c2 = _np_decode(fmt, rows, resid)
    n = X.shape[0]
    offsets = np.array([0, n], np.int64)
    ids = np.arange(n, dtype=np.int32)
    for level in (oracle.PRIMARY, oracle.FULL):
        full = level == oracle.FULL and b2 > 0
        for q in Q:
            qd = q.astype(np.float64)
            cm = means.astype(np.float64) @ qd
            lo = l.astype(np.float64) - (dl.astype(np.float64) / 2 if full else 0.0)
            ip = cm[mid] + lo * qd.sum() + dl * (c1 @ qd)
            if full:
                ip = ip + dl2 * (c2 @ qd)
            xp = lo[:, None] + dl[:, None].astype(np.float64) * c1
            if full:
                xp = xp + dl2[:, None].astype(np.float64) * c2
            l2 = (((qd[None] - means[mid].astype(np.float64)) - xp) ** 2).sum(1)
            got_ip = oracle.distances(fmt, oracle.IP, level, q[None], rows, resid, means, offsets, ids)
            got_l2 = oracle.distances(fmt, oracle.L2, level, q[None], rows, resid, means, offsets, ids)
            np.testing.assert_allclose(got_ip, ip, rtol=1e-12, atol=1e-12)
            np.testing.assert_allclose(got_l2, l2, rtol=1e-12, atol=1e-12)


def test_full_level_is_closer_than_primary():
    """The second level refines the first: two-level error below one-level."""
    fmt, means, X, Q, rows, resid = _setup(130, 4, 8, oracle.TURBO, 1, n=60)
    e1 = ((oracle.reconstruct(fmt, rows, resid, means, oracle.PRIMARY) - X) ** 2).sum()
    e2 = ((oracle.reconstruct(fmt, rows, resid, means, oracle.FULL) - X) ** 2).sum()
    assert e2 < e1 / 100


@pytest.mark.parametrize("metric", [oracle.L2, oracle.IP])
def test_topk_order_ties_and_padding(metric):
    g = synth.rng(556, metric)
    score = np.round(g.standard_normal(300), 1)     # many exact ties
    slot = g.permutation(1000)[:300].astype(np.int32)
    keep = (g.uniform(size=300) > 0.2).astype(np.uint8)
    score[5] = np.nan
    k = 17
    ts, tv = oracle.select_topk(metric, score, slot, k, keep)
    m = keep.astype(bool) & ~np.isnan(score)
    key = score[m] if metric == oracle.L2 else -score[m]
    order = np.lexsort((slot[m], key))[:k]
    np.testing.assert_array_equal(ts, slot[m][order])
    np.testing.assert_array_equal(tv, score[m][order])
    # fewer survivors than k: padded with -1 and the worst value
    ts, tv = oracle.select_topk(metric, score[:3], slot[:3], 6, np.array([1, 0, 1], np.uint8))
    assert list(ts[2:]) == [-1] * 4
    assert np.all(tv[2:] == (np.inf if metric == oracle.L2 else -np.inf))
    # NaN ranks after every number
    ts, tv = oracle.select_topk(metric, np.array([np.nan, 1.0]), np.array([0, 1], np.int32), 2)
    assert list(ts) == [1, 0]


def test_exhaustive_topk_and_recall():
    fmt, means, X, Q, rows, resid = _setup(96, 8, 0, oracle.SEQUENTIAL, 1, n=200, nq=4)
    live = np.ones(200, bool)
    live[::7] = False
    ts, tv = oracle.topk_exhaustive(fmt, oracle.L2, oracle.PRIMARY, Q, rows, None, means, 10, live)
    assert not np.any(np.isin(ts, np.flatnonzero(~live)))
    gt = oracle.float_groundtruth(oracle.L2, Q, X, 10, live)
    xh = oracle.reconstruct(fmt, rows, None, means)
    for i in range(4):
        d = ((Q[i].astype(np.float64) - xh) ** 2).sum(1)
        d[~live] = np.inf
        np.testing.assert_array_equal(ts[i], np.lexsort((np.arange(200), d))[:10])
        dx = ((Q[i].astype(np.float64) - X) ** 2).sum(1)
        dx[~live] = np.inf
        np.testing.assert_array_equal(np.sort(gt[i]), np.sort(np.argsort(dx, kind="stable")[:10]))
    assert oracle.recall(ts, gt) >= 0.9
    assert oracle.recall(gt, gt) == 1.0


def test_recall_hand_value():
    # Sec. 2.1: k-recall@k = |S n G| / k averaged over queries; order and
    # padding do not count.  Query 0: {3, 2} of G = {3, 2, 9} found (2 of 3);
    # query 1: {4} of {7, 8, 4} (1 of 3): (2 + 1) / 6 = 0.5
    found = np.array([[1, 2, 3], [4, 5, -1]])
    truth = np.array([[3, 2, 9], [7, 8, 4]])
    assert oracle.recall(found, truth) == 0.5
    assert oracle.recall(found[:, ::-1], truth) == 0.5
    assert oracle.recall(truth[:, ::-1], truth) == 1.0
    # an id returned twice counts once
    assert oracle.recall(np.array([[3, 3, 2]]), np.array([[3, 2, 9]])) == 2.0 / 3.0

"""Graph construction on the GPU (lvq_graph_prune, lvq_graph_build of the C
ABI) against the oracle's Alg. 2 and App. A update routine.

* Pruning: every pruned row equals the oracle's robust_prune of the same
  candidates and current out-neighbours (binary32 against binary64 may decide
  a near-tie of the pruning rule differently: nearly every row, not all).
  Long candidate lists are pruned in groups (whole blocks of 256 positions,
  as many as fit beside the kept out-neighbours): the result equals the
  oracle's pruning folded over the same groups.
* Build with batches of one node is the paper's sequential routine: the rows
  equal the oracle's vamana_build (as sets; again nearly all rows).
* Batched build: rows are valid (distinct, no self edge, -1 padded at the
  end), nearly every node is found by a walk (where the sequential routine
  finds all), and greedy search over the LVQ store with the built graph
  reaches high recall.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2402_02044_amd as lib
    return lib


def _rows_ok(graph, n, nodes=None):
    for i in (range(n) if nodes is None else nodes):
        row = graph[i]
        k = int((row >= 0).sum())
        assert (row[:k] >= 0).all() and (row[k:] == -1).all(), i
        v = row[:k]
        assert (v < n).all() and i not in v.tolist() and len(set(v.tolist())) == k, i


@pytest.mark.parametrize("metric,alpha,d", [(0, 1.2, 48), (1, 0.95, 48), (0, 1.0, 48), (0, 1.2, 160)])
def test_prune_matches_oracle(L, metric, alpha, d):
    g = synth.rng(9000 + d, metric)
    n, R, m = 2000, 16, 300
    X = g.standard_normal((n, d)).astype(np.float32)
    if metric == oracle.IP:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    graph = g.integers(-1, n, (n, R)).astype(np.int32)   # arbitrary current rows (may hold repeats, -1)
    nodes = g.choice(n, m, replace=False).astype(np.int32)
    lens = g.integers(0, 257, m)
    lens[0] = 600                                        # three groups of candidates
    lens[1] = 0                                          # only the current out-neighbours
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cand = g.integers(-1, n, int(offs[-1])).astype(np.int32)
    for i in range(m):                                   # the node itself and repeats among its candidates
        if lens[i] > 4:
            cand[offs[i]] = nodes[i]
            cand[offs[i] + 1] = cand[offs[i] + 2]
    before = graph.copy()
    gd = torch.from_numpy(graph).cuda()
    L.graph_prune(torch.from_numpy(X).cuda(), torch.from_numpy(nodes).cuda(), torch.from_numpy(offs).cuda(),
                  torch.from_numpy(cand).cuda(), gd, alpha, metric)
    got = gd.cpu().numpy()
    same = 0
    for i, p in enumerate(nodes):
        c = cand[offs[i]:offs[i + 1]]
        cur = [int(v) for v in before[p] if 0 <= v < n and v != p]   # repeats included, as the kernel reads the row
        pos = 0
        while True:
            # the kernel's groups: whole blocks of 256 candidate positions, in
            # order, while their valid entries fit beside the kept ones (320)
            group = []
            while pos < len(c):
                valid = [int(y) for y in c[pos:pos + 256] if 0 <= y < n and y != p]
                if len(cur) + len(group) + len(valid) > 320:
                    break
                group += valid
                pos += 256
            cur = oracle.robust_prune(metric, X, int(p), group, cur, alpha, R)
            if pos >= len(c):
                break
        row = got[p][got[p] >= 0].tolist()
        same += row == cur
    assert same >= m - 3, "%d of %d pruned rows equal the oracle's" % (same, m)
    untouched = np.setdiff1d(np.arange(n), nodes)
    np.testing.assert_array_equal(got[untouched], before[untouched])
    _rows_ok(got, n, nodes)


@pytest.mark.parametrize("metric,alpha", [(0, 1.2), (1, 0.95)])
def test_sequential_build_matches_oracle(L, metric, alpha):
    g = synth.rng(9100, metric)
    n, d, R, W = 600, 16, 10, 24
    X = g.standard_normal((n, d)).astype(np.float32)
    if metric == oracle.IP:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    entry = int(np.argmin(((X - X.mean(0)) ** 2).sum(1)))
    got = L.graph_build(torch.from_numpy(X).cuda(), R, W, alpha, metric, entry, passes=2, max_batch=1).cpu().numpy()
    want = oracle.vamana_build(metric, X, entry, W, alpha, R)
    _rows_ok(got, n)
    same = sum(set(got[i][got[i] >= 0].tolist()) == set(want[i][want[i] >= 0].tolist()) for i in range(n))
    assert same >= int(0.95 * n), "%d of %d rows equal the oracle's sequential build" % (same, n)


def test_batched_build_and_insert(L):
    # 8-d data: the oracle's sequential routine (two passes over the first
    # 2400 nodes, then one over the rest) leaves every node findable by a walk
    # from the entry at W = 32; in 24-d it misses 20 of the 600 inserted ones
    g = synth.rng(9200, 0)
    n, n0, d, R, W = 3000, 2400, 8, 16, 32
    X = g.standard_normal((n, d)).astype(np.float32)
    xd = torch.from_numpy(X).cuda()
    entry = int(np.argmin(((X[:n0] - X[:n0].mean(0)) ** 2).sum(1)))
    graph = torch.full((n, R), -7, dtype=torch.int32, device="cuda")
    # the initial build over the first n0 nodes (rows beyond n0 untouched)
    L.graph_build(xd[:n0].contiguous(), R, W, 1.2, 0, entry, passes=2, max_batch=256, graph=graph[:n0])
    g0 = graph.cpu().numpy()
    assert (g0[n0:] == -7).all()
    _rows_ok(g0, n0)
    # insert the rest with one pass
    graph[n0:] = -1
    L.graph_build(xd, R, W, 1.2, 0, entry, passes=1, first=n0, max_batch=128, graph=graph)
    g1 = graph.cpu().numpy()
    _rows_ok(g1, n)
    # nodes found by a walk from the entry with themselves as the query: the
    # batched routine (a batch searches the graph as it was before the batch)
    # against the sequential routine's all
    found_old = sum(int(oracle.greedy_search_float(0, X[i], X, g0, [entry], W, 1)[0][0] == i) for i in range(n0))
    found_new = sum(int(oracle.greedy_search_float(0, X[i], X, g1, [entry], W, 1)[0][0] == i) for i in range(n0, n))
    assert found_old >= int(0.99 * n0) and found_new >= int(0.99 * (n - n0)), (found_old, found_new)
    # the inserted nodes got in-edges from old nodes (the reverse edges)
    assert sum(int((g1[i] >= n0).any()) for i in range(n0)) >= (n - n0) // 2


def test_built_graph_search_recall(L):
    g = synth.rng(9300, 0)
    n, d, R, W, k, nq = 20000, 32, 24, 48, 10, 200
    scale = (1.0 / np.sqrt(np.arange(1, d + 1))).astype(np.float32)
    X = g.standard_normal((n, d)).astype(np.float32) * scale
    Q = g.standard_normal((nq, d)).astype(np.float32) * scale
    entry = int(np.argmin(((X - X.mean(0)) ** 2).sum(1)))
    graph = L.graph_build(torch.from_numpy(X).cuda(), R, W, 1.2, 0, entry, passes=2, max_batch=2048)
    mu = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    ix = L.Index(d, 8, 0, L.LVQ_L2, L.LVQ_SEQUENTIAL, capacity=n, means=mu)
    slots = ix.insert(torch.from_numpy(X).cuda()).cpu().numpy()
    assert (slots == np.arange(n)).all()
    ids, _, _ = ix.graph_search(torch.from_numpy(Q).cuda(), graph,
                                torch.tensor([entry], dtype=torch.int32, device="cuda"), 64, k)
    assert ix.sync() == 0
    Xd, Qd = X.astype(np.float64), Q.astype(np.float64)
    d2 = (Qd * Qd).sum(1)[:, None] - 2 * Qd @ Xd.T + (Xd * Xd).sum(1)[None, :]
    truth = np.argsort(d2, axis=1)[:, :k]
    rec = oracle.recall(ids.cpu().numpy(), truth)
    assert rec >= 0.9, rec
    ix.close()


def test_graph_build_rejects_bad_arguments(L):
    X = torch.zeros((100, 8), dtype=torch.float32, device="cuda")
    for degree, window, alpha, entry, passes in ((16, 8, 1.2, 0, 2), (65, 128, 1.2, 0, 2), (8, 300, 1.2, 0, 2),
                                                  (8, 16, 0.0, 0, 2), (8, 16, 1.2, 100, 2), (8, 16, 1.2, 0, 3)):
        with pytest.raises(L.LVQError):
            L.graph_build(X, degree, window, alpha, 0, entry, passes=passes)
    with pytest.raises(L.LVQError):
        L.graph_build(torch.zeros((100, 5000), dtype=torch.float32, device="cuda"), 8, 16, 1.2, 0, 0)


@pytest.mark.parametrize("metric,alpha", [(0, 1.2), (1, 0.95)])
def test_delete_consolidation_matches_oracle(L, metric, alpha):
    # degree 16: the 16 x 16 neighbour table is one group of candidates, so
    # the GPU prunes each affected row in one step as the oracle does
    g = synth.rng(9400, metric)
    n, d, R, W = 3000, 16, 16, 32
    X = g.standard_normal((n, d)).astype(np.float32)
    if metric == oracle.IP:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    entry = int(np.argmin(((X - X.mean(0)) ** 2).sum(1)))
    xd = torch.from_numpy(X).cuda()
    graph = L.graph_build(xd, R, W, alpha, metric, entry, passes=2, max_batch=512)
    before = graph.cpu().numpy()
    deleted = np.zeros(n, bool)
    deleted[g.choice([i for i in range(n) if i != entry], 450, replace=False)] = True
    L.graph_delete(xd, graph, torch.from_numpy(deleted).cuda(), alpha, metric)
    got = graph.cpu().numpy()
    want = oracle.vamana_delete(metric, X, before, deleted, alpha, R)
    assert (got[deleted] == -1).all()
    kept = np.flatnonzero(~deleted)
    _rows_ok(got, n, kept)
    for i in kept:
        assert not deleted[got[i][got[i] >= 0]].any()
    same = sum(set(got[i][got[i] >= 0].tolist()) == set(want[i][want[i] >= 0].tolist()) for i in kept)
    assert same >= len(kept) - 5, "%d of %d rows equal the oracle's consolidation" % (same, len(kept))
    # rows without deleted out-neighbours are untouched
    clean = [i for i in kept if not deleted[before[i][before[i] >= 0]].any()]
    np.testing.assert_array_equal(got[clean], before[clean])


def test_insert_listed_nodes_matches_oracle(L):
    # one node at a time: the paper's sequential insert of scattered nodes
    g = synth.rng(9500, 0)
    n, d, R, W = 800, 8, 10, 24
    X = g.standard_normal((n, d)).astype(np.float32)
    xd = torch.from_numpy(X).cuda()
    new = np.sort(g.choice(np.arange(1, n), 120, replace=False)).astype(np.int32)
    old = np.setdiff1d(np.arange(n), new)
    entry = int(old[np.argmin(((X[old] - X[old].mean(0)) ** 2).sum(1))])
    base = np.full((n, R), -1, np.int32)
    oracle.vamana_insert(0, X, base, [entry] + [int(v) for v in old if v != entry], entry, W, 1.2, R)
    graph = torch.from_numpy(base.copy()).cuda()
    order = g.permutation(new).astype(np.int32)
    L.graph_insert(xd, graph, order, W, 1.2, 0, entry, max_batch=1)
    got = graph.cpu().numpy()
    want = base.copy()
    oracle.vamana_insert(0, X, want, order, entry, W, 1.2, R)
    _rows_ok(got, n)
    same = sum(set(got[i][got[i] >= 0].tolist()) == set(want[i][want[i] >= 0].tolist()) for i in range(n))
    assert same >= int(0.98 * n), "%d of %d rows equal the oracle's inserts" % (same, n)
    with pytest.raises(L.LVQError):   # the entry cannot be inserted
        L.graph_insert(xd, graph, [entry], W, 1.2, 0, entry)
    with pytest.raises(L.LVQError):   # repeated node
        L.graph_insert(xd, graph, [new[0], new[0]], W, 1.2, 0, entry)

"""Graph construction on the GPU (lvq_graph_prune, lvq_graph_build,
lvq_graph_insert, lvq_graph_delete of the C ABI) against the oracle's Alg. 2
and App. A routines.

* Pruning over real-valued vectors: the oracle's robust_prune records the
  margin of each decision (the ranking of the candidates, every test of the
  rule) against the binary32 error bound of the similarities compared; every
  row whose decisions all clear their bounds must equal the oracle's exactly.
  Long candidate lists are pruned in groups (whole blocks of 256 positions,
  as many as fit beside the kept out-neighbours), as the oracle is folded.
* Construction, inserts and delete consolidation over small-integer vectors,
  whose similarities binary32 computes exactly: every row must equal the
  oracle's (as a set) -- the sequential routine with batches of one, and the
  batched routine (a batch searches the graph as it was before the batch,
  reverse edges merged per target) with larger batches.  Exact ties abound
  in such data, so the tie rules (lower node first) are held too.
* A batched build over real-valued vectors gives valid, searchable graphs
  with high recall.
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


def _sim_tol(metric, X):
    """A realistic bound on the binary32 rounding error of a similarity of
    two of the vectors: 4 sqrt(d) unit roundoffs (2^-24) of the magnitude
    summed (the squared distance for L2, sum_j |a_j b_j| for IP).  Rounding
    errors of d terms grow like sqrt(d) in practice."""
    eps = 2.0 ** -24
    d = X.shape[1]
    Xd = X.astype(np.float64)

    def tol(a, b, s):
        if metric == oracle.L2:
            return 4.0 * np.sqrt(d) * eps * abs(s)
        return 4.0 * np.sqrt(d) * eps * float(np.abs(Xd[a] * Xd[b]).sum())

    return tol


def _int_vectors(g, n, d):
    """Small-integer vectors: every similarity of two of them is an integer
    below 2^24, exact in binary32 as in binary64."""
    return g.integers(-6, 7, (n, d)).astype(np.float32)


def _row_sets(graph):
    return [set(int(v) for v in r if v >= 0) for r in graph]


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
    tol = _sim_tol(metric, X)
    decisive = 0
    for i, p in enumerate(nodes):
        c = cand[offs[i]:offs[i + 1]]
        cur = [int(v) for v in before[p] if 0 <= v < n and v != p]   # repeats included, as the kernel reads the row
        pos = 0
        margins = []
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
            cur = oracle.robust_prune(metric, X, int(p), group, cur, alpha, R, tol=tol, margins=margins)
            if pos >= len(c):
                break
        row = got[p][got[p] >= 0].tolist()
        if min(margins, default=1.0) > 0:
            decisive += 1
            assert row == cur, "row of node %d (decisions clear of their bounds) differs from the oracle's" % p
    assert decisive >= m // 2, "only %d of %d prunings clear every bound" % (decisive, m)
    untouched = np.setdiff1d(np.arange(n), nodes)
    np.testing.assert_array_equal(got[untouched], before[untouched])
    _rows_ok(got, n, nodes)


@pytest.mark.parametrize("metric,alpha", [(0, 1.25), (1, 0.875)])
def test_sequential_build_matches_oracle(L, metric, alpha):
    # batches of one: the paper's sequential routine
    g = synth.rng(9100, metric)
    n, d, R, W = 500, 8, 10, 24
    X = _int_vectors(g, n, d)
    entry = int(np.argmin(((X - X.mean(0)) ** 2).sum(1)))
    got = L.graph_build(torch.from_numpy(X).cuda(), R, W, alpha, metric, entry, passes=2, max_batch=1).cpu().numpy()
    want = oracle.vamana_build(metric, X, entry, W, alpha, R)
    _rows_ok(got, n)
    bad = [i for i, (a, b) in enumerate(zip(_row_sets(got), _row_sets(want))) if a != b]
    assert not bad, "%d rows differ from the oracle's sequential build, e.g. %s" % (len(bad), bad[:5])


@pytest.mark.parametrize("metric,alpha,max_batch", [(0, 1.25, 7), (0, 1.25, 64), (1, 0.875, 32)])
def test_batched_build_matches_oracle(L, metric, alpha, max_batch):
    # the batched reading of the construction: batches of up to max_batch
    # nodes (in the first pass at most the graph's size) search the graph as
    # it was before the batch; reverse edges are merged per target
    g = synth.rng(9150, metric * 100 + max_batch)
    n, d, R, W = 600, 8, 10, 24
    X = _int_vectors(g, n, d)
    entry = int(np.argmin(((X - X.mean(0)) ** 2).sum(1)))
    xd = torch.from_numpy(X).cuda()
    got = L.graph_build(xd, R, W, alpha, metric, entry, passes=2, max_batch=max_batch).cpu().numpy()
    want = np.full((n, R), -1, np.int32)
    order = [entry] + [i for i in range(n) if i != entry]
    oracle.vamana_update(metric, X, want, order, 0, entry, W, alpha, R, 2, max_batch)
    _rows_ok(got, n)
    bad = [i for i, (a, b) in enumerate(zip(_row_sets(got), _row_sets(want))) if a != b]
    assert not bad, "%d rows differ from the oracle's batched build, e.g. %s" % (len(bad), bad[:5])
    # inserts: one pass over 150 new nodes in batches into the graph of the others
    m = 150
    base = np.full((n + m, R), -1, np.int32)
    base[:n] = want
    Xa = np.concatenate([X, _int_vectors(g, m, d)])
    ga = torch.from_numpy(base.copy()).cuda()
    L.graph_build(torch.from_numpy(Xa).cuda(), R, W, alpha, metric, entry, passes=1, first=n, max_batch=max_batch,
                  graph=ga)
    want_a = oracle.vamana_update(metric, Xa, base.copy(), list(range(n, n + m)), n, entry, W, alpha, R, 1, max_batch)
    got_a = ga.cpu().numpy()
    bad = [i for i, (a, b) in enumerate(zip(_row_sets(got_a), _row_sets(want_a))) if a != b]
    assert not bad, "%d rows differ after batched inserts, e.g. %s" % (len(bad), bad[:5])


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


@pytest.mark.parametrize("metric,alpha", [(0, 1.25), (1, 0.875)])
def test_delete_consolidation_matches_oracle(L, metric, alpha):
    # degree 16: the 16 x 16 neighbour table is one group of candidates, so
    # the GPU prunes each affected row in one step as the oracle does
    g = synth.rng(9400, metric)
    n, d, R, W = 3000, 16, 16, 32
    X = _int_vectors(g, n, d)
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
    bad = [int(i) for i in kept if set(got[i][got[i] >= 0].tolist()) != set(want[i][want[i] >= 0].tolist())]
    assert not bad, "%d rows differ from the oracle's consolidation, e.g. %s" % (len(bad), bad[:5])
    # rows without deleted out-neighbours are untouched
    clean = [i for i in kept if not deleted[before[i][before[i] >= 0]].any()]
    np.testing.assert_array_equal(got[clean], before[clean])


def test_insert_listed_nodes_matches_oracle(L):
    # one node at a time: the paper's sequential insert of scattered nodes
    g = synth.rng(9500, 0)
    n, d, R, W = 800, 8, 10, 24
    X = _int_vectors(g, n, d)
    xd = torch.from_numpy(X).cuda()
    new = np.sort(g.choice(np.arange(1, n), 120, replace=False)).astype(np.int32)
    old = np.setdiff1d(np.arange(n), new)
    entry = int(old[np.argmin(((X[old] - X[old].mean(0)) ** 2).sum(1))])
    base = np.full((n, R), -1, np.int32)
    oracle.vamana_insert(0, X, base, [entry] + [int(v) for v in old if v != entry], entry, W, 1.25, R)
    graph = torch.from_numpy(base.copy()).cuda()
    order = g.permutation(new).astype(np.int32)
    L.graph_insert(xd, graph, order, W, 1.25, 0, entry, max_batch=1)
    got = graph.cpu().numpy()
    want = base.copy()
    oracle.vamana_insert(0, X, want, order, entry, W, 1.25, R)
    _rows_ok(got, n)
    bad = [i for i in range(n) if set(got[i][got[i] >= 0].tolist()) != set(want[i][want[i] >= 0].tolist())]
    assert not bad, "%d rows differ from the oracle's inserts, e.g. %s" % (len(bad), bad[:5])
    # listed inserts in batches of 16: the batched routine over the same order
    graph = torch.from_numpy(base.copy()).cuda()
    L.graph_insert(xd, graph, order, W, 1.25, 0, entry, max_batch=16)
    want = oracle.vamana_update(0, X, base.copy(), order, n - len(order), entry, W, 1.25, R, 1, 16)
    got = graph.cpu().numpy()
    bad = [i for i in range(n) if set(got[i][got[i] >= 0].tolist()) != set(want[i][want[i] >= 0].tolist())]
    assert not bad, "%d rows differ from the oracle's batched inserts, e.g. %s" % (len(bad), bad[:5])
    with pytest.raises(L.LVQError):   # the entry cannot be inserted
        L.graph_insert(xd, graph, [entry], W, 1.25, 0, entry)
    with pytest.raises(L.LVQError):   # repeated node
        L.graph_insert(xd, graph, [new[0], new[0]], W, 1.25, 0, entry)

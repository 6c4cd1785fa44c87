"""Pins of the oracle's neighbourhood pruning (Alg. 2), its float-vector walk
and the graph construction routine of App. A (initial build, inserts)."""
import numpy as np

import oracle
import synth


def _line(pos):
    return np.asarray(pos, np.float32)[:, None]


def test_prune_on_a_line_keeps_the_nearest_on_each_side():
    # p at 0; candidates at 1, 2, 3, -1, -2 (slots 1..5).  alpha = 1, L2:
    # order 1, -1, 2, -2, 3 (ties to the lower slot).  x* = 1 removes 2
    # (|1-2|^2 = 1 <= 4) and 3 (4 <= 9) but not -1 (4 > 1) or -2 (9 > 4);
    # x* = -1 removes -2 (1 <= 4).  Result [1, -1].
    X = _line([0, 1, 2, 3, -1, -2])
    assert oracle.robust_prune(oracle.L2, X, 0, [1, 2, 3, 4, 5], [], 1.0, 8) == [1, 4]
    # alpha = 4.5: x* = 1 removes x' when 4.5 |1-x'|^2 <= |x'|^2: 2 (4.5 > 4)
    # and 3 (18 > 9) survive; -1: 18 > 1.  x* = -1: -2 survives (4.5 > 4).
    # x* = 2 removes 3 (4.5 <= 9) but not -2 (72 > 4).  Then -2: [1, -1, 2, -2].
    assert oracle.robust_prune(oracle.L2, X, 0, [1, 2, 3, 4, 5], [], 4.5, 8) == [1, 4, 2, 5]
    # the degree bound stops the selection
    assert oracle.robust_prune(oracle.L2, X, 0, [1, 2, 3, 4, 5], [], 4.5, 2) == [1, 4]


def test_prune_merges_current_neighbours_and_drops_p_and_duplicates():
    X = _line([0, 1, 2, 3, -1, -2])
    got = oracle.robust_prune(oracle.L2, X, 0, [0, 2, 2, -1, 5], [1, 4, 1], 1.0, 8)
    assert got == [1, 4]


def test_prune_inner_product_by_hand():
    # p = e1; candidates at angles 10, -15, 20, 90 degrees (slots 1..4) on the
    # unit circle.  Order: 10 (cos 10 = .985), -15 (.966), 20 (.940), 90 (0).
    # alpha = .95.  x* = 10 deg: 20 stays (.95 cos 10 = .936 < .940), -15
    # stays (.95 cos 25 = .861 < .966), 90 goes (.95 cos 80 = .165 >= 0).
    # x* = -15: 20 stays (.95 cos 35 = .778 < .940).  Then 20.
    ang = np.radians([0.0, 10.0, -15.0, 20.0, 90.0])
    X = np.stack([np.cos(ang), np.sin(ang)], 1).astype(np.float32)
    assert oracle.robust_prune(oracle.IP, X, 0, [1, 2, 3, 4], [], 0.95, 8) == [1, 2, 3]
    # alpha = 1.1 (> 1: the more similar x* prunes more): x* = 10 removes -15?
    # 1.1 cos 25 = .997 >= .966 yes; 20: 1.1 cos 10 = 1.083 >= .940 yes; 90:
    # 1.1 cos 80 = .191 >= 0 yes.  Result [1].
    assert oracle.robust_prune(oracle.IP, X, 0, [1, 2, 3, 4], [], 1.1, 8) == [1]


def test_prune_with_no_pruning_is_the_nearest_r():
    # alpha so large (L2) that no candidate is ever removed: the R nearest by
    # brute force, ties to the lower slot
    g = synth.rng(8900, 0)
    X = g.standard_normal((200, 16)).astype(np.float32)
    cand = g.choice(np.arange(1, 200), 80, replace=False)
    got = oracle.robust_prune(oracle.L2, X, 0, cand, [], 1e30, 12)
    d = ((X[cand].astype(np.float64) - X[0].astype(np.float64)) ** 2).sum(1)
    want = [int(cand[i]) for i in np.lexsort((cand, d))[:12]]
    assert got == want


def test_float_walk_on_a_complete_graph_is_exhaustive():
    g = synth.rng(8901, 0)
    X = g.standard_normal((120, 8)).astype(np.float32)
    q = g.standard_normal(8).astype(np.float32)
    graph = np.array([[j for j in range(120) if j != i] for i in range(120)], np.int32)
    for metric in (oracle.L2, oracle.IP):
        s, v, ne = oracle.greedy_search_float(metric, q, X, graph, [3], 120, 10)
        sims = np.array([oracle.float_sim(metric, q, x) for x in X])
        key = sims if metric == oracle.L2 else -sims
        assert s.tolist() == np.lexsort((np.arange(120), key))[:10].tolist()
        assert ne == 120


def test_build_on_a_line_is_the_path():
    # alpha = 1 and R = 2 on distinct points of a line: every node ends with
    # its two neighbours on the line (one at the ends), the relative
    # neighbourhood graph of the points
    g = synth.rng(8902, 0)
    n = 30
    pos = g.permutation(n)
    X = _line(pos)
    graph = oracle.vamana_build(oracle.L2, X, int(np.argmin(np.abs(pos - n // 2))), 6, 1.0, 2,
                                order=g.permutation(n))
    slot_of = {int(p): i for i, p in enumerate(pos)}
    for i, p in enumerate(pos):
        want = {slot_of[q] for q in (p - 1, p + 1) if 0 <= q < n}
        assert set(int(v) for v in graph[i] if v >= 0) == want, (i, p)


def test_build_properties_and_navigability():
    g = synth.rng(8903, 0)
    n, R = 300, 8
    X = g.standard_normal((n, 2)).astype(np.float32)
    entry = int(np.argmin(((X - X.mean(0)) ** 2).sum(1)))
    graph = oracle.vamana_build(oracle.L2, X, entry, 16, 1.2, R)
    for i in range(n):
        row = [int(v) for v in graph[i] if v >= 0]
        assert 1 <= len(row) <= R and i not in row and len(set(row)) == len(row)
        # the -1 padding is at the end
        assert (graph[i, len(row):] == -1).all()
    # every stored point, as a query, is found by the walk from the entry
    hit = sum(int(oracle.greedy_search_float(oracle.L2, X[i], X, graph, [entry], 16, 1)[0][0] == i)
              for i in range(n))
    assert hit == n


def test_insert_adds_reachable_nodes():
    # the update routine on new nodes (App. A, insertions): after inserting
    # 50 more points into a graph of 250 every new point is found by a walk
    g = synth.rng(8904, 0)
    X = g.standard_normal((300, 3)).astype(np.float32)
    entry = 0
    graph = np.full((300, 10), -1, np.int32)
    oracle.vamana_insert(oracle.L2, X, graph, range(250), entry, 20, 1.2, 10)
    assert (graph[250:] == -1).all()
    oracle.vamana_insert(oracle.L2, X, graph, range(250, 300), entry, 20, 1.2, 10)
    for i in range(250, 300):
        assert oracle.greedy_search_float(oracle.L2, X[i], X, graph, [entry], 20, 1)[0][0] == i


def test_delete_consolidation_by_hand():
    # points on a line 0..5 (slot = position), path graph; delete 2 and 3.
    # Node 1 had {0, 2}: 2 is deleted, its kept neighbour is 1 itself (dropped)
    # and 3 is deleted too, so node 1 keeps {0} -- only one hop is bridged.
    # Node 4 had {3, 5}: 3's kept neighbours are none (2 deleted, 4 itself),
    # so 4 keeps {5}.  With R = 1, node 1's candidates {0} fit; nothing pruned.
    X = _line([0, 1, 2, 3, 4, 5])
    g = np.full((6, 2), -1, np.int32)
    for i in range(6):
        nb = [j for j in (i - 1, i + 1) if 0 <= j < 6]
        g[i, :len(nb)] = nb
    deleted = np.zeros(6, bool)
    deleted[[2, 3]] = True
    out = oracle.vamana_delete(oracle.L2, X, g, deleted, 1.2, 2)
    assert [set(int(v) for v in out[i] if v >= 0) for i in range(6)] == [{1}, {0}, set(), set(), {5}, {4}]
    # delete only 2: node 1 bridges to 3, node 3 bridges to 1
    deleted[3] = False
    out = oracle.vamana_delete(oracle.L2, X, g, deleted, 1.2, 2)
    assert set(int(v) for v in out[1] if v >= 0) == {0, 3}
    assert set(int(v) for v in out[3] if v >= 0) == {1, 4}
    # R = 1 forces a prune: node 1's candidates {0, 3} -> the nearer, 0
    g1 = g.copy()
    out = oracle.vamana_delete(oracle.L2, X, g1, deleted, 1.2, 1)
    assert set(int(v) for v in out[1] if v >= 0) == {0}


def test_delete_consolidation_keeps_search_working():
    g = synth.rng(8905, 0)
    n, R = 400, 10
    X = g.standard_normal((n, 2)).astype(np.float32)
    entry = int(np.argmin(((X - X.mean(0)) ** 2).sum(1)))
    graph = oracle.vamana_build(oracle.L2, X, entry, 20, 1.2, R)
    deleted = np.zeros(n, bool)
    deleted[g.choice([i for i in range(n) if i != entry], 80, replace=False)] = True
    out = oracle.vamana_delete(oracle.L2, X, graph, deleted, 1.2, R)
    assert (out[deleted] == -1).all()
    for i in np.flatnonzero(~deleted):
        row = [int(v) for v in out[i] if v >= 0]
        assert len(row) <= R and not deleted[row].any() and i not in row
    hit = sum(int(oracle.greedy_search_float(oracle.L2, X[i], X, out, [entry], 20, 1)[0][0] == i)
              for i in np.flatnonzero(~deleted))
    assert hit >= int(0.98 * (~deleted).sum())

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


def test_batched_update_with_batches_of_one_is_the_sequential_routine():
    # the batched reading of App. A's construction: with max_batch = 1 every
    # batch is one node, which searches the graph left by the node before it
    g = synth.rng(8906, 0)
    n, R, W = 150, 6, 12
    X = g.standard_normal((n, 3)).astype(np.float32)
    entry = int(np.argmin(((X - X.mean(0)) ** 2).sum(1)))
    want = oracle.vamana_build(oracle.L2, X, entry, W, 1.2, R)
    got = np.full((n, R), -1, np.int32)
    order = [entry] + [i for i in range(n) if i != entry]
    oracle.vamana_update(oracle.L2, X, got, order, 0, entry, W, 1.2, R, 2, 1)
    np.testing.assert_array_equal(got, want)
    # inserts: one pass over new nodes into a graph of the others
    base = np.full((n, R), -1, np.int32)
    oracle.vamana_insert(oracle.L2, X, base, order[:120], entry, W, 1.2, R)
    want = base.copy()
    oracle.vamana_insert(oracle.L2, X, want, order[120:], entry, W, 1.2, R)
    got = base.copy()
    oracle.vamana_update(oracle.L2, X, got, order[120:], 120, entry, W, 1.2, R, 1, 1)
    np.testing.assert_array_equal(got, want)


def test_batched_update_by_hand():
    # points on a line: node 0 at 0 (entry), 1 at 10, 2 at 4, 3 at 6; the
    # graph of {0, 1} with R = 1 is 0 -> 1, 1 -> 0.  Nodes 2 and 3 inserted in
    # one batch (in_graph = 2 allows a batch of 2) both search the pre-batch
    # graph: 2 finds (0, 1) and keeps 0; 3 finds (1, 0) and keeps 1.  Reverse
    # edges: node 0 takes source 2, its row {1, 2} exceeds R and is pruned to
    # the nearer, 2; node 1 likewise ends at 3.  Inserted one at a time, 3
    # would search the graph already holding 2, never reach 1, and link to 2.
    X = _line([0, 10, 4, 6])
    graph = np.array([[1], [0], [-1], [-1]], np.int32)
    batched = oracle.vamana_update(oracle.L2, X, graph.copy(), [2, 3], 2, 0, 2, 1.2, 1, 1, 2)
    assert batched[:, 0].tolist() == [2, 3, 0, 1]
    seq = oracle.vamana_update(oracle.L2, X, graph.copy(), [2, 3], 2, 0, 2, 1.2, 1, 1, 1)
    assert seq[:, 0].tolist() == [2, 0, 3, 2]


def test_batch_members_do_not_link_to_each_other_in_one_pass():
    g = synth.rng(8907, 0)
    n, R, W = 200, 8, 16
    X = g.standard_normal((n, 4)).astype(np.float32)
    graph = oracle.vamana_build(oracle.L2, X[:150], 0, W, 1.2, R)
    full = np.full((n, R), -1, np.int32)
    full[:150] = graph
    oracle.vamana_update(oracle.L2, X, full, list(range(150, 200)), 150, 0, W, 1.2, R, 1, 50)
    new = set(range(150, 200))
    for i in range(150, 200):
        row = [int(v) for v in full[i] if v >= 0]
        assert row and not (set(row) & new) and len(row) <= R
    for i in range(n):
        row = [int(v) for v in full[i] if v >= 0]
        assert len(row) == len(set(row)) and i not in row and len(row) <= R


def test_decision_margins_by_hand():
    # pruning 0 over candidates at 1 and 2 on a line (alpha 1): the ranking
    # gap |1 - 4| = 3, and the rule test of 2 against x* = 1: |1 * 1 - 4| = 3;
    # error bounds subtract from each margin
    X = _line([0, 1, 2])
    m = []
    assert oracle.robust_prune(oracle.L2, X, 0, [1, 2], [], 1.0, 8, tol=lambda a, b, s: 0.0, margins=m) == [1]
    assert m == [3.0, 3.0]
    m = []
    oracle.robust_prune(oracle.L2, X, 0, [1, 2], [], 1.0, 8, tol=lambda a, b, s: 0.25 * s, margins=m)
    assert m == [3.0 - 1.25, 3.0 - 1.25]
    # the walk on a line (d = 1 rows decode exactly): margins are the score
    # gaps of its decisions, minus the bounds
    Xl = _line([0, 1, 2, 3, 4])
    graph = np.array([[1, -1], [0, 2], [1, 3], [2, 4], [3, -1]], np.int32)
    scores = lambda q: (lambda slots: np.array([(q - float(Xl[s, 0])) ** 2 for s in slots]))
    m = []
    out, _, _ = oracle._walk(scores(3.4), oracle.L2, graph, [0], 2, 1, tol=lambda s: 0.0, margins=m)
    assert out.tolist() == [3] and min(m) > 0
    m = []
    oracle._walk(scores(3.5), oracle.L2, graph, [0], 2, 1, tol=lambda s: 0.0, margins=m)
    assert min(m) == 0.0      # 3 and 4 tie at 0.25: the walk has a decision at zero margin


def test_first_pass_batches_never_outgrow_the_graph():
    # line 0..3, entry 0, R = 2, W = 2, one pass, max_batch = 4.  Batches are
    # [0], [1], [2, 3]: 0 finds only itself (empty row); 1 links to 0, which
    # takes 1 back; 2 and 3 both find (1, 0) in the graph {0, 1} and keep 1
    # (x* = 1 removes 0: 1.2 * 1 <= 4 and <= 9); node 1 then takes sources 2
    # and 3 beside 0, three > R, pruned: order 0, 2 (both at 1), 3; x* = 0
    # keeps 2 (1.2 * 4 > 1) and 3 (1.2 * 9 > 4); x* = 2 fills R: {0, 2}.
    # All four in one batch would search an empty graph and all link to 0.
    X = _line([0, 1, 2, 3])
    g = np.full((4, 2), -1, np.int32)
    oracle.vamana_update(oracle.L2, X, g, [0, 1, 2, 3], 0, 0, 2, 1.2, 2, 1, 4)
    assert [[int(v) for v in r if v >= 0] for r in g] == [[1], [0, 2], [1], [1]]

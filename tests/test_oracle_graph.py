"""Pins of the oracle's greedy graph search (Alg. 1): exploration order, the
cut of the candidate set to W, ties, lazy deletes, and the exhaustive result
on a complete graph."""
import numpy as np

import oracle
import synth


def _line(positions):
    """One-dimensional rows: with d = 1 every vector has u == l, so Delta = 0,
    the codes are 0 and the reconstruction mu + l is the value itself: the L2
    similarity is exactly (q - x)^2 and the walk can be followed by hand."""
    X = np.asarray(positions, np.float32)[:, None]
    mu = np.zeros((1, 1), np.float32)
    fmt = oracle.Format(1, 8, 0, oracle.SEQUENTIAL)
    rows, _, _ = oracle.encode_rows(fmt, X, mu)
    return fmt, rows, mu


def _chain(n):
    g = np.full((n, 2), -1, np.int32)
    for i in range(n):
        if i > 0:
            g[i, 0] = i - 1
        if i + 1 < n:
            g[i, 1] = i + 1
    return g


def _search(fmt, rows, mu, graph, q, W, k, entries=(0,), live=None):
    return oracle.greedy_search(fmt, oracle.L2, oracle.PRIMARY, np.float32([q]), rows, None, mu, graph,
                                list(entries), W, k, live)


def test_greedy_descent_on_a_line():
    fmt, rows, mu = _line(np.arange(10))
    s, v, ne = _search(fmt, rows, mu, _chain(10), 7.3, W=1, k=1)
    # 0 -> 1 -> ... -> 7; node 8 (0.49) is worse than 7 (0.09): stop at 7
    assert s.tolist() == [7] and ne == 8
    np.testing.assert_allclose(v, [(float(np.float32(7.3)) - 7.0) ** 2], rtol=1e-12)   # the binary32 query


def test_window_lets_the_search_climb_out_of_a_local_minimum():
    # positions along the chain 0-1-2-3-4; query 11
    fmt, rows, mu = _line([0, 5, 3, 10, 12])
    # W = 1: 0 (121) -> 1 (36); its other neighbour 2 (64) is cut: stuck at 1
    s, _, ne = _search(fmt, rows, mu, _chain(5), 11.0, W=1, k=1)
    assert s.tolist() == [1] and ne == 2
    # W = 2: 2 survives the cut, is explored and leads to 3 and 4 (both at
    # distance 1: the tie goes to the lower slot)
    s, v, ne = _search(fmt, rows, mu, _chain(5), 11.0, W=2, k=2)
    assert s.tolist() == [3, 4] and v.tolist() == [1.0, 1.0] and ne == 5


def test_deleted_nodes_are_traversed_not_returned():
    fmt, rows, mu = _line(np.arange(10))
    live = np.ones(10, bool)
    live[[4, 9]] = False
    # the only way from 0 to 9 passes through the deleted node 4
    s, _, _ = _search(fmt, rows, mu, _chain(10), 9.2, W=3, k=3, live=live)
    assert s.tolist() == [8, 7]        # 9 is deleted; the window holds 9, 8, 7
    s, _, _ = _search(fmt, rows, mu, _chain(10), 9.2, W=4, k=3, live=live)
    assert s.tolist() == [8, 7, 6]


def test_complete_graph_and_full_window_is_exhaustive():
    g = synth.rng(8500, 0)
    d, n = 32, 300
    X = g.standard_normal((n, d)).astype(np.float32)
    mu = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    Q = g.standard_normal((5, d)).astype(np.float32)
    for metric, layout, b1 in ((oracle.L2, oracle.SEQUENTIAL, 8), (oracle.IP, oracle.TURBO, 4)):
        fmt = oracle.Format(d, b1, 0, layout)
        rows, _, _ = oracle.encode_rows(fmt, X, mu)
        graph = np.array([[j for j in range(n) if j != i] for i in range(n)], np.int32)
        es, ev = oracle.topk_exhaustive(fmt, metric, oracle.PRIMARY, Q, rows, None, mu, 10)
        for i in range(Q.shape[0]):
            s, v, ne = oracle.greedy_search(fmt, metric, oracle.PRIMARY, Q[i], rows, None, mu, graph, [7], n, 10)
            assert ne == n
            np.testing.assert_array_equal(s, es[i])
            np.testing.assert_array_equal(v, ev[i])


def test_the_closest_unexplored_node_is_explored_first():
    # positions 0, 5, -5, 9 (slots 0..3); edges 0 -> {1, 2}, 1 -> {3}; query 10,
    # W = 3.  Exploring 0 adds 1 (25) and 2 (225); the closest unexplored, 1,
    # adds 3 (1), and the cut to W = 3 drops 2 before it is ever explored:
    # explored {0, 1, 3}.  (Taking 2 first would explore four nodes.)
    fmt, rows, mu = _line([0, 5, -5, 9])
    graph = np.array([[1, 2], [3, -1], [-1, -1], [-1, -1]], np.int32)
    s, v, ne = _search(fmt, rows, mu, graph, 10.0, W=3, k=3)
    assert ne == 3
    assert s.tolist() == [3, 1, 0] and v.tolist() == [1.0, 25.0, 100.0]

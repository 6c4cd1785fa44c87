"""Pins of the oracle's soft-inverted-index routing (M-LVQ as an inverted
index, the Sec. 3.2 remark that a query touches few centres): the probed
means are the nprobe nearest by the Def. 1 distance, nearest first, ties to
the lower index, and the candidate lists are exactly the rows assigned to
them."""
import numpy as np

import oracle
import synth


def test_worked_example_by_hand():
    # four means on the unit square, one query: distances by hand
    means = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], np.float32)
    q = np.array([0.5, 0.25], np.float32)
    # |q - mu|^2: 0.3125, 0.3125, 0.8125, 0.8125 -> ties broken by index
    np.testing.assert_array_equal(oracle.mean_dists(q, means), np.float32([0.3125, 0.3125, 0.8125, 0.8125]))
    np.testing.assert_array_equal(oracle.probe_means(q, means, 4)[0], [0, 1, 2, 3])
    q = np.array([0.9, 0.2], np.float32)
    # 0.85, 0.05, 1.45, 0.65 -> means 1, 3, 0, 2
    np.testing.assert_array_equal(oracle.probe_means(q, means, 4)[0], [1, 3, 0, 2])
    np.testing.assert_array_equal(oracle.probe_means(q, means, 2)[0], [1, 3])


def test_order_matches_binary64_except_near_ties():
    g = synth.rng(8100, 0)
    M, d = 40, 24
    means = g.standard_normal((M, d)).astype(np.float32)
    Q = g.standard_normal((150, d)).astype(np.float32)
    full = oracle.probe_means(Q, means, M)
    ex = ((Q.astype(np.float64)[:, None, :] - means.astype(np.float64)[None]) ** 2).sum(-1)
    for i in range(Q.shape[0]):
        p = full[i]
        assert sorted(p.tolist()) == list(range(M)), "a permutation of all means"
        v = ex[i, p]
        # consecutive pairs in binary64 order, up to binary32 rounding
        bad = np.flatnonzero(v[1:] < v[:-1] * (1 - 1e-5))
        assert bad.size == 0, (i, bad)
        # the probed set for nprobe = 5 is the binary64 top 5 unless the 5th
        # and 6th are within rounding of each other
        top = oracle.probe_means(Q[i], means, 5)[0]
        np.testing.assert_array_equal(top, p[:5])
        o = np.sort(ex[i])
        if o[5] > o[4] * (1 + 1e-5):
            assert set(top.tolist()) == set(np.argsort(ex[i])[:5].tolist())


def test_first_probe_is_the_assignment_rule():
    g = synth.rng(8101, 0)
    means = g.standard_normal((16, 32)).astype(np.float32)
    Q = g.standard_normal((300, 32)).astype(np.float32)
    first = oracle.probe_means(Q, means, 1)[:, 0]
    np.testing.assert_array_equal(first, [oracle.assign(q, means) for q in Q])


def test_exact_ties_go_to_the_lower_index_and_nan_last():
    g = synth.rng(8102, 0)
    means = g.standard_normal((10, 8)).astype(np.float32)
    means[7] = means[2]
    means[4] = means[2]
    means[9, 3] = np.nan
    q = means[2] + np.float32(0.01)
    p = oracle.probe_means(q, means, 10)[0]
    np.testing.assert_array_equal(p[:3], [2, 4, 7])
    assert p[-1] == 9


def test_lists_are_the_members_of_the_probed_means():
    g = synth.rng(8103, 0)
    row_mean = g.integers(0, 6, 500)
    live = g.random(500) > 0.2
    probe = np.array([[3, 1], [5, 0], [2, 4]], np.int32)
    offs, ids = oracle.probe_lists(probe, row_mean, live)
    for i in range(3):
        want = [s for s in range(500) if live[s] and row_mean[s] in probe[i].tolist()]
        assert ids[offs[i]:offs[i + 1]].tolist() == want


def test_probing_every_mean_equals_the_exhaustive_top_k():
    g = synth.rng(8104, 0)
    d, M, n = 48, 6, 700
    cent = g.standard_normal((M, d)).astype(np.float32)
    X = (cent[g.integers(0, M, n)] + 0.3 * g.standard_normal((n, d))).astype(np.float32)
    Q = (cent[g.integers(0, M, 9)] + 0.3 * g.standard_normal((9, d))).astype(np.float32)
    fmt = oracle.Format(d, 8, 0, oracle.SEQUENTIAL)
    rows, resid, _ = oracle.encode_rows(fmt, X, cent)
    live = g.random(n) > 0.1
    probe = oracle.probe_means(Q, cent, M)
    offs, ids = oracle.probe_lists(probe, rows[:, 12], live)
    dist = oracle.distances(fmt, oracle.L2, oracle.PRIMARY, Q, rows, resid, cent, offs, ids)
    ts, tv = oracle.topk_lists(oracle.L2, dist, offs, ids, 10)
    es, ev = oracle.topk_exhaustive(fmt, oracle.L2, oracle.PRIMARY, Q, rows, resid, cent, 10, live)
    np.testing.assert_array_equal(ts, es)
    np.testing.assert_array_equal(tv, ev)

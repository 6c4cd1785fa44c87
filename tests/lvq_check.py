"""Comparison helpers: GPU results against the oracle, to the tolerances the
tests state.

Distances (binary32 on the GPU vs binary64 in the oracle):
  L2: |g - r| <= 1e-4 * r + 1e-7 * (||q - mu*||^2 + ||x_hat - mu*||^2)
  IP: |g - r| <= 1e-4 * S,  S = sum_j |q_j x_hat_j|
The relative term is the bound the distances are held to; the second term
covers values near zero, where a relative bound is meaningless (an IP between
unrelated unit vectors, or L2 between near-duplicates), scaled by the
magnitudes that enter the binary32 computation.
"""
import numpy as np

import oracle


def pair_tolerance(metric, Q, xhat, mean_rows, q_index):
    """Tolerance per pair; xhat / mean_rows are (pairs, d), q_index (pairs,)."""
    q = np.asarray(Q, np.float64)[q_index]
    if metric == oracle.IP:
        S = np.abs(q * xhat).sum(1)
        return 1e-4 * S
    r = ((q - xhat) ** 2).sum(1)
    scale = ((q - mean_rows) ** 2).sum(1) + ((xhat - mean_rows) ** 2).sum(1)
    return 1e-4 * r + 1e-7 * scale


def rounding_bound(fmt, metric, level, q, rows, resid, means):
    """A realistic bound on the binary32 rounding error of the similarity of
    query q to every row, for deciding whether two oracle scores are too
    close for a binary32 evaluation to be sure to order them alike: 4 sqrt(d)
    unit roundoffs (2^-24) of the magnitudes summed, sum_j (|q_j - mu_j| +
    |x_hat_j - mu_j|)^2 for L2 (the direct form's terms) and
    sum_j |q_j| (|mu_j| + |x_hat_j - mu_j|) for IP (the terms of the
    identity).  Rounding errors of d terms grow like sqrt(d) in practice; the
    worst case, d, is what the acceptance tolerance covers."""
    q = np.asarray(q, np.float64)
    xh = reconstruct_all(fmt, rows, resid, means, level)
    mu = np.asarray(means, np.float64)[oracle.unpack(fmt, rows)[3]]
    xr = np.abs(xh - mu)
    if metric == oracle.IP:
        T = (np.abs(q)[None, :] * (np.abs(mu) + xr)).sum(1)
    else:
        T = ((np.abs(q[None, :] - mu) + xr) ** 2).sum(1)
    return 4.0 * np.sqrt(fmt.dim) * 2.0 ** -24 * T


def reconstruct_all(fmt, rows, resid, means, level):
    return oracle.reconstruct(fmt, rows, resid, means, level)


def pair_reference(fmt, metric, level, Q, rows, resid, means, offsets, ids, chunk=1 << 15):
    """Oracle values and tolerances for every listed pair (the tolerances are
    evaluated in chunks of pairs, so long lists need no pairs x d array)."""
    ref = oracle.distances(fmt, metric, level, Q, rows, resid, means, offsets, ids)
    ids = np.asarray(ids)
    uniq, inv = np.unique(ids, return_inverse=True)
    xh_u = oracle.reconstruct(fmt, rows[uniq], None if resid is None else resid[uniq], means, level)
    mid_u = oracle.unpack(fmt, rows[uniq])[3]
    mrow_u = np.asarray(means, np.float64)[mid_u]
    q_index = np.repeat(np.arange(len(offsets) - 1), np.diff(offsets))
    tol = np.empty(len(ids), np.float64)
    for a in range(0, len(ids), chunk):
        c = slice(a, a + chunk)
        tol[c] = pair_tolerance(metric, Q, xh_u[inv[c]], mrow_u[inv[c]], q_index[c])
    return ref, tol


class ExhaustiveReference:
    """Oracle values and tolerances of a few queries against every row of a
    store (for checking exhaustive top-k lists on a query sample).  The
    reconstructions are computed once per level; each query's values come
    from its own oracle call, run on host threads (the calls release the
    interpreter lock)."""

    def __init__(self, fmt, rows, resid, means):
        self.fmt, self.rows, self.resid = fmt, rows, resid
        self.means = np.asarray(means, np.float32)
        self.mid = oracle.unpack(fmt, rows)[3]
        self._xh = {}

    def xhat(self, level):
        if level not in self._xh:
            self._xh[level] = oracle.reconstruct(self.fmt, self.rows, self.resid, self.means, level)
        return self._xh[level]

    def __call__(self, metric, level, Qs):
        from concurrent.futures import ThreadPoolExecutor
        n = self.rows.shape[0]
        Qs = np.ascontiguousarray(Qs, np.float32)
        ids = np.arange(n, dtype=np.int32)
        offs = np.array([0, n], np.int64)

        def one(i):
            return oracle.distances(self.fmt, metric, level, Qs[i:i + 1], self.rows, self.resid, self.means,
                                    offs, ids)

        with ThreadPoolExecutor(min(16, max(1, Qs.shape[0]))) as ex:
            ref = np.stack(list(ex.map(one, range(Qs.shape[0]))))
        # pair_tolerance's formulas, as products over the whole store
        xh = self.xhat(level)
        q = np.asarray(Qs, np.float64)
        if metric == oracle.IP:
            return ref, 1e-4 * (np.abs(q) @ np.abs(xh).T)
        m = np.asarray(self.means, np.float64)
        qm = ((q[:, None, :] - m[None, :, :]) ** 2).sum(2)[:, self.mid]
        xm = ((xh - m[self.mid]) ** 2).sum(1)
        return ref, 1e-4 * ref + 1e-7 * (qm + xm[None, :])


def check_values(got, ref, tol, what="distances"):
    got = np.asarray(got, np.float64)
    bad = ~(np.abs(got - ref) <= tol)
    bad &= ~(np.isnan(got) & np.isnan(ref))
    if bad.any():
        i = np.flatnonzero(bad)[:5]
        raise AssertionError("%s: %d of %d outside tolerance, e.g. idx %s got %s ref %s tol %s"
                             % (what, bad.sum(), bad.size, i, got[i], ref[i], tol[i]))


def better(metric, a, b):
    return a < b if metric == oracle.L2 else a > b


def check_topk(metric, got_ids, got_dist, cand_ids, cand_ref, cand_tol, k, keep=None):
    """One query: the GPU's k ids against the oracle's scores of the candidates.

    Every id the oracle ranks clearly inside the top k (better than the k-th
    value by more than the tolerance) must be returned; every returned id must
    be a candidate whose oracle value is within tolerance of the k-th value or
    better; returned values must match the oracle within tolerance and be
    sorted.  Ids may be padded with -1 when fewer than k candidates survive."""
    cand_ids = np.asarray(cand_ids)
    m = np.ones(len(cand_ids), bool) if keep is None else np.asarray(keep, bool)
    ids_v, ref_v, tol_v = cand_ids[m], np.asarray(cand_ref)[m], np.asarray(cand_tol)[m]
    # ties and duplicates: rank by oracle value then slot
    key = ref_v if metric == oracle.L2 else -ref_v
    order = np.lexsort((ids_v, key))
    n_valid = min(k, len(ids_v))
    got_ids = np.asarray(got_ids)
    got_dist = np.asarray(got_dist, np.float64)
    assert np.all(got_ids[n_valid:] == -1), "padding"
    if n_valid == 0:
        return
    kth = ref_v[order[n_valid - 1]]
    tol_max = tol_v.max() if len(tol_v) else 0.0
    clearly_in = ids_v[better(metric, ref_v, kth) & (np.abs(ref_v - kth) > 2 * tol_max)]
    gi = got_ids[:n_valid]
    assert set(clearly_in.tolist()) <= set(gi.tolist()), "missing a clear top-k member"
    lookup = {}
    for s, r, t in zip(ids_v, ref_v, tol_v):
        lookup.setdefault(int(s), (r, t))
    for s, dv in zip(gi, got_dist[:n_valid]):
        assert int(s) in lookup, "returned id %d is not a live candidate" % s
        r, t = lookup[int(s)]
        assert abs(dv - r) <= t or (np.isnan(dv) and np.isnan(r)), "value of id %d" % s
        assert not better(metric, kth, r) or abs(r - kth) <= 2 * tol_max, "id %d outside the top k" % s
    gd = got_dist[:n_valid]
    srt = gd if metric == oracle.L2 else -gd
    assert np.all(np.diff(srt[~np.isnan(srt)]) >= 0), "not sorted"

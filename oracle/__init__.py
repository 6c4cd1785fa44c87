"""Plain CPU oracle for LVQ encoding and LVQ similarities (arXiv 2402.02044).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the package smoke
check and by the benchmark's CPU-baseline leg, never by the library.  It shares
no code with the HIP library.

The arithmetic lives in ``lvq_oracle.c`` (plain scalar C, binary32 encoder with
one rounding per operation, binary64 similarities); this module is ctypes and
numpy marshalling around it, plus the list/top-k bookkeeping of Sec. 2.1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lvq_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblvqoracle.so")

L2, IP = 0, 1
SEQUENTIAL, TURBO = 0, 1
PRIMARY, FULL = 1, 2
HEADER_BYTES = 32


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < max(os.path.getmtime(_SRC),
                                              os.path.getmtime(os.path.join(_HERE, "lvq_oracle.h"))):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Fmt(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("dim", "bits1", "bits2", "layout", "align", "npos", "code_bytes",
                 "row_bytes", "resid_bytes")]


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.orc_format_init.argtypes = [ctypes.POINTER(_Fmt), i32, i32, i32, i32, i32]
        lib.orc_pos_to_dim.argtypes = [ctypes.POINTER(_Fmt), i32]
        lib.orc_assign.argtypes = [P, i32, P, i32]
        lib.orc_mean_dists.argtypes = [P, i32, P, i32, P]
        lib.orc_mean_dists.restype = None
        lib.orc_probe.argtypes = [P, i32, P, i32, i32, P]
        lib.orc_encode_codes.argtypes = [P, i32, P, i32, i32, P, P, P, P, P]
        lib.orc_encode_rows.argtypes = [ctypes.POINTER(_Fmt), P, i64, P, i32, P, P]
        lib.orc_encode_rows.restype = i64
        lib.orc_unpack.argtypes = [ctypes.POINTER(_Fmt), P, P, P, P, P, P, P, P]
        lib.orc_reconstruct.argtypes = [ctypes.POINTER(_Fmt), P, P, P, i32, P]
        lib.orc_unpack_rows.argtypes = [ctypes.POINTER(_Fmt), P, P, i64, P, P, P, P, P, P]
        lib.orc_unpack_rows.restype = None
        lib.orc_reconstruct_rows.argtypes = [ctypes.POINTER(_Fmt), P, P, i64, P, i32, P]
        lib.orc_reconstruct_rows.restype = None
        lib.orc_distances.argtypes = [ctypes.POINTER(_Fmt), i32, i32, P, i64, P, P, P, P, P, P]
        lib.orc_select_topk.argtypes = [i32, P, P, P, i64, i32, P, P]
        lib.orc_eps1.argtypes = [ctypes.POINTER(_Fmt), P, i64, P, P]
        lib.orc_eps1.restype = ctypes.c_double
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass(frozen=True)
class Format:
    """Row format: see ``lvq_oracle.h``."""
    dim: int
    bits1: int
    bits2: int = 0
    layout: int = SEQUENTIAL
    align: int = 32

    def _c(self) -> _Fmt:
        f = _Fmt()
        rc = _L().orc_format_init(ctypes.byref(f), self.dim, self.bits1, self.bits2,
                                  self.layout, self.align)
        if rc != 0:
            raise ValueError("unsupported LVQ format %r" % (self,))
        return f

    @property
    def npos(self) -> int:
        return self._c().npos

    @property
    def code_bytes(self) -> int:
        return self._c().code_bytes

    @property
    def row_bytes(self) -> int:
        return self._c().row_bytes

    @property
    def resid_bytes(self) -> int:
        return self._c().resid_bytes


def pos_to_dim(fmt: Format) -> np.ndarray:
    f = fmt._c()
    return np.array([_L().orc_pos_to_dim(ctypes.byref(f), p) for p in range(f.npos)], np.int32)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def assign(x, means) -> int:
    x, means = _f32(x), _f32(means)
    return _L().orc_assign(_p(x), x.shape[-1], _p(means), means.shape[0])


def mean_dists(x, means) -> np.ndarray:
    """Def. 1 distances of one vector to every mean (binary32, dimension order)."""
    x, means = _f32(x), _f32(means)
    out = np.zeros(means.shape[0], np.float32)
    _L().orc_mean_dists(_p(x), x.shape[-1], _p(means), means.shape[0], _p(out))
    return out


def probe_means(Q, means, nprobe) -> np.ndarray:
    """Soft inverted index routing (Sec. 3.2): for every query the nprobe
    means nearest it by the Def. 1 distance, nearest first, ties to the lower
    index, NaN distances last.  Returns nq x nprobe int32."""
    Q, means = _f32(np.atleast_2d(Q)), _f32(means)
    out = np.zeros((Q.shape[0], nprobe), np.int32)
    for i in range(Q.shape[0]):
        rc = _L().orc_probe(_p(Q[i]), Q.shape[1], _p(means), means.shape[0], nprobe, _p(out[i]))
        if rc != 0:
            raise ValueError("orc_probe: invalid nprobe %d for %d means" % (nprobe, means.shape[0]))
    return out


def probe_lists(probe, row_mean, live=None):
    """Candidate lists of the soft inverted index: for every query, the slots
    whose row is assigned to one of its probed means (and live, if given), in
    ascending slot order.  row_mean: the mean id of every slot (header byte
    12).  Returns (offsets, ids) in the layout of lvq_distances."""
    row_mean = np.asarray(row_mean)
    ok = np.ones(row_mean.shape[0], bool) if live is None else np.asarray(live, bool)
    lists = [np.flatnonzero(np.isin(row_mean, p) & ok).astype(np.int32) for p in np.asarray(probe)]
    offsets = np.zeros(len(lists) + 1, np.int64)
    offsets[1:] = np.cumsum([len(x) for x in lists])
    ids = np.concatenate(lists) if lists and offsets[-1] else np.zeros(0, np.int32)
    return offsets, ids


def encode_codes(x, mean, bits1, bits2=0):
    """Codes of one vector: returns (rc, l, delta, delta2, c1, c2)."""
    x, mean = _f32(x), _f32(mean)
    d = x.shape[-1]
    out = np.zeros(3, np.float32)
    c1 = np.zeros(d, np.uint8)
    c2 = np.zeros(d, np.uint8)
    rc = _L().orc_encode_codes(_p(x), d, _p(mean), bits1, bits2, _p(out[0:1]), _p(out[1:2]),
                               _p(out[2:3]), _p(c1), _p(c2) if bits2 else None)
    return rc, float(out[0]), float(out[1]), float(out[2]), c1, c2


def encode_rows(fmt: Format, X, means):
    """Encode vectors into (rows, resid, n_rejected)."""
    X, means = _f32(X), _f32(means)
    n = X.shape[0]
    f = fmt._c()
    rows = np.zeros((n, f.row_bytes), np.uint8)
    resid = np.zeros((n, f.resid_bytes), np.uint8) if fmt.bits2 else None
    rej = _L().orc_encode_rows(ctypes.byref(f), _p(X), n, _p(means), means.shape[0],
                               _p(rows), _p(resid))
    return rows, resid, int(rej)


def unpack(fmt: Format, rows, resid=None):
    """Header fields and codes (logical dim order) of every row."""
    f = fmt._c()
    rows = np.ascontiguousarray(rows, np.uint8).reshape(-1, f.row_bytes)
    n = rows.shape[0]
    hdr = np.zeros((3, n), np.float32)
    mid = np.zeros(n, np.int32)
    c1 = np.zeros((n, fmt.dim), np.uint8)
    c2 = np.zeros((n, fmt.dim), np.uint8)
    res = None if resid is None else np.ascontiguousarray(resid, np.uint8).reshape(n, f.resid_bytes)
    _L().orc_unpack_rows(ctypes.byref(f), _p(rows), _p(res), n, _p(hdr[0]), _p(hdr[1]), _p(hdr[2]), _p(mid),
                         _p(c1), _p(c2))
    return hdr[0], hdr[1], hdr[2], mid, c1, c2


def reconstruct(fmt: Format, rows, resid, means, level=PRIMARY) -> np.ndarray:
    f = fmt._c()
    rows = np.ascontiguousarray(rows, np.uint8).reshape(-1, f.row_bytes)
    means = _f32(means)
    out = np.zeros((rows.shape[0], fmt.dim), np.float64)
    res = None if resid is None else np.ascontiguousarray(resid, np.uint8).reshape(rows.shape[0], f.resid_bytes)
    _L().orc_reconstruct_rows(ctypes.byref(f), _p(rows), _p(res), rows.shape[0], _p(means), level, _p(out))
    return out


def distances(fmt: Format, metric, level, Q, rows, resid, means, offsets, ids) -> np.ndarray:
    """binary64 similarity of every (query, listed slot) pair."""
    f = fmt._c()
    Q, means = _f32(Q), _f32(means)
    rows = np.ascontiguousarray(rows, np.uint8)
    resid = None if resid is None else np.ascontiguousarray(resid, np.uint8)
    offsets = np.ascontiguousarray(offsets, np.int64)
    ids = np.ascontiguousarray(ids, np.int32)
    out = np.zeros(ids.shape[0], np.float64)
    _L().orc_distances(ctypes.byref(f), metric, level, _p(Q), Q.shape[0], _p(rows), _p(resid),
                       _p(means), _p(offsets), _p(ids), _p(out))
    return out


def select_topk(metric, score, slot, k, keep=None):
    score = np.ascontiguousarray(score, np.float64)
    slot = np.ascontiguousarray(slot, np.int32)
    keep = None if keep is None else np.ascontiguousarray(keep, np.uint8)
    ts = np.zeros(k, np.int32)
    tv = np.zeros(k, np.float64)
    _L().orc_select_topk(metric, _p(score), _p(slot), _p(keep), score.shape[0], k, _p(ts), _p(tv))
    return ts, tv


def topk_lists(metric, dist, offsets, ids, k, keep_slot=None):
    """Best k of every candidate list; keep_slot masks slots (lazy deletes)."""
    nq = len(offsets) - 1
    out_s = np.zeros((nq, k), np.int32)
    out_v = np.zeros((nq, k), np.float64)
    for i in range(nq):
        a, b = int(offsets[i]), int(offsets[i + 1])
        keep = None if keep_slot is None else keep_slot[ids[a:b]]
        out_s[i], out_v[i] = select_topk(metric, dist[a:b], ids[a:b], k, keep)
    return out_s, out_v


def topk_exhaustive(fmt: Format, metric, level, Q, rows, resid, means, k, live=None):
    """Best k over every live slot for every query (brute-force scan)."""
    nq = Q.shape[0]
    n = rows.shape[0]
    slots = np.arange(n, dtype=np.int32) if live is None else np.flatnonzero(live).astype(np.int32)
    out_s = np.zeros((nq, k), np.int32)
    out_v = np.zeros((nq, k), np.float64)
    for i in range(nq):
        offs = np.array([0, slots.shape[0]], np.int64)
        d = distances(fmt, metric, level, Q[i:i + 1], rows, resid, means, offs, slots)
        out_s[i], out_v[i] = select_topk(metric, d, slots, k)
    return out_s, out_v


def _walk(score, metric, graph, entries, W, k, live=None, tol=None, margins=None):
    """The steps of Alg. 1 around a scoring function (slots -> binary64
    values): the candidate set starts as the entry nodes; while it holds an
    unexplored node, the closest one is explored and its out-neighbours join
    the set, which is then cut to the W closest; the result is the k closest.
    Nodes are ranked by similarity, ties to the lower slot (Sec. 2.1); deleted
    rows are traversed but left out of the result (App. A, lazy deletes).

    A node proposed once is never proposed again: the W-th best rank of the
    set never worsens, so a node cut from the set could not re-enter it.

    With `tol` (slot -> error bound of an approximate score) and a list
    `margins`, every decision that compares two scores appends its margin,
    |a - b| - (tol(a) + tol(b)): the choice of the next node (the closest
    unexplored one against the runner-up), each cut of the set (its W-th
    against the (W+1)-th) and the result (its k-th against the next live one).
    A walk all of whose margins are positive is taken by any evaluation of
    the scores within those bounds."""

    def rank(item):
        slot, v = item
        return (v if metric == L2 else -v, slot)

    def note(a, b):
        if margins is not None:
            margins.append(abs(a[1] - b[1]) - (tol(a[0]) + tol(b[0])))

    entries = sorted(set(int(e) for e in entries))
    cand = dict(zip(entries, score(entries)))
    seen = set(entries)
    explored = set()
    while True:
        open_ = sorted((it for it in cand.items() if it[0] not in explored), key=rank)
        if not open_:
            break
        if len(open_) > 1:
            note(open_[0], open_[1])
        x = open_[0][0]
        explored.add(x)
        new = [int(y) for y in graph[x] if y >= 0 and int(y) not in seen]
        seen.update(new)
        if new:
            cand.update(zip(new, score(new)))
        if len(cand) > W:
            ranked = sorted(cand.items(), key=rank)
            note(ranked[W - 1], ranked[W])
            cand = dict(ranked[:W])
    ranked = [it for it in sorted(cand.items(), key=rank) if live is None or live[it[0]]]
    if len(ranked) > k:
        note(ranked[k - 1], ranked[k])
    out = ranked[:k]
    return (np.array([s for s, _ in out], np.int32), np.array([v for _, v in out], np.float64), len(explored))


def greedy_search(fmt: Format, metric, level, q, rows, resid, means, graph, entries, W, k, live=None, tol=None,
                  margins=None):
    """Greedy graph search (Alg. 1) for one query over LVQ rows, with the
    similarities of ``distances`` at the given level.  graph: n x R slots, -1
    for no edge.  Returns (slots, values) of length <= k, best first, and the
    number of nodes explored.  tol / margins: as ``_walk``."""
    q = np.asarray(q, np.float32)[None, :]

    def score(slots):
        slots = np.asarray(slots, np.int32)
        return distances(fmt, metric, level, q, rows, resid, means, np.array([0, slots.size], np.int64), slots)

    return _walk(score, metric, graph, entries, W, k, live, tol, margins)


def float_sim(metric, a, b) -> float:
    """Similarity of two float vectors in binary64: the squared Euclidean
    distance (L2, smaller is closer) or the inner product (IP)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(((a - b) ** 2).sum()) if metric == L2 else float((a * b).sum())


def greedy_search_float(metric, q, X, graph, entries, W, k):
    """Alg. 1 over float vectors X (binary64 similarities): the search that
    graph construction runs for a node (App. A, initial build)."""

    def score(slots):
        return np.array([float_sim(metric, q, X[s]) for s in slots], np.float64)

    return _walk(score, metric, graph, entries, W, k)


def robust_prune(metric, X, p, cand, current, alpha, R, tol=None, margins=None):
    """Neighbourhood pruning (Alg. 2) of node p over float vectors X.

    The candidates are the given ones and p's current out-neighbours, without
    p.  The closest candidate x* (ties to the lower slot) becomes an
    out-neighbour and leaves the candidates; stop at R out-neighbours;
    otherwise every candidate x' for which x* is at least alpha times as
    similar as p is removed: for the inner product alpha * <x*, x'> >=
    <p, x'>, for L2 (similarity = the squared distance, smaller is closer)
    alpha * |x* - x'|^2 <= |p - x'|^2.  Returns the new out-neighbours in
    selection order.

    With `tol` ((a, b, similarity) -> error bound of an approximate
    similarity of vectors a and b) and a list `margins`, the decisions append
    their margins: the ranking of the candidates by similarity to p (each
    adjacent pair, |s - s'| - (tol + tol')) and every test of the rule
    (|alpha t - s| - (alpha tol_t + tol_s)).  A pruning all of whose margins
    are positive is reproduced by any evaluation within those bounds."""
    C = sorted(set(int(c) for c in list(cand) + list(current) if c >= 0) - {int(p)})
    sims = {c: float_sim(metric, X[p], X[c]) for c in C}
    order = sorted(C, key=lambda c: (sims[c] if metric == L2 else -sims[c], c))
    if margins is not None:
        for a, b in zip(order, order[1:]):
            margins.append(abs(sims[a] - sims[b]) - (tol(p, a, sims[a]) + tol(p, b, sims[b])))
    out = []
    while order:
        xs = order.pop(0)
        out.append(xs)
        if len(out) == R:
            break
        keep = []
        for c in order:
            t = float_sim(metric, X[xs], X[c])
            removed = alpha * t <= sims[c] if metric == L2 else alpha * t >= sims[c]
            if margins is not None:
                margins.append(abs(alpha * t - sims[c]) - (alpha * tol(xs, c, t) + tol(p, c, sims[c])))
            if not removed:
                keep.append(c)
        order = keep
    return out


def vamana_insert(metric, X, graph, nodes, entry, W, alpha, R):
    """The update routine of graph construction (App. A) for each node x of
    `nodes` in turn, in place on graph (n x R, -1 for no edge): the W nearest
    nodes to x found by Alg. 1 from `entry` are pruned together with x's
    current out-neighbours (Alg. 2) into its new out-neighbours; x then joins
    the out-neighbours of each of them, which are pruned (Alg. 2) when that
    exceeds R."""
    def row(y):
        return [int(v) for v in graph[y] if v >= 0]

    def put(y, ns):
        graph[y] = -1
        graph[y, :len(ns)] = ns

    for x in nodes:
        x = int(x)
        found, _, _ = greedy_search_float(metric, X[x], X, graph, [entry], W, W)
        nx = robust_prune(metric, X, x, found, row(x), alpha, R)
        put(x, nx)
        for y in nx:
            ny = row(y)
            if x in ny:
                continue
            if len(ny) < R:
                put(y, ny + [x])
            else:
                put(y, robust_prune(metric, X, y, [x], ny, alpha, R))
    return graph


def vamana_update(metric, X, graph, order, in_graph, entry, W, alpha, R, passes, max_batch):
    """The update routine of App. A run in batches, as the batched reading of
    the construction takes it: the rows of the nodes of `order` are cleared;
    then, `passes` times (alpha = 1 first when there are two passes), the
    nodes are taken in batches of at most max_batch (and, in the first pass,
    at most the number of nodes already in the graph: in_graph plus the
    nodes processed so far, at least one).  Every node of a batch finds its
    W nearest by Alg. 1 from `entry` in the graph as it was before the batch
    and prunes them with its current out-neighbours (Alg. 2) into its new
    out-neighbours; then each node y named by the batch's new rows takes all
    of its new sources at once: their union with N(y) if it holds at most R
    nodes, else Alg. 2 over the sources and N(y).  With max_batch = 1 this is
    vamana_insert / vamana_build.  In place on graph (n x R, -1 padded)."""
    n = X.shape[0]
    order = [int(v) for v in order]

    def row(y):
        return [int(v) for v in graph[y] if v >= 0]

    def put(y, ns):
        graph[y] = -1
        graph[y, :len(ns)] = ns

    for v in order:
        graph[v] = -1
    count = len(order)
    B = min(max_batch, count)
    for pass_ in range(passes):
        a = 1.0 if (passes == 2 and pass_ == 0) else alpha
        b = 0
        while b < count:
            now = in_graph + b if pass_ == 0 else n
            bs = min(B, max(1, now), count - b)
            batch = order[b:b + bs]
            before = graph.copy()
            new_rows = []
            for x in batch:
                found, _, _ = greedy_search_float(metric, X[x], X, before, [entry], W, W)
                new_rows.append(robust_prune(metric, X, x, found, [int(v) for v in before[x] if v >= 0], a, R))
            for x, nx in zip(batch, new_rows):
                put(x, nx)
            sources = {}
            for x, nx in zip(batch, new_rows):
                for y in nx:
                    sources.setdefault(y, []).append(x)
            for y, S in sources.items():
                ny = row(y)
                union = ny + [v for v in dict.fromkeys(S) if v not in ny and v != y]
                if len(union) <= R:
                    put(y, union)
                else:
                    put(y, robust_prune(metric, X, y, S, ny, a, R))
            b += bs
    return graph


def vamana_delete(metric, X, graph, deleted, alpha, R):
    """Delete consolidation (App. A) of the nodes flagged in `deleted`, on a
    copy of graph: every kept node x' with deleted out-neighbours gets as
    candidates its kept out-neighbours and the kept out-neighbours of each
    deleted one (x' -> x -> x'' becomes x' -> x''), without x' itself; more
    than R distinct candidates are pruned (Alg. 2).  All rows are read from
    the graph before the consolidation; rows of deleted nodes are cleared."""
    deleted = np.asarray(deleted, bool)
    out = graph.copy()
    for p in range(graph.shape[0]):
        if deleted[p]:
            continue
        row = [int(v) for v in graph[p] if v >= 0]
        if not any(deleted[v] for v in row):
            continue
        cand = set()
        for v in row:
            if deleted[v]:
                cand.update(int(u) for u in graph[v] if u >= 0 and not deleted[u] and u != p)
            else:
                cand.add(v)
        cand = sorted(cand)
        keep = robust_prune(metric, X, p, cand, [], alpha, R) if len(cand) > R else cand
        out[p] = -1
        out[p, :len(keep)] = keep
    out[deleted] = -1
    return out


def vamana_build(metric, X, entry, W, alpha, R, order=None):
    """Initial build (App. A): an empty graph, then the update routine for
    every node twice, first with alpha = 1 and then with the given alpha.
    The entry node goes first; the others follow `order` (default: slot
    order)."""
    n = X.shape[0]
    graph = np.full((n, R), -1, np.int32)
    rest = [int(v) for v in (range(n) if order is None else order) if int(v) != int(entry)]
    seq = [int(entry)] + rest
    for a in (1.0, alpha):
        vamana_insert(metric, X, graph, seq, entry, W, a, R)
    return graph


def eps1(fmt: Format, X, rows, means) -> float:
    """Eq. 4 first-level quantisation error (sum over vectors)."""
    f = fmt._c()
    X = _f32(X)
    rows = np.ascontiguousarray(rows, np.uint8)
    return float(_L().orc_eps1(ctypes.byref(f), _p(X), X.shape[0], _p(rows), _p(_f32(means))))


def recall(found, truth) -> float:
    """k-recall@k = |S intersect G| / k averaged over queries (Sec. 2.1)."""
    found = np.asarray(found)
    truth = np.asarray(truth)
    k = truth.shape[1]
    hits = sum(len(set(found[i].tolist()) & set(truth[i].tolist())) for i in range(truth.shape[0]))
    return hits / float(k * truth.shape[0])


def float_groundtruth(metric, Q, X, k, live=None, chunk=4096):
    """binary64 brute-force top-k over the original float vectors (the ground
    truth G_t of Sec. 2.1), ties to the lower slot."""
    Q = np.asarray(Q, np.float64)
    slots = np.arange(X.shape[0]) if live is None else np.flatnonzero(live)
    best_s = np.zeros((Q.shape[0], 0), np.int64)
    best_v = np.zeros((Q.shape[0], 0), np.float64)
    for a in range(0, slots.shape[0], chunk):
        sl = slots[a:a + chunk]
        Xs = np.asarray(X[sl], np.float64)
        if metric == IP:
            v = -(Q @ Xs.T)                       # rank by descending similarity
        else:
            v = (Q * Q).sum(1)[:, None] - 2.0 * (Q @ Xs.T) + (Xs * Xs).sum(1)[None, :]
        cv = np.concatenate([best_v, v], 1)
        cs = np.concatenate([best_s, np.broadcast_to(sl, v.shape)], 1)
        order = np.lexsort((cs, cv), axis=1)[:, :k]
        best_v = np.take_along_axis(cv, order, 1)
        best_s = np.take_along_axis(cs, order, 1)
    return best_s.astype(np.int32)

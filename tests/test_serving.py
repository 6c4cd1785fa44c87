"""Request server (lvq_server_* of the C ABI): batches admitted by stream
slots and pool memory, run concurrently beside store updates, answered at
their admission epoch.

* A batch's result in the mix (several batches in flight, inserts and deletes
  issued meanwhile from the host) is bit-identical to the same batch served
  alone on a store replayed to the same epoch, and to the direct calls it
  stands for (lvq_topk first level, then lvq_distances at both levels with a
  top-k over those candidates).
* The alone results hold oracle values: every returned distance matches the
  oracle's two-level value of that slot, every slot is live at the epoch.
* Admission by memory: a pool that fits one largest batch runs one at a time,
  while small batches share it.
* Batches overlap on the device: a burst is admitted into several slots and
  their admission-to-completion intervals overlap.
* Consolidation during serving never hands a batch a slot that was not live
  at the batch's epoch.
"""
import threading

import numpy as np
import pytest

import oracle
import synth
from lvq_check import check_values, pair_reference

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

D, N0, CAP = 256, 6000, 9000
K, KF, MAXB = 10, 32, 48


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2402_02044_amd as lib
    return lib


def _data():
    g = synth.rng(7000, 0)
    cent = g.standard_normal((16, D)).astype(np.float32)

    def draw(n, shift=0.0):
        x = cent[g.integers(0, 16, n)] + shift + 0.5 * g.standard_normal((n, D)).astype(np.float32)
        return (x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)

    X0 = draw(N0)
    means = X0[g.choice(N0, 4, replace=False)]
    # an operation script: batches (sizes U{1..MAXB}) and updates in between
    ops = []
    for i in range(36):
        nq = int(g.integers(1, MAXB + 1))
        ops.append(("batch", draw(nq)))
        if i % 6 == 5:
            ops.append(("insert", draw(150, 0.05)))
            ops.append(("delete", int(g.integers(0, 1 << 30))))
    return X0, means, ops


class Store:
    """The index plus a host model of slot contents and liveness."""

    def __init__(self, L, X0, means):
        self.L = L
        self.ix = L.Index(D, 4, 8, L.LVQ_IP, L.LVQ_TURBO, capacity=CAP, means=means)
        self.means = means
        self.X = np.zeros((CAP, D), np.float32)
        self.live = np.zeros(CAP, bool)
        self.stream = torch.cuda.Stream()
        self.insert(X0)
        torch.cuda.synchronize()

    def insert(self, X):
        with torch.cuda.stream(self.stream):
            xd = torch.from_numpy(X).cuda()
            slots = self.ix.insert(xd).cpu().numpy()    # the copy synchronises this stream
        self.X[slots] = X
        self.live[slots] = True

    def delete(self, seed):
        cand = np.flatnonzero(self.live)
        dead = np.sort(np.random.default_rng(seed).choice(cand, 200, replace=False)).astype(np.int32)
        with torch.cuda.stream(self.stream):
            self.ix.delete(torch.from_numpy(dead).cuda())
        self.stream.synchronize()
        self.live[dead] = False

    def apply(self, op):
        if op[0] == "insert":
            self.insert(op[1])
        else:
            self.delete(op[1])

    def epoch(self):
        return self.ix.stats().epoch


def _run_mix(L, prec, scan_level, slots, pool_batches):
    X0, means, ops = _data()
    st = Store(L, X0, means)
    kw = dict(max_batch=MAXB, k=K, k_first=KF, precision=prec, scan_level=scan_level)
    probe = L.Server(st.ix, slots=1, **kw)
    pool = int(probe.stats().batch_bytes_max * pool_batches)
    probe.close()
    sv = L.Server(st.ix, slots=slots, pool_bytes=pool, **kw)
    tickets = []
    for op in ops:
        if op[0] == "batch":
            tickets.append((sv.submit(op[1]), op[1]))
        else:
            st.apply(op)
    out = [sv.wait(t, q.shape[0]) for t, q in tickets]
    stats = sv.stats()
    sv.close()
    assert st.ix.sync() == 0
    st.ix.close()
    return ops, out, stats


def _replay_alone(L, prec, scan_level, ops, epochs):
    """Serve each batch alone (one slot) on a store replayed to its epoch;
    also run the direct calls the server stands for."""
    X0, means, _ = _data()
    st = Store(L, X0, means)
    sv = L.Server(st.ix, slots=1, max_batch=MAXB, k=K, k_first=KF, precision=prec, scan_level=scan_level)
    updates = [op for op in ops if op[0] != "batch"]
    batches = [op[1] for op in ops if op[0] == "batch"]
    order = np.argsort(np.asarray(epochs), kind="stable")
    done = 0
    res = [None] * len(batches)
    fmt = oracle.Format(D, 4, 8, oracle.TURBO)
    tdt = {L.LVQ_FP32: torch.float32, L.LVQ_BF16: torch.bfloat16, L.LVQ_FP16: torch.float16}[prec]
    for b in order:
        while st.epoch() < epochs[b]:
            st.apply(updates[done])
            done += 1
        assert st.epoch() == epochs[b]
        q = batches[b]
        t = sv.submit(q)
        ids, dist, info = sv.wait(t, q.shape[0])
        assert info.epoch == epochs[b]
        # the direct calls: an exhaustive scan at both levels, or first-level
        # top-k' and both-level re-rank
        qd = torch.from_numpy(q).cuda()
        if scan_level == L.LVQ_FULL:
            ti, td = st.ix.topk(qd.to(tdt), K, level=L.LVQ_FULL)
        else:
            cid, _ = st.ix.topk(qd.to(tdt), KF)
            offs = torch.arange(0, (q.shape[0] + 1) * KF, KF, dtype=torch.int64, device="cuda")
            _, ti, td = st.ix.distances(qd, offs, cid.reshape(-1), level=L.LVQ_FULL, k=K, want_dist=False)
        assert np.array_equal(ti.cpu().numpy(), ids) and np.array_equal(td.cpu().numpy(), dist), b
        # oracle values of the returned slots, all live at the epoch
        assert st.live[ids].all() and (ids >= 0).all()
        rows, resid, _ = oracle.encode_rows(fmt, st.X[ids.reshape(-1)], means)
        loc = np.arange(ids.size, dtype=np.int32)
        offs_h = np.arange(q.shape[0] + 1, dtype=np.int64) * K
        # values: two-level similarities of the fp32 queries after a re-rank,
        # of the 16-bit queries when the matrix-core scan produced them
        qv = q if (prec == L.LVQ_FP32 or scan_level != L.LVQ_FULL) else torch.from_numpy(q).to(tdt).float().numpy()
        ref, tol = pair_reference(fmt, oracle.IP, oracle.FULL, qv, rows, resid, means, offs_h, loc)
        check_values(dist.reshape(-1), ref, tol, "served distances")
        assert np.all(np.diff(dist, axis=1) <= 0), "results ordered best first"
        res[b] = (ids, dist)
    sv.close()
    assert st.ix.sync() == 0
    st.ix.close()
    return res


@pytest.mark.parametrize("form", ["fp32-rerank", "bf16-rerank", "fp32-full", "bf16-full"])
def test_mix_equals_alone(L, form):
    prec = {"fp32": L.LVQ_FP32, "bf16": L.LVQ_BF16}[form.split("-")[0]]
    scan_level = L.LVQ_FULL if form.endswith("full") else L.LVQ_PRIMARY
    ops, mixed, stats = _run_mix(L, prec, scan_level, slots=5, pool_batches=2.5)
    assert stats.completed == len(mixed) and stats.peak_in_flight >= 2
    assert stats.pool_peak <= stats.pool_bytes
    epochs = [info.epoch for _, _, info in mixed]
    assert len(set(epochs)) > 1, "updates should interleave with the batches"
    alone = _replay_alone(L, prec, scan_level, ops, epochs)
    for b, ((ids, dist, info), (ids1, dist1)) in enumerate(zip(mixed, alone)):
        assert np.array_equal(ids, ids1), "batch %d (epoch %d): ids differ from the alone run" % (b, info.epoch)
        assert np.array_equal(dist, dist1), "batch %d (epoch %d): values differ" % (b, info.epoch)
        assert info.t_submit <= info.t_admit <= info.t_done


def test_admission_by_memory(L):
    X0, means, _ = _data()
    st = Store(L, X0, means)
    sv = L.Server(st.ix, slots=1, max_batch=MAXB, k=K, k_first=KF)
    one = sv.stats().batch_bytes_max
    sv.close()
    # a pool for one largest batch: largest batches run one at a time although
    # four slots are free; small batches share the pool
    sv = L.Server(st.ix, slots=4, max_batch=MAXB, k=K, k_first=KF, pool_bytes=one)
    g = synth.rng(7001, 0)
    big = [sv.submit(g.standard_normal((MAXB, D)).astype(np.float32)) for _ in range(6)]
    for t in big:
        sv.wait(t, MAXB)
    s1 = sv.stats()
    assert s1.peak_in_flight == 1 and s1.pool_peak <= one
    small = [sv.submit(g.standard_normal((1, D)).astype(np.float32)) for _ in range(24)]
    for t in small:
        sv.wait(t, 1)
    s2 = sv.stats()
    assert s2.pool_peak <= one and s2.completed == 30
    assert s2.peak_in_flight >= 2, "small batches should share the pool of one large batch"
    with pytest.raises(L.LVQError):
        sv.submit(np.zeros((MAXB + 1, D), np.float32))
    with pytest.raises(L.LVQError):
        sv.wait(10 ** 9, 1)
    sv.close()
    st.ix.close()


def _overlapping_pairs(infos):
    iv = sorted((i.t_admit, i.t_done) for i in infos)
    return sum(1 for a in range(len(iv)) for b in range(a + 1, len(iv)) if iv[b][0] < iv[a][1])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batches_overlap_on_the_device(L, prec):
    """Continuous batching: a burst of batches over a 200,000-row store is
    admitted into several slots at once, so batches run on the device at the
    same time (overlapping admission-to-completion intervals), and each
    result equals the direct exhaustive call on the same store."""
    g = synth.rng(7003, 0)
    n, nb = 200_000, 16
    cent = g.standard_normal((16, D)).astype(np.float32)
    X = cent[g.integers(0, 16, n)] + 0.5 * g.standard_normal((n, D)).astype(np.float32)
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    ix = L.Index(D, 4, 8, L.LVQ_IP, L.LVQ_TURBO, capacity=n, means=X[:4])
    ix.insert(torch.from_numpy(X).cuda())
    assert ix.sync() == 0
    p = {"fp32": L.LVQ_FP32, "bf16": L.LVQ_BF16}[prec]
    sv = L.Server(ix, slots=6, max_batch=MAXB, k=K, k_first=KF, precision=p, scan_level=L.LVQ_FULL)
    qs = [(X[g.integers(0, n, MAXB)] + 0.1 * g.standard_normal((MAXB, D))).astype(np.float32) for _ in range(nb)]
    tickets = [sv.submit(q) for q in qs]
    res = [sv.wait(t, MAXB) for t in tickets]
    st = sv.stats()
    sv.close()
    assert st.completed == nb and st.peak_in_flight >= 2
    assert _overlapping_pairs([info for _, _, info in res]) >= 1
    tdt = torch.float32 if prec == "fp32" else torch.bfloat16
    for q, (ids, dist, info) in zip(qs, res):
        ti, td = ix.topk(torch.from_numpy(q).cuda().to(tdt), K, level=L.LVQ_FULL)
        assert np.array_equal(ti.cpu().numpy(), ids) and np.array_equal(td.cpu().numpy(), dist)
    assert ix.sync() == 0
    ix.close()


def test_consolidation_while_serving(L):
    """Deletes and consolidations race with batches in flight; every batch
    returns only slots live at its own epoch (per the host model, recorded at
    every epoch), so no reclaimed-and-reused slot leaks into a result."""
    X0, means, _ = _data()
    st = Store(L, X0, means)
    sv = L.Server(st.ix, slots=6, max_batch=MAXB, k=K, k_first=KF)
    live_at = {st.epoch(): st.live.copy()}
    g = synth.rng(7002, 0)
    stop = threading.Event()
    submitted = []

    def client():
        while not stop.is_set() and len(submitted) < 400:
            q = g.standard_normal((int(g.integers(1, MAXB + 1)), D)).astype(np.float32)
            submitted.append((sv.submit(q), q.shape[0]))

    th = threading.Thread(target=client)
    th.start()
    try:
        for r in range(6):
            st.delete(1000 + r)
            live_at[st.epoch()] = st.live.copy()
            st.ix.consolidate(stream=st.stream)
            st.insert(np.ascontiguousarray(X0[r * 100:(r + 1) * 100]))
            live_at[st.epoch()] = st.live.copy()
    finally:
        stop.set()
        th.join()
    seen = set()
    for t, nq in submitted:
        ids, _, info = sv.wait(t, nq)
        seen.add(info.epoch)
        assert info.epoch in live_at, info.epoch
        assert live_at[info.epoch][ids].all(), "a batch returned a slot not live at its epoch"
    sv.close()
    assert st.ix.sync() == 0
    st.ix.close()

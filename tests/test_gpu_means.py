"""Online re-estimation of M-LVQ means (lvq_retire_means, lvq_add_means,
lvq_mean_members of the C ABI) against the oracle and a host model.

* Retired means are never chosen: rows inserted afterwards are bit-exact with
  the oracle's encoding against the active means only.
* A retired id is reused only once no occupied slot refers to it (its rows
  deleted and freed by a consolidation); otherwise new ids are appended, up
  to 256 ids.
* The live members of a mean are exactly the live rows the oracle assigns to
  it; re-encoding them (delete + insert of the original vectors) moves them
  to the new centres.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

D = 64


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2402_02044_amd as lib
    return lib


def _rows_match(L, ix, fmt, slots, X, means_by_id, active):
    """Stored rows of `slots` against the oracle's encoding of X with the
    active means only (mean byte mapped back to the ids)."""
    act = np.flatnonzero(active)
    rows, _, _ = oracle.encode_rows(fmt, X, means_by_id[act])
    g_rows, _ = ix.read_rows(torch.from_numpy(np.asarray(slots, np.int32)).cuda())
    g = g_rows.cpu().numpy()
    np.testing.assert_array_equal(g[:, :12], rows[:, :12])
    np.testing.assert_array_equal(g[:, 12], act[rows[:, 12]])
    np.testing.assert_array_equal(g[:, 32:], rows[:, 32:])
    return g[:, 12]


def _store(L, M, n, cap, seed):
    g = synth.rng(8400 + seed, 0)
    cent = (2.0 * g.standard_normal((M, D))).astype(np.float32)
    X = (cent[g.integers(0, M, n)] + 0.4 * g.standard_normal((n, D))).astype(np.float32)
    ix = L.Index(D, 8, 0, L.LVQ_L2, L.LVQ_SEQUENTIAL, capacity=cap, means=cent)
    return g, cent, X, ix


def test_retired_means_are_not_chosen(L):
    g, cent, X, ix = _store(L, 6, 2000, 4000, 0)
    fmt = oracle.Format(D, 8, 0, oracle.SEQUENTIAL)
    ix.retire_means([1, 4])
    slots = ix.insert(torch.from_numpy(X).cuda()).cpu().numpy()
    assert ix.sync() == 0
    active = np.array([1, 0, 1, 1, 0, 1], bool)
    mid = _rows_match(L, ix, fmt, slots, X, cent, active)
    assert not np.isin(mid, [1, 4]).any()
    with pytest.raises(L.LVQError):
        ix.retire_means([0, 2, 3, 5])          # no active mean would be left
    with pytest.raises(L.LVQError):
        ix.retire_means([6])                   # not an id
    ix.close()


def test_add_means_reuses_freed_ids_and_members_follow(L):
    M, n = 4, 3000
    g, cent, X, ix = _store(L, M, n, 5000, 1)
    fmt = oracle.Format(D, 8, 0, oracle.SEQUENTIAL)
    ext = np.arange(n, dtype=np.uint64) + 10_000
    slots = ix.insert(torch.from_numpy(X).cuda(), ext_ids=torch.from_numpy(ext.astype(np.int64)).cuda())
    slots = slots.cpu().numpy()
    assert ix.sync() == 0
    means_by_id = np.zeros((256, D), np.float32)
    means_by_id[:M] = cent
    active = np.zeros(256, bool)
    active[:M] = True
    live = np.zeros(5000, bool)
    live[slots] = True
    Xs = np.zeros((5000, D), np.float32)
    Xs[slots] = X
    mid = np.full(5000, -1)
    mid[slots] = _rows_match(L, ix, fmt, slots, X, means_by_id[:M], active[:M])

    # members of every mean: the live rows assigned to it
    dead = np.sort(g.choice(slots, 500, replace=False)).astype(np.int32)
    ix.delete(torch.from_numpy(dead).cuda())
    live[dead] = False
    offs, mem = ix.mean_members(np.arange(M), cap=n)
    mem = mem.cpu().numpy()
    for m in range(M):
        got = np.sort(mem[offs[m]:offs[m + 1]])
        np.testing.assert_array_equal(got, np.flatnonzero(live & (mid == m)))
    with pytest.raises(L.LVQError) as e:
        ix.mean_members(np.arange(M), cap=10)
    assert e.value.code == L.LVQ_ERR_CAPACITY

    # centre 2 moves: add the new centre, retire the old id, re-encode its rows
    new_c = (cent[2] + 0.3).astype(np.float32)
    ids = ix.add_means(new_c)
    assert ids.tolist() == [M]                  # nothing retired yet: appended
    means_by_id[M] = new_c
    active[M] = True
    ix.retire_means([2])
    active[2] = False
    offs, mem = ix.mean_members([2], cap=n)
    move = np.sort(mem.cpu().numpy())
    np.testing.assert_array_equal(move, np.flatnonzero(live & (mid == 2)))
    ix.delete(torch.from_numpy(move.astype(np.int32)).cuda())
    live[move] = False
    new_slots = ix.insert(torch.from_numpy(Xs[move]).cuda(),
                          ext_ids=torch.from_numpy((move.astype(np.int64) + 10_000)).cuda()).cpu().numpy()
    assert ix.sync() == 0
    live[new_slots] = True
    Xs[new_slots] = Xs[move]
    mid[new_slots] = _rows_match(L, ix, fmt, new_slots, Xs[move], means_by_id[:M + 1], active[:M + 1])
    assert not (mid[new_slots] == 2).any()

    # id 2 is retired but its deleted rows still occupy slots: a new mean is appended
    ids = ix.add_means((cent[0] + 0.1).astype(np.float32))
    assert ids.tolist() == [M + 1]
    means_by_id[M + 1] = cent[0] + 0.1
    active[M + 1] = True
    # after a consolidation frees them, id 2 is reused
    ix.consolidate()
    assert ix.sync() == 0
    ids = ix.add_means((cent[1] - 0.2).astype(np.float32))
    assert ids.tolist() == [2]
    means_by_id[2] = cent[1] - 0.2
    active[2] = True
    more = (cent[1] - 0.2 + 0.05 * g.standard_normal((50, D))).astype(np.float32)
    s3 = ix.insert(torch.from_numpy(more).cuda()).cpu().numpy()
    assert ix.sync() == 0
    m3 = _rows_match(L, ix, fmt, s3, more, means_by_id[:M + 2], active[:M + 2])
    assert (m3 == 2).mean() > 0.5                # the reused id serves its new centre
    # at most 256 ids over the index's life
    with pytest.raises(L.LVQError) as e:
        ix.add_means(np.zeros((256, D), np.float32))
    assert e.value.code == L.LVQ_ERR_CAPACITY
    ids = ix.add_means(np.ones((256 - (M + 2), D), np.float32))
    assert sorted(ids.tolist()) == list(range(M + 2, 256))
    ix.close()

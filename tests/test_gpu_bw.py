"""Bandwidth probes (lvq_bw_stream, lvq_bw_gather): measurement kernels that
perform only the loads of an access pattern.  Their sink is the XOR of every
32-bit word read, checked here against the same words on the host."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2402_02044_amd as lib
    return lib


def _xor(words):
    return int(np.bitwise_xor.reduce(np.asarray(words, np.uint32).ravel(), initial=np.uint32(0)))


def test_stream_reads_every_word(L):
    g = synth.rng(9600, 0)
    for nbytes in (0, 16, 16 * 1001, 1 << 22):
        buf = g.integers(0, 2 ** 32, nbytes // 4, dtype=np.uint64).astype(np.uint32)
        src = torch.from_numpy(buf.view(np.int32)).cuda()
        sink = torch.full((1,), 7, dtype=torch.int32, device="cuda")
        L.lvq_bw_stream(src.data_ptr() if nbytes else sink.data_ptr(), nbytes, sink.data_ptr(), 0)
        torch.cuda.synchronize()
        assert int(sink.cpu().numpy().view(np.uint32)[0]) == _xor(buf), nbytes
    with pytest.raises(L.LVQError):
        L.lvq_bw_stream(src.data_ptr(), 20, sink.data_ptr(), 0)        # not a multiple of 16 bytes
    with pytest.raises(L.LVQError):
        L.lvq_bw_stream(src.data_ptr() + 4, 16, sink.data_ptr(), 0)    # not 16-byte aligned


@pytest.mark.parametrize("d,b1,b2,layout", [(130, 4, 8, 1), (96, 8, 0, 0), (768, 4, 8, 1)])
def test_gather_reads_the_candidate_bytes(L, d, b1, b2, layout):
    g = synth.rng(9610 + d, b1)
    n = 500
    X = g.standard_normal((n, d)).astype(np.float32)
    mu = X.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    ix = L.Index(d, b1, b2, L.LVQ_IP, layout, capacity=n, means=mu)
    ix.insert(torch.from_numpy(X).cuda())
    rows, resid = ix.read_rows(torch.arange(n, dtype=torch.int32, device="cuda"))
    rows = rows.cpu().numpy()
    resid = None if resid is None else resid.cpu().numpy()
    npos = -(-d // ({(4, 1): 128, (8, 1): 64, (4, 0): 8, (8, 0): 4}[(b1, layout)])) * \
        {(4, 1): 128, (8, 1): 64, (4, 0): 8, (8, 0): 4}[(b1, layout)]
    code_bytes = 32 + -(-(npos * b1 // 8) // 16) * 16      # header + the code chunks the kernels read
    ids = g.integers(0, n, 3000).astype(np.int32)
    ids[::7] = ids[1::7][:len(ids[::7])]                    # repeats
    ids[5] = -1
    ids[9] = n + 3                                          # out of range: skipped
    ok = (ids >= 0) & (ids < n)
    for level in ([L.LVQ_PRIMARY, L.LVQ_FULL] if b2 else [L.LVQ_PRIMARY]):
        want = _xor(rows[ids[ok], :code_bytes].view(np.uint32))
        if level == L.LVQ_FULL:
            want ^= _xor(resid[ids[ok]].view(np.uint32))
        sink = torch.zeros(1, dtype=torch.int32, device="cuda")
        idd = torch.from_numpy(ids).cuda()
        L.lvq_bw_gather(ix.handle, idd.data_ptr(), len(ids), level, sink.data_ptr(), 0)
        torch.cuda.synchronize()
        assert int(sink.cpu().numpy().view(np.uint32)[0]) == want, level
    assert ix.sync() == 0
    ix.close()

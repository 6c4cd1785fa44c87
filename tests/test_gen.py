"""The seeded generators are chunk-addressable and deterministic."""
import numpy as np

import synth


def test_slices_regenerate_exactly():
    full = synth.anisotropic(2, synth.S_BASE, 0, 3 * synth.CHUNK // 2, 16)
    part = synth.anisotropic(2, synth.S_BASE, synth.CHUNK - 5, 10, 16)
    np.testing.assert_array_equal(full[synth.CHUNK - 5:synth.CHUNK + 5], part)
    np.testing.assert_allclose(np.linalg.norm(full, axis=1), 1.0, rtol=1e-5)
    cent = synth.centres(1, 32, 8)
    a = synth.mixture(1, synth.S_BASE, 100, 50, cent, 0.3)
    b = synth.mixture(1, synth.S_BASE, 0, 200, cent, 0.3)
    np.testing.assert_array_equal(a, b[100:150])


def test_candidate_lists():
    off, ids = synth.candidate_lists(2, 300, 5000, length=100)
    assert off[-1] == 300 * 100 and ids.dtype == np.int32
    for i in range(300):
        lst = ids[off[i]:off[i + 1]]
        assert len(np.unique(lst)) == len(lst) and lst.min() >= 0 and lst.max() < 5000
    off2, ids2 = synth.candidate_lists(2, 300, 5000, length=100)
    np.testing.assert_array_equal(ids, ids2)
    off, ids = synth.candidate_lists(3, 2000, 100000, lmin=64, lmax=4096)
    lens = np.diff(off)
    assert lens.min() >= 64 and lens.max() <= 4096
    # log-uniform: mean near (4097 - 64) / ln(4097 / 64)
    assert abs(lens.mean() - (4097 - 64) / np.log(4097 / 64)) < 60

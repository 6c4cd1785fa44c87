"""Pins of the oracle's encoder against facts fixed by the paper and by the
mathematics (Eq. 1-3, the residual level of Sec. 2.3, Def. 1, the Turbo layout
of Sec. 3.1 / App. B).  Nothing here re-types the oracle's own formulas: codes
are checked by brute-force nearest-level search, bounds, extremes, the App. C
level-1 formula evaluated independently in numpy, and the worked example."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

BITS = [1, 2, 3, 4, 5, 6, 7, 8]
KINDS = ["normal", "uniform", "wide", "lowcard"]


def _data(seed, n, d, kind):
    X = synth.small_vectors(seed, n, d, kind)
    mu = X.astype(np.float64).mean(0).astype(np.float32)
    return X, mu


def _half_tie(v, tol=2.0 ** -16):
    """True where v is within tol of a half-integer (rounding is ambiguous)."""
    return np.abs((v - np.floor(v)) - 0.5) < tol


@pytest.mark.parametrize("bits", BITS)
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("d", [1, 3, 8, 96, 130])
def test_first_level_is_nearest_level(bits, kind, d):
    """Eq. 2: the code picks the nearest of the 2^B levels l + Delta c."""
    X, mu = _data(bits * 10 + len(kind), 24, d, kind)
    top = 2 ** bits - 1
    for x in X:
        rc, l, delta, _, c1, _ = oracle.encode_codes(x, mu, bits)
        assert rc == 0
        t = x.astype(np.float64) - mu.astype(np.float64)
        assert c1.max() <= top
        if delta == 0.0:
            assert np.all(c1 == 0)
            assert np.all(np.float32(x - mu) == np.float32(l))
            continue
        levels = np.float64(l) + np.float64(delta) * np.arange(top + 1)
        best = np.argmin(np.abs(t[:, None] - levels[None, :]), axis=1)
        # binary32 rounding of x - mu moves (t - l) / Delta by a few ulps of t
        tol = 4 * float(np.spacing(np.float32(np.abs(t).max() + abs(l)))) / delta + 2.0 ** -16
        amb = _half_tie((t - l) / delta, tol)
        assert np.all((best == c1) | amb)
        # Eq. 1 bounds are attained: the minimum component maps to 0, the
        # maximum to 2^B - 1
        assert c1[np.argmin(t)] == 0
        assert c1[np.argmax(t)] == top
        # |t - (l + Delta c)| <= Delta / 2 (residual range stated in Sec. 2.3)
        err = np.abs(t - (np.float64(l) + np.float64(delta) * c1))
        ulp = np.spacing(np.float32(np.maximum(np.abs(t).max(), np.float64(delta) * top)))
        assert np.all(err <= np.float64(delta) / 2 + 4 * ulp)


@pytest.mark.parametrize("bits", [2, 4, 8])
@pytest.mark.parametrize("kind", KINDS)
def test_first_level_matches_appendix_listing(bits, kind):
    """App. C evaluates level one as floor((x - l) * (1/Delta) + 0.5) clipped to
    [0, 2^B-1] in float32 arrays; numpy float32 evaluation of that formula gives
    the same codes for every vector with Delta > 0."""
    X, mu = _data(40 + bits, 64, 96, kind)
    Xc = (X - mu).astype(np.float32)
    u = Xc.max(1, keepdims=True)
    lo = Xc.min(1, keepdims=True)
    delta = ((u - lo) / np.float32(2 ** bits - 1)).astype(np.float32)
    ok = (delta[:, 0] >= np.finfo(np.float32).tiny)
    delta[~ok] = 1.0
    inv = (np.float32(1.0) / delta).astype(np.float32)
    codes = np.clip(np.floor(inv * (Xc - lo) + np.float32(0.5)), 0, 2 ** bits - 1)
    for i, x in enumerate(X):
        rc, l, dl, _, c1, _ = oracle.encode_codes(x, mu, bits)
        if ok[i]:
            assert dl == delta[i, 0] and l == lo[i, 0]
            np.testing.assert_array_equal(c1, codes[i].astype(np.uint8))
        else:
            assert dl == 0.0 and np.all(c1 == 0)


@pytest.mark.parametrize("b1,b2", [(4, 8), (4, 4), (8, 8), (2, 3), (8, 2)])
@pytest.mark.parametrize("kind", KINDS)
def test_residual_is_nearest_level(b1, b2, kind):
    """Residual level (Sec. 2.3, Def. 1): Q_{B2,-Delta/2,Delta/2}(r) with
    r = x - mu - Q(x): the code picks the nearest of the levels
    -Delta/2 + c Delta/(2^B2-1), and the two-level reconstruction error is
    at most half a residual step."""
    X, mu = _data(70 + b1 * 8 + b2, 24, 130, kind)
    top2 = 2 ** b2 - 1
    for x in X:
        rc, l, delta, delta2, c1, c2 = oracle.encode_codes(x, mu, b1, b2)
        assert rc == 0 and c2.max() <= top2
        if delta == 0.0:
            assert delta2 == 0.0 and np.all(c2 == 0)
            continue
        assert delta2 == np.float32(np.float32(delta) / np.float32(top2))
        t = x.astype(np.float64) - mu.astype(np.float64)
        y = np.float64(np.float32(np.float32(delta) * c1.astype(np.float32)) + np.float32(l))
        r = t - y
        levels = -np.float64(delta) / 2 + np.float64(delta2) * np.arange(top2 + 1)
        best = np.argmin(np.abs(r[:, None] - levels[None, :]), axis=1)
        tol = 8 * float(np.spacing(np.float32(np.abs(t).max() + abs(l)))) / delta2 + 2.0 ** -16
        amb = _half_tie((r + np.float64(delta) / 2) / np.float64(delta2), tol)
        assert np.all((best == c2) | amb)
        xh = np.float64(l) + np.float64(delta) * c1 - np.float64(delta) / 2 + np.float64(delta2) * c2
        scale = np.maximum(np.abs(t).max(), abs(l) + np.float64(delta) * 2 ** b1)
        assert np.all(np.abs(t - xh) <= np.float64(delta2) / 2 + 8 * np.spacing(np.float32(scale)))


def test_single_mean_is_lvq():
    """M = 1 reduces M-LVQ to LVQ (Sec. 3.2): identical rows."""
    X, mu = _data(5, 50, 96, "normal")
    fmt = oracle.Format(96, 4, 8, oracle.TURBO)
    r1, s1, _ = oracle.encode_rows(fmt, X, mu[None])
    r2, s2, _ = oracle.encode_rows(fmt, X, np.stack([mu, mu + 1000.0]))
    np.testing.assert_array_equal(r1, r2)
    np.testing.assert_array_equal(s1, s2)


@pytest.mark.parametrize("M", [2, 5, 16])
def test_assignment_is_nearest_mean(M):
    """Def. 1: mu_* = argmin_m ||x - mu_m||^2; checked against a binary64
    argmin (binary32 summation may flip only near-ties)."""
    g = synth.rng(77, M)
    X = g.standard_normal((200, 24)).astype(np.float32)
    means = g.standard_normal((M, 24)).astype(np.float32)
    for x in X:
        m = oracle.assign(x, means)
        s = ((x.astype(np.float64)[None] - means.astype(np.float64)) ** 2).sum(1)
        best = int(np.argmin(s))
        assert m == best or abs(s[m] - s[best]) <= 1e-5 * s[best]
    # ties go to the lowest index
    means2 = np.stack([means[0], means[0], means[1]])
    assert oracle.assign(means[0], means2) == 0


def test_mlvq_rows_use_the_assigned_mean():
    g = synth.rng(78, 0)
    means = (g.standard_normal((4, 32)) * 5).astype(np.float32)
    lab = g.integers(0, 4, 64)
    X = (means[lab] + 0.1 * g.standard_normal((64, 32))).astype(np.float32)
    fmt = oracle.Format(32, 8, 0)
    rows, _, rej = oracle.encode_rows(fmt, X, means)
    assert rej == 0
    l, delta, _, mid, c1, _ = oracle.unpack(fmt, rows)
    np.testing.assert_array_equal(mid, lab)
    for i in range(64):
        rc, l2, d2, _, cc, _ = oracle.encode_codes(X[i], means[lab[i]], 8)
        assert l2 == l[i] and d2 == delta[i]
        np.testing.assert_array_equal(cc, c1[i])


def _golden(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def _turbo_dim_to_place(dim):
    """The worked example read as a rule: within a 128-dim block, dimension j
    sits in word j mod 16, nibble j div 16."""
    b, r = divmod(dim, 128)
    return b, r % 16, r // 16


def test_turbo_worked_example(golden_dir):
    gold = _golden(golden_dir, "turbo_layout.json")
    for p in gold["placements"]:
        assert _turbo_dim_to_place(p["dim"])[1:] == (p["word"], p["nibble"])
    fmt = oracle.Format(128, 4, 0, oracle.TURBO)
    p2d = oracle.pos_to_dim(fmt)
    for p in gold["placements"]:
        pos = 8 * p["word"] + p["nibble"]
        assert p2d[pos] == p["dim"]
    # encode a vector whose codes equal the dimension index mod 16 and decode
    # the block the way the appendix describes (mask, then shift + mask)
    x = np.zeros(128, np.float32)
    x[:] = (np.arange(128) % 16).astype(np.float32)
    rows, _, _ = oracle.encode_rows(fmt, x[None], np.zeros((1, 128), np.float32))
    words = rows[0, 32:32 + 64].view("<u4")
    assert words.shape[0] == gold["words_per_block"]
    for grp in ("mask_group", "shift_group"):
        sh = gold[grp]["shift"]
        got = (words >> sh) & 0xF
        np.testing.assert_array_equal(got, np.array(gold[grp]["dims"]) % 16)


def test_turbo8_layout_from_the_lane_remark(golden_dir):
    """App. B: with 8-bit codes the sixteen lanes of a 64-byte block hold four
    dimensions each (tests/golden/turbo8_layout.json).  Rows spanning exactly
    0 .. 255 (mean 0) have Delta = 1 and codes equal to their coordinates, so
    the bytes of the block can be read against the placements directly."""
    gold = _golden(golden_dir, "turbo8_layout.json")
    d = 70                                          # a second block, partly filled
    g = np.random.default_rng(8000)
    x = g.integers(0, 256, d).astype(np.float32)
    x[0], x[1] = 0, 255
    fmt = oracle.Format(d, 8, 0, oracle.TURBO)
    rows, _, _ = oracle.encode_rows(fmt, x[None], np.zeros((1, d), np.float32))
    assert oracle.unpack(fmt, rows)[1][0] == 1.0
    code = rows[0, 32:]
    for p in gold["placements"]:
        if p["dim"] < d:
            assert code[4 * p["word"] + p["byte"]] == x[p["dim"]], p
    words = code[:gold["block_bytes"]].view("<u4")
    assert words.shape[0] == gold["words_per_block"]
    for grp in gold["groups"]:
        got = (words >> grp["shift"]) & 0xFF
        np.testing.assert_array_equal(got, x[grp["first_dim"]:grp["first_dim"] + 16].astype(np.uint32))
    # the second block holds dimensions 64 .. 69 in byte 0 of words 0 .. 5; the rest is zero
    blk = code[64:128].reshape(16, 4)
    np.testing.assert_array_equal(blk[:6, 0], x[64:70].astype(np.uint8))
    assert blk[6:, 0].sum() == 0 and blk[:, 1:].sum() == 0 and code[128:].sum() == 0


def test_eps1_hand_value():
    """Eq. 4 on rows whose codes are exact: Delta = (u - l) / 15 = 1 for 4-bit
    codes when the centred vector spans 0 .. 15.  Centred vector (0, 15,
    7.25, 3.5): codes 0, 15, 7, 4 (round half up: 3.5 -> 4), reconstruction
    (0, 15, 7, 4), squared error 0.25^2 + 0.5^2 = 0.3125.  Two such vectors,
    one encoded against mean (1, 1, 1, 1) and one against (40, 40, 40, 40)
    (their nearest means, Def. 1: squared distances 289.8 against over 4,000),
    give the sum 0.625 of Eq. 4; a per-vector mean would give 0.3125."""
    t = np.array([0.0, 15.0, 7.25, 3.5], np.float32)
    means = np.array([[1, 1, 1, 1], [40, 40, 40, 40]], np.float32)
    X = np.stack([t + 1.0, t + 40.0]).astype(np.float32)
    fmt = oracle.Format(4, 4, 0, oracle.SEQUENTIAL)
    rows, _, _ = oracle.encode_rows(fmt, X, means)
    l, delta, _, mid, c1, _ = oracle.unpack(fmt, rows)
    assert mid.tolist() == [0, 1] and (l == 0).all() and (delta == 1).all()
    assert c1.tolist() == [[0, 15, 7, 4], [0, 15, 7, 4]]
    assert oracle.eps1(fmt, X, rows, means) == 0.625
    assert oracle.eps1(fmt, X[:1], rows[:1], means) == 0.3125


@pytest.mark.parametrize("d", [1, 96, 130, 200, 768])
def test_turbo_and_sequential_hold_the_same_codes(d):
    """The permutation changes where codes live, not their values (Sec. 3.1);
    a partial last block is zero padded (App. B)."""
    X, mu = _data(9, 16, d, "normal")
    ft = oracle.Format(d, 4, 8, oracle.TURBO)
    fs = oracle.Format(d, 4, 8, oracle.SEQUENTIAL)
    rt, st, _ = oracle.encode_rows(ft, X, mu[None])
    rs, ss, _ = oracle.encode_rows(fs, X, mu[None])
    ut = oracle.unpack(ft, rt, st)
    us = oracle.unpack(fs, rs, ss)
    for a, b in zip(ut, us):
        np.testing.assert_array_equal(a, b)
    # independent decode of the Turbo rows with the worked-example rule
    for i in range(X.shape[0]):
        for j in range(d):
            b, w, k = _turbo_dim_to_place(j)
            word = rt[i, 32 + 64 * b + 4 * w: 32 + 64 * b + 4 * w + 4].view("<u4")[0]
            assert (word >> (4 * k)) & 0xF == ut[4][i, j]
            # residual byte 8w + k of the block's 128 bytes
            assert st[i, 128 * b + 8 * w + k] == ut[5][i, j]
    # zero padding past the last dimension, in codes and in the row tail
    used = set()
    for j in range(d):
        b, w, k = _turbo_dim_to_place(j)
        used.add((b, w, k))
    for b in range(ft.npos // 128):
        for w in range(16):
            for k in range(8):
                if (b, w, k) not in used:
                    word = rt[:, 32 + 64 * b + 4 * w: 32 + 64 * b + 4 * w + 4].copy().view("<u4")[:, 0]
                    assert np.all((word >> (4 * k)) & 0xF == 0)
                    assert np.all(st[:, 128 * b + 8 * w + k] == 0)
    assert np.all(rt[:, 32 + ft.code_bytes:] == 0)


def test_sequential_nibble_order():
    """Sequential 4-bit: dimension j in 32-bit word j div 8, nibble j mod 8."""
    fmt = oracle.Format(16, 4, 0, oracle.SEQUENTIAL)
    x = np.arange(16, dtype=np.float32) % 16
    rows, _, _ = oracle.encode_rows(fmt, x[None], np.zeros((1, 16), np.float32))
    words = rows[0, 32:40].view("<u4")
    for j in range(16):
        assert (words[j // 8] >> (4 * (j % 8))) & 0xF == j


def test_row_format_sizes():
    assert oracle.Format(96, 8).row_bytes == 128
    f = oracle.Format(768, 4, 8, oracle.TURBO)
    assert (f.row_bytes, f.resid_bytes, f.code_bytes) == (416, 768, 384)
    assert oracle.Format(512, 8).row_bytes == 544
    assert oracle.Format(768, 4, 8, oracle.TURBO, 128).row_bytes == 512
    for d in (1, 7, 96, 130, 768, 1000):
        for b1 in (4, 8):
            for lay in (0, 1):
                f = oracle.Format(d, b1, 8, lay)
                assert f.row_bytes % 32 == 0 and f.row_bytes >= 32 + (d * b1 + 7) // 8


def test_footprint_numbers(golden_dir):
    """Sec. 3.3 arithmetic on the per-dimension code widths."""
    g = _golden(golden_dir, "footprint.json")
    a = g["lvq8x2_vs_fp16"]
    saved = (a["fp16_bits"] - a["bits1"] - a["bits2"]) * a["dim"] * a["n"] / 8
    assert int(saved / 2 ** 30) == a["saving_gib_floor"]
    b = g["half_bit_m_lvq"]
    assert b["dim"] * b["bits"] / 8 == b["total_bytes"]
    assert b["dim"] * 0.5 / 8 == b["saving_bytes"]
    # the format's code bytes reproduce the widths (B1 + B2 bits per dim)
    f = oracle.Format(512, 8, 8)
    assert f.code_bytes == 512 and f.resid_bytes == 512
    f = oracle.Format(512, 4, 4, oracle.TURBO)
    assert f.code_bytes + f.resid_bytes == 512


def test_nonfinite_rejected():
    X, mu = _data(3, 4, 16, "normal")
    X[1, 3] = np.nan
    X[2, 0] = np.inf
    fmt = oracle.Format(16, 8, 8)
    rows, resid, rej = oracle.encode_rows(fmt, X, mu[None])
    assert rej == 2
    for i in (1, 2):
        assert np.isnan(rows[i, :4].view(np.float32)[0])
        assert np.all(rows[i, 4:] == 0) and np.all(resid[i] == 0)
    assert not np.isnan(rows[0, :4].view(np.float32)[0])


def test_constant_vector():
    """u == l: Delta is stored as 0, all codes 0, reconstruction exactly mu + l."""
    mu = (np.arange(20) / 8.0 - 1.0).astype(np.float32)
    x = (mu + np.float32(0.5)).astype(np.float32)
    fmt = oracle.Format(20, 4, 8)
    rows, resid, _ = oracle.encode_rows(fmt, x[None], mu[None])
    l, delta, delta2, _, c1, c2 = oracle.unpack(fmt, rows, resid)
    assert delta[0] == 0 and delta2[0] == 0 and np.all(c1 == 0) and np.all(c2 == 0)
    xh = oracle.reconstruct(fmt, rows, resid, mu[None], oracle.FULL)
    np.testing.assert_array_equal(xh[0], mu.astype(np.float64) + np.float64(l[0]))


def test_eps1_decreases_with_bits_and_means():
    """Eq. 4 sanity: more bits or more (k-means-like) means lower eps1."""
    w = synth.WORKLOADS["C1"]
    cent = synth.centres(101, 8, 32)
    X = synth.mixture(101, synth.S_BASE, 0, 400, cent, 0.3)
    mu = X.astype(np.float64).mean(0).astype(np.float32)
    prev = np.inf
    for b in range(2, 9):
        e = 0.0
        for x in X:
            _, l, dl, _, c1, _ = oracle.encode_codes(x, mu, b)
            e += ((x.astype(np.float64) - mu - (l + np.float64(dl) * c1)) ** 2).sum()
        assert e < prev
        prev = e
    fmt = oracle.Format(32, 4)
    r1, _, _ = oracle.encode_rows(fmt, X, mu[None])
    r8, _, _ = oracle.encode_rows(fmt, X, cent)
    assert oracle.eps1(fmt, X, r8, cent) < oracle.eps1(fmt, X, r1, mu[None])
    assert w["dim"] == 96


@pytest.mark.parametrize("b1,b2", [(4, 8), (8, 8), (8, 4)])
def test_far_from_mean_residual_clamps(b1, b2):
    """A vector far from the mean with a tiny spread: binary32 rounding of the
    level-one reconstruction l + Delta c1 exceeds Delta/2, so the residual
    falls outside [-Delta/2, Delta/2] and both clamps of Q_{B2} are reached;
    codes stay in range and still pick the nearest residual level."""
    g = synth.rng(79, b1 * 16 + b2)
    # spread chosen so that Delta is about 1.5 binary32 ulps of the values
    s = 0.9 * (2 ** b1 - 1) * float(np.spacing(np.float32(1000.0)))
    x = (1000.0 + s * g.uniform(-1, 1, 256)).astype(np.float32)
    mu = np.zeros(256, np.float32)
    rc, l, delta, delta2, c1, c2 = oracle.encode_codes(x, mu, b1, b2)
    top2 = 2 ** b2 - 1
    assert rc == 0 and c2.max() <= top2
    assert (c2 == 0).any() and (c2 == top2).any()
    t = x.astype(np.float64)
    y = (np.float32(delta) * c1.astype(np.float32) + np.float32(l)).astype(np.float64)
    r = t - y
    levels = -np.float64(delta) / 2 + np.float64(delta2) * np.arange(top2 + 1)
    best = np.argmin(np.abs(r[:, None] - levels[None, :]), axis=1)
    # r = 0 sits exactly between two residual levels when 2^B2 is even
    amb = _half_tie((r + np.float64(delta) / 2) / np.float64(delta2), 2.0 ** -12)
    assert np.all((best == c2) | amb)
    assert (~amb).sum() > 100

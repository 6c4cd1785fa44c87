"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds random-number generation only (no LVQ arithmetic).  Every
stream is chunk-addressable: rows are generated in chunks of CHUNK vectors, each
chunk from its own PCG64 generator seeded with
``SeedSequence([SEED, workload, stream, chunk])``, so any slice of any input can
be regenerated exactly without materialising the rest.

Workloads (shapes and value laws stand in for the paper's datasets: d in
{96, 512, 768}, 10^4 queries, inner product for the 512/768-d sets and
Euclidean for the 96-d set):

* ``C1``: 32 Gaussian clusters in 96-d (centres N(0, I), spread 0.3),
  10,000 base vectors, 100 queries from the same mixture.
* ``C2``: anisotropic Gaussian in 768-d (component j scaled by 1/sqrt(j+1)),
  unit normalised; 10^6 base vectors, 10^4 queries, 1,000 distinct uniform
  candidate ids per query.
* ``C3``: 256 Gaussian clusters in 96-d (spread 0.3); 10^7 base vectors,
  10^4 queries, candidate list lengths floor(exp(U(ln 64, ln 4097))).
* ``C4``: the C2 law in 512-d; 5 * 10^6 base vectors, 10^4 queries.
* ``C5``: 64 clusters in 768-d, unit normalised; centres drift each round.
* ``G1``: the C2 law in 96-d (low intrinsic dimension, like the 96-d set the
  paper searches with a graph); 10^6 base vectors, 10^4 queries, Euclidean.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

SEED = 20240203
CHUNK = 65536

# stream ids
S_CENTRES, S_BASE, S_QUERY, S_LISTS, S_SAMPLE, S_DRIFT, S_INSERT, S_DELETE, S_ARRIVAL = range(9)

WORKLOADS = {
    "C1": dict(id=1, dim=96, n=10_000, nq=100, clusters=32, spread=0.3, law="mixture"),
    "C2": dict(id=2, dim=768, n=1_000_000, nq=10_000, list_len=1000, law="aniso"),
    "C3": dict(id=3, dim=96, n=10_000_000, nq=10_000, clusters=256, spread=0.3, law="mixture",
               list_min=64, list_max=4096),
    "C4": dict(id=4, dim=512, n=5_000_000, nq=10_000, law="aniso"),
    "C5": dict(id=5, dim=768, n=1_000_000, nq=10_000, clusters=64, spread=0.3, law="mixture_unit"),
    "G1": dict(id=6, dim=96, n=1_000_000, nq=10_000, law="aniso"),
}


def rng(workload: int, stream: int, chunk: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED, workload, stream, chunk])))


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(fill, start: int, count: int, dim: int) -> np.ndarray:
    """Assemble rows [start, start+count) from per-chunk generators."""
    out = np.empty((count, dim), np.float32)
    c0, c1 = start // CHUNK, (start + count - 1) // CHUNK if count else start // CHUNK - 1

    def one(c):
        block = fill(c)
        a = max(start, c * CHUNK)
        b = min(start + count, (c + 1) * CHUNK)
        out[a - start:b - start] = block[a - c * CHUNK:b - c * CHUNK]

    chunks = list(range(c0, c1 + 1))
    if len(chunks) > 1:
        with ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(one, chunks))
    else:
        for c in chunks:
            one(c)
    return out


def centres(workload: int, k: int, dim: int) -> np.ndarray:
    return rng(workload, S_CENTRES).standard_normal((k, dim), dtype=np.float32)


def mixture(workload: int, stream: int, start: int, count: int, cent: np.ndarray, spread: float,
            unit: bool = False) -> np.ndarray:
    """centre[U{0..K-1}] + spread * N(0, I), optionally unit normalised."""
    k, dim = cent.shape

    def fill(c):
        g = rng(workload, stream, c)
        lab = g.integers(0, k, CHUNK)
        x = g.standard_normal((CHUNK, dim), dtype=np.float32)
        x *= np.float32(spread)
        x += cent[lab]
        if unit:
            x /= np.linalg.norm(x, axis=1, keepdims=True)
        return x

    return _chunked(fill, start, count, dim)


def anisotropic(workload: int, stream: int, start: int, count: int, dim: int) -> np.ndarray:
    """x_j = g_j / sqrt(j + 1), g ~ N(0, 1), then unit normalised."""
    scale = (1.0 / np.sqrt(np.arange(1, dim + 1, dtype=np.float64))).astype(np.float32)

    def fill(c):
        x = rng(workload, stream, c).standard_normal((CHUNK, dim), dtype=np.float32)
        x *= scale
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        return x

    return _chunked(fill, start, count, dim)


def vectors(name: str, stream: int, start: int, count: int) -> np.ndarray:
    """Base (stream S_BASE) or query (S_QUERY) vectors of a named workload."""
    w = WORKLOADS[name]
    if w["law"] == "aniso":
        return anisotropic(w["id"], stream, start, count, w["dim"])
    cent = centres(w["id"], w["clusters"], w["dim"])
    return mixture(w["id"], stream, start, count, cent, w["spread"], unit=w["law"] == "mixture_unit")


def candidate_lists(workload: int, nq: int, n: int, length=None, lmin=None, lmax=None,
                    q_chunk: int = 256):
    """Per-query lists of distinct uniform slot ids in [0, n).

    Fixed ``length``, or log-uniform lengths floor(exp(U(ln lmin, ln lmax+1))).
    Returns CSR ``offsets`` (nq+1, int64) and ``ids`` (int32)."""
    lens = np.empty(nq, np.int64)
    lists = [None] * nq

    def one(c):
        g = rng(workload, S_LISTS, c)
        for i in range(c * q_chunk, min(nq, (c + 1) * q_chunk)):
            if length is not None:
                L = int(length)
            else:
                L = int(np.floor(np.exp(g.uniform(np.log(lmin), np.log(lmax + 1)))))
                L = min(max(L, lmin), lmax)
            L = min(L, n)
            lists[i] = g.choice(n, L, replace=False).astype(np.int32)
            lens[i] = L

    nchunks = (nq + q_chunk - 1) // q_chunk
    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(one, range(nchunks)))
    offsets = np.zeros(nq + 1, np.int64)
    np.cumsum(lens, out=offsets[1:])
    ids = np.concatenate(lists) if nq else np.zeros(0, np.int32)
    return offsets, ids


def sample_indices(workload: int, n: int, count: int) -> np.ndarray:
    """`count` distinct uniform indices in [0, n), sorted."""
    return np.sort(rng(workload, S_SAMPLE).choice(n, min(count, n), replace=False))


def drift_directions(workload: int, k: int, dim: int) -> np.ndarray:
    """One fixed random unit direction per cluster for centre drift."""
    v = rng(workload, S_DRIFT).standard_normal((k, dim)).astype(np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v.astype(np.float32)


C5_DRIFT_PER_COORD = 0.05   # centre displacement per round, RMS per coordinate


def c5_centres(round_: int) -> np.ndarray:
    """C5 cluster centres after `round_` rounds of drift: each centre moves
    C5_DRIFT_PER_COORD * sqrt(d) per round along its own fixed unit direction."""
    w = WORKLOADS["C5"]
    cent = centres(w["id"], w["clusters"], w["dim"])
    step = np.float32(C5_DRIFT_PER_COORD * np.sqrt(w["dim"]))
    return (cent + np.float32(round_) * step * drift_directions(w["id"], w["clusters"], w["dim"])).astype(np.float32)


def c5_points(stream: int, round_: int, count: int, part: int = 0) -> np.ndarray:
    """`count` C5 vectors from the round's (drifted) mixture: a uniform centre
    plus spread * N(0, I), unit normalised.  One generator per (stream, round,
    part), so rounds are independent of each other and of the base store."""
    w = WORKLOADS["C5"]
    cent = c5_centres(round_)
    g = rng(w["id"], stream, 1 + round_ * 64 + part)
    lab = g.integers(0, w["clusters"], count)
    x = g.standard_normal((count, w["dim"]), dtype=np.float32)
    x *= np.float32(w["spread"])
    x += cent[lab]
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x


def small_vectors(seed: int, n: int, dim: int, kind: str = "normal") -> np.ndarray:
    """Small seeded test inputs of a few distributions (tests only)."""
    g = rng(900 + seed, 0)
    if kind == "normal":
        return g.standard_normal((n, dim), dtype=np.float32)
    if kind == "uniform":
        return g.uniform(-1, 1, (n, dim)).astype(np.float32)
    if kind == "wide":     # magnitudes spanning many binades
        return (g.standard_normal((n, dim)) * np.exp2(g.integers(-20, 20, (n, 1)))).astype(np.float32)
    if kind == "lowcard":  # few distinct values: exact ties and u == l rows
        return g.integers(-2, 3, (n, dim)).astype(np.float32) * np.float32(0.25)
    raise ValueError(kind)

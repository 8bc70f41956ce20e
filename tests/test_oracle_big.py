"""Pins of the oracle on universes of 2^53 slots and more (Sec. 1: the
paper's headline instance has far more slots than binary64 counts exactly),
where slot counts reach the variates rounded to nearest: the hypergeometric
and binomial variates at N near 2^60 against their exact means and variances
(every branch: direct simulation, ratio of uniforms, waiting times), the
whole generator's invariants and its communication-free recomputation on a
directed universe of about 2^54 slots, and the limits agreeing between the
oracle's and the library's argument checks."""
import ctypes
import math
import os

import numpy as np
import pytest

from oracle import kgref

S = 6000          # variates per moment check


def _moments(xs):
    xs = np.asarray(xs, dtype=np.float64)
    return xs.mean(), xs.var(ddof=1)


def _check(xs, mu, var):
    m, v = _moments(xs)
    n = len(xs)
    assert abs(m - mu) < 5 * math.sqrt(var / n), (m, mu)
    # the sample variance has standard error about var sqrt(2 / n)
    assert abs(v - var) < 5 * var * math.sqrt(2.0 / n) + 1e-9, (v, var)


@pytest.mark.parametrize("N,K,k", [(2**60 + 12345, (2**60 + 12345) // 3, 10**6),      # ratio of uniforms
                                   (2**62 - 7, 2**61, 2**20 + 3),                         # near-even split
                                   (2**59 + 1, 2**40, 10**5),                             # rare marks
                                   (2**61 + 5, 2**58, 12)])                               # direct simulation
def test_hypergeometric_moments_beyond_2_53(N, K, k):
    xs = [kgref.hyp(N, K, k, seed=s, a=7, b=1) for s in range(S)]
    assert all(0 <= x <= min(k, K) for x in xs)
    q = K / N
    mu = k * q
    var = k * q * (1 - q) * (N - k) / (N - 1)
    _check(xs, mu, var)


@pytest.mark.parametrize("N,mean", [(2**60 + 3, 1.0e6), (2**62 + 11, 5.0e4), (2**59 + 1, 9.0)])
def test_binomial_moments_beyond_2_53(N, mean):
    p = mean / N
    xs = [kgref.bin(N, p, seed=s, a=3) for s in range(S)]
    _check(xs, N * p, N * p * (1 - p))


def test_binomial_stays_in_range_near_the_top():
    """p close to 1 at N near 2^60: every variate lies in [0, N] (the
    proposal range check is made on the integer, not on its rounding)."""
    N = 2**60 + 3
    for s in range(200):
        x = kgref.bin(N, 1.0 - 2.0**-40, seed=s)
        assert 0 <= x <= N
        assert N - x < 2**24


# a directed universe above 2^53: n = 2^27 + 9, about 2^54 slots
BIG = dict(n=2**27 + 9, m=2**31 + 77, directed=True, seed=5, chunks=2**10)


def test_generator_invariants_beyond_2_53():
    I = kgref.inst(**BIG)
    n = BIG["n"]
    assert n * (n - 1) >= 2**53
    assert kgref.validate(I) == 0
    assert kgref.tile_exponent(I) == 32
    counts = kgref.chunk_counts(I)
    assert int(counts.sum()) == BIG["m"]
    rng = np.random.default_rng(1)
    P = BIG["chunks"]
    for c in [0, 1, P // 2, P - 1] + list(rng.integers(0, P, 4)):
        c = int(c)
        # the communication-free count: the chunk's root path alone
        assert kgref.chunk_count_path(I, c) == int(counts[c])
        E = kgref.chunk_edges(I, c, int(counts[c]))
        assert len(E) == int(counts[c])
        u, v = E[:, 0].astype(np.int64), E[:, 1].astype(np.int64)
        r0, r1 = c * n // P, (c + 1) * n // P
        assert np.all((u >= r0) & (u < r1) & (v < n) & (u != v))
        slot = u * (n - 1) + v - (v > u)
        assert np.all(slot[1:] > slot[:-1])           # ascending slots, no repeats


def test_chunk_counts_are_hypergeometric_beyond_2_53():
    """Chunk 0's count over seeds: Hyp(N, N_0, m) with N_0 = rows(0) (n - 1)."""
    n, m, P = 2**27 + 9, 2**20, 8
    N = n * (n - 1)
    N0 = (n // P) * (n - 1)
    xs = []
    for s in range(1500):
        I = kgref.inst(n, m=m, directed=True, seed=s, chunks=P)
        xs.append(kgref.chunk_count_path(I, 0))
    q = N0 / N
    mu, var = m * q, m * q * (1 - q) * (N - m) / (N - 1)
    m_, v_ = _moments(xs)
    assert abs(m_ - mu) < 5 * math.sqrt(var / len(xs))
    assert abs(v_ - var) < 5 * var * math.sqrt(2.0 / len(xs))


def _lib():
    from paper_1710_07565_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1710_07565_amd import build
        build.build(force=True)
    return _lib


@pytest.mark.parametrize("kw", [
    dict(n=2**27, m=2**31, chunks=2**10), dict(n=2**27, m=2**53, chunks=2**10),
    dict(n=2**27, m=2**53 - 1, chunks=2**16), dict(n=2**32, m=0, chunks=1), dict(n=2**32, m=2**40, chunks=2**8),
    dict(n=2**32, directed=False, m=2**40, chunks=2**8), dict(n=2**32, directed=False, m=0, chunks=1),
    dict(n=2**28, directed=False, p=32.0 / (2**28 - 1), chunks=256),
    dict(n=2**27, p=2.0**52 / (2**27 * (2**27 - 1)), chunks=2**10),
    dict(n=2**26, m=2**31, directed=False, chunks=256), dict(n=94906267, m=0, chunks=4)])
def test_limits_agree_with_the_library(kw):
    L = _lib()
    d = dict(directed=True, seed=1, m=0, p=0.0)
    d.update(kw)
    model = 1 if d["p"] else 0
    I = kgref.inst(d["n"], m=d["m"], p=d["p"], directed=d["directed"], seed=1, chunks=d["chunks"], model=model)
    K = L.KgInstance(d["n"], model, int(d["directed"]), d["m"], d["p"], 1, d["chunks"], 0)
    out = ctypes.c_uint64(0)
    st = L.lib().kg_workspace_bytes(ctypes.byref(K), 1, ctypes.byref(out))
    assert (kgref.validate(I) == 0) == (st == 0), (kw, kgref.validate(I), st)

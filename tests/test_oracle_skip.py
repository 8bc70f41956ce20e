"""Pins of the geometric-skip G(n,p) variant of the oracle (every slot an
independent Bernoulli(p) trial, Sec. 2.1.1 / 4.3, sampled by waiting times
per tile instead of a binomial count and a sample): brute force over every
graph on 6 slots (both the success and the failure form of the waiting
times), binomial tile and chunk counts, the same degree law as the main
path's G(n,p), and the invariants of the output."""
from itertools import product

import numpy as np
import pytest
from scipy import stats


def slot_bits(E, n, directed):
    # index of (u, v) among the instance's slots, as a bitmask per graph
    if directed:
        return [(u * (n - 1) + v - (v > u)) for u, v in E.tolist()]
    return [sum(n - 1 - r for r in range(u)) + (v - u - 1) for u, v in E.tolist()]


@pytest.mark.parametrize("p", [0.3, 0.7])
def test_every_graph_on_six_slots(kgref, p):
    """Directed n = 3 has 6 slots: each of the 64 graphs must appear with
    probability p^e (1 - p)^(6 - e) (chi-square over 6,000 seeds)."""
    n, trials = 3, 6000
    hist = np.zeros(64, dtype=np.int64)
    for seed in range(trials):
        E = kgref.skip_generate(kgref.inst(n, p=p, directed=True, seed=seed + 1, chunks=1, model=kgref.GNP))
        mask = 0
        for b in slot_bits(E, n, True):
            mask |= 1 << b
        hist[mask] += 1
    prob = np.array([p ** bin(g).count("1") * (1 - p) ** (6 - bin(g).count("1")) for g in range(64)])
    chi2 = ((hist - trials * prob) ** 2 / (trials * prob)).sum()
    assert stats.chi2.sf(chi2, 63) > 1e-4


def test_chunk_counts_are_binomial(kgref):
    """Edges of one chunk over 3,000 seeds: Binomial(N_c, p) by chi-square on
    binned counts (several tiles per chunk, a ragged last tile)."""
    n, p, P = 300, 0.02, 3
    I0 = kgref.inst(n, p=p, directed=True, seed=1, chunks=P, model=kgref.GNP)
    Nc = 100 * (n - 1)          # rows 0..99 of 300 (floor(n/P) per chunk)
    counts = np.array([len(kgref.skip_chunk_edges(kgref.inst(n, p=p, directed=True, seed=s, chunks=P,
                                                              model=kgref.GNP), 0)) for s in range(1, 3001)])
    rv = stats.binom(Nc, p)
    edges = np.arange(rv.ppf(0.001), rv.ppf(0.999) + 2, 8)
    obs, _ = np.histogram(counts, bins=edges)
    exp = np.diff(rv.cdf(edges - 1)) * len(counts)
    keep = exp > 5
    chi2 = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4
    assert abs(counts.mean() - Nc * p) < 4 * np.sqrt(Nc * p * (1 - p) / len(counts))
    del I0


@pytest.mark.parametrize("directed", [True, False])
def test_same_degree_law_as_main_path(kgref, directed):
    """Out-degrees (directed) / degrees (undirected) of the skip variant and
    of the main path's G(n,p) over 40 seeds: same distribution (two-sample
    chi-square on pooled bins)."""
    n, P = 400, 5
    p = 12.0 / (n - 1)
    da, db = [], []
    for s in range(1, 41):
        I = kgref.inst(n, p=p, directed=directed, seed=s, chunks=P, model=kgref.GNP)
        for E, acc in ((kgref.skip_generate(I), da), (kgref.generate(I), db)):
            deg = np.bincount(E[:, 0], minlength=n)
            if not directed:
                deg = deg + np.bincount(E[:, 1], minlength=n)
            acc.append(deg)
    da, db = np.concatenate(da), np.concatenate(db)
    hi = int(max(da.max(), db.max())) + 1
    ha, hb = np.bincount(da, minlength=hi), np.bincount(db, minlength=hi)
    keep = (ha + hb) > 10
    chi2, pval, _, _ = stats.chi2_contingency(np.vstack([ha[keep], hb[keep]]))
    assert pval > 1e-4


@pytest.mark.parametrize("n,p,directed,P", [(200, 0.05, False, 4), (120, 0.6, True, 7), (90, 0.0, False, 3),
                                            (50, 1.0, True, 2), (50, 1.0, False, 5), (1000, 0.001, True, 10)])
def test_invariants(kgref, n, p, directed, P):
    I = kgref.inst(n, p=p, directed=directed, seed=7, chunks=P, model=kgref.GNP)
    E = kgref.skip_generate(I)
    N = n * (n - 1) // (1 if directed else 2)
    if p == 0.0:
        assert len(E) == 0
    if p == 1.0:
        assert len(E) == N
    assert np.all(E[:, 0] != E[:, 1]) and np.all(E < n)
    if not directed:
        assert np.all(E[:, 0] < E[:, 1])
    # canonical order: chunk by chunk, each chunk strictly ascending, and the
    # concatenation of the per-chunk lists
    parts = [kgref.skip_chunk_edges(I, c) for c in range(kgref.num_chunks(I))]
    assert np.array_equal(np.concatenate(parts) if len(E) else E.reshape(0, 2), E)
    for c, Ec in enumerate(parts):
        k = Ec[:, 0].astype(np.int64) * n + Ec[:, 1]
        assert np.all(np.diff(k) > 0), c

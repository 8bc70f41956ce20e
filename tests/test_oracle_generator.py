"""Whole-generator pins of the oracle.

* G(n,m) is uniform over all simple graphs with m edges (Sec. 2.1.1): brute
  force over every edge set of tiny instances.
* G(n,p) includes each slot independently with probability p (Sec. 2.1.1).
* Invariants: m edges, no self-loops, no repeats, u < v when undirected,
  canonical order.
* The communication-free property (Sec. 2.2, 4.1, 4.2): a chunk's count
  from its own root path equals the count of the whole-tree expansion.
* Marginal laws: chunk counts are hypergeometric (G(n,m), Sec. 2.2) or
  binomial (G(n,p), Sec. 4.3); degrees follow the matching laws.
"""
import math
from itertools import combinations

import numpy as np
import pytest
from scipy import stats


def edge_key(E, n):
    return E[:, 0].astype(np.int64) * n + E[:, 1].astype(np.int64)


def check_invariants(kgref, I, E):
    n = I.n
    assert E.dtype == np.uint32
    assert np.all(E[:, 0] != E[:, 1])
    assert np.all(E < n)
    keys = edge_key(E, n)
    assert len(np.unique(keys)) == len(keys)
    if not I.directed:
        assert np.all(E[:, 0] < E[:, 1])
    if I.model == kgref.GNM:
        assert len(E) == I.m
    # canonical order: chunks in order, ascending local index inside a chunk
    counts = kgref.chunk_counts(I)
    assert counts.sum() == len(E)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    if I.directed:
        assert np.all(np.diff(keys) > 0)      # global slot order = (u, v) lexicographic
    else:
        for c in range(len(counts)):
            seg = keys[off[c]:off[c + 1]]
            assert np.all(np.diff(seg) > 0)
    return counts


def _all_edge_sets(n, m, directed):
    slots = [(u, v) for u in range(n) for v in range(n) if u != v and (directed or u < v)]
    return {tuple(c): i for i, c in enumerate(combinations(slots, m))}


@pytest.mark.parametrize("directed,P", [(True, 1), (True, 2), (True, 3), (True, 4),
                                         (False, 1), (False, 2), (False, 3), (False, 4)])
def test_gnm_uniform_over_edge_sets_n4(kgref, directed, P):
    """n=4, m=3: each of the C(12,3)=220 directed (C(6,3)=20 undirected) edge
    sets appears equally often across seeds."""
    sets = _all_edge_sets(4, 3, directed)
    per = 150 if directed else 600
    counts = np.zeros(len(sets), dtype=np.int64)
    for seed in range(1, per * len(sets) + 1):
        E = kgref.generate(kgref.inst(4, m=3, directed=directed, seed=seed, chunks=P))
        assert len(E) == 3
        tup = tuple(sorted((int(u), int(v)) for u, v in E))
        counts[sets[tup]] += 1
    assert stats.chisquare(counts).pvalue > 1e-5


@pytest.mark.parametrize("directed", [True, False])
def test_gnm_every_m_small(kgref, directed):
    n = 5
    N = n * (n - 1) // (1 if directed else 2)
    for P in [1, 2, 5]:
        for m in range(N + 1):
            I = kgref.inst(n, m=m, directed=directed, seed=m + 17 * P, chunks=P)
            check_invariants(kgref, I, kgref.generate(I))


@pytest.mark.parametrize("directed,n", [(True, 3), (False, 4)])
def test_gnp_graph_probabilities(kgref, directed, n):
    """Each of the 2^6 graphs on 6 slots has probability p^e (1-p)^(6-e)."""
    p = 0.3
    slots = [(u, v) for u in range(n) for v in range(n) if u != v and (directed or u < v)]
    assert len(slots) == 6
    idx = {s: i for i, s in enumerate(slots)}
    reps = 30000
    counts = np.zeros(64, dtype=np.int64)
    for seed in range(reps):
        E = kgref.generate(kgref.inst(n, p=p, directed=directed, seed=seed, chunks=2))
        mask = 0
        for u, v in E:
            mask |= 1 << idx[(int(u), int(v))]
        counts[mask] += 1
    probs = np.array([p ** bin(g).count("1") * (1 - p) ** (6 - bin(g).count("1")) for g in range(64)])
    assert stats.chisquare(counts, probs * reps).pvalue > 1e-5


def test_config_small_directed_invariants(kgref):
    # directed G(n,m), n=2^16, m=2^20, 64 chunks, seed 1
    I = kgref.inst(2**16, m=2**20, directed=True, seed=1, chunks=64)
    assert kgref.tile_exponent(I) == 22
    E = kgref.generate(I)
    check_invariants(kgref, I, E)


@pytest.mark.parametrize("n,m,P,seed", [(2**12, 2**16, 8, 1), (1000, 30000, 7, 2), (3000, 10**5, 33, 3),
                                         (50, 1225, 4, 4), (50, 1000, 50, 5)])
def test_undirected_invariants(kgref, n, m, P, seed):
    I = kgref.inst(n, m=m, directed=False, seed=seed, chunks=P)
    check_invariants(kgref, I, kgref.generate(I))


@pytest.mark.parametrize("n,p,directed,P", [(2**12, 16 / (2**12 - 1), True, 64), (3000, 0.01, False, 16),
                                             (200, 0.6, True, 3), (300, 0.97, False, 5)])
def test_gnp_invariants(kgref, n, p, directed, P):
    I = kgref.inst(n, p=p, directed=directed, seed=9, chunks=P)
    check_invariants(kgref, I, kgref.generate(I))


@pytest.mark.parametrize("n,directed,P,model", [
    (2**16, True, 64, 0), (1000, True, 37, 0), (2**20, True, 1000, 0),
    (2**12, False, 8, 0), (1000, False, 13, 0), (2**16, False, 100, 0),
    (2**14, True, 77, 1), (2**14, False, 21, 1)])
def test_communication_free_chunk_counts(kgref, n, directed, P, model):
    """Every chunk finds its count alone, on its root-to-leaf path, and the
    result equals the whole-tree expansion (Sec. 2.2, 4.1, 4.2)."""
    N = n * (n - 1) // (1 if directed else 2)
    if model == 0:
        I = kgref.inst(n, m=N // 1000 + 7, directed=directed, seed=5, chunks=P, model=0)
    else:
        I = kgref.inst(n, p=0.001, directed=directed, seed=5, chunks=P, model=1)
    counts = kgref.chunk_counts(I)
    if model == 0:
        assert counts.sum() == I.m
    for c in range(len(counts)):
        assert kgref.chunk_count_path(I, c) == counts[c]


def test_quadtree_size_formula():
    """Sec. 4.2: for P a power of two the full quadrant tree over the P x P
    chunk matrix has (4P^2 - 1)/3 nodes; our recursion visits the non-empty
    ones, N(P) = 2 N(P/2) + R(P/2) + 1 with R(q) = (4 q^2 - 1)/3."""
    def rect_nodes(q):   # full quadtree of a q x q rectangle
        return 1 if q == 1 else 1 + 4 * rect_nodes(q // 2)

    def tri_nodes(P):
        return 1 if P == 1 else 1 + 2 * tri_nodes(P // 2) + rect_nodes(P // 2)
    for k in range(0, 9):
        P = 2**k
        assert rect_nodes(P) == (4 * P * P - 1) // 3
        if P > 1:
            assert tri_nodes(P) == 2 * tri_nodes(P // 2) + (P * P - 1) // 3 + 1


@pytest.mark.parametrize("directed", [True, False])
def test_chunk_count_marginal_hypergeometric(kgref, directed):
    n, P = 64, 5
    N = n * (n - 1) // (1 if directed else 2)
    m = 300
    reps = 4000
    C = P if directed else P * (P + 1) // 2
    samples = np.zeros((reps, C), dtype=np.int64)
    for s in range(reps):
        samples[s] = kgref.chunk_counts(kgref.inst(n, m=m, directed=directed, seed=1000 + s, chunks=P))
    assert np.all(samples.sum(axis=1) == m)
    bounds = [c * n // P for c in range(P + 1)]
    if directed:
        sizes = [(bounds[c + 1] - bounds[c]) * (n - 1) for c in range(C)]
    else:
        sizes = []
        for i in range(P):
            for j in range(i, P):
                hi, hj = bounds[i + 1] - bounds[i], bounds[j + 1] - bounds[j]
                sizes.append(hi * (hi - 1) // 2 if i == j else hi * hj)
    assert sum(sizes) == N
    for c in [0, C // 2, C - 1]:
        rv = stats.hypergeom(N, sizes[c], m)
        lo, hi = int(rv.ppf(1e-6)), int(rv.ppf(1 - 1e-6))
        x = np.clip(samples[:, c], lo, hi)
        obs = np.bincount(x - lo, minlength=hi - lo + 1)
        exp = np.array([rv.pmf(v) for v in range(lo, hi + 1)])
        exp[0] += rv.cdf(lo - 1)
        exp[-1] += rv.sf(hi)
        keep = exp * reps >= 5
        o = np.concatenate([obs[keep], [obs[~keep].sum()]])
        e = np.concatenate([exp[keep], [exp[~keep].sum()]]) * reps
        if e[-1] == 0:
            o, e = o[:-1], e[:-1]
        e *= o.sum() / e.sum()
        assert stats.chisquare(o, e).pvalue > 1e-5
    # covariance of two chunk counts: -m (N-m) Ni Nj / (N^2 (N-1))
    i, j = 0, C - 1
    cov = np.cov(samples[:, i], samples[:, j])[0, 1]
    want = -m * (N - m) * sizes[i] * sizes[j] / (N * N * (N - 1))
    var_i = m * sizes[i] / N * (1 - sizes[i] / N) * (N - m) / (N - 1)
    var_j = m * sizes[j] / N * (1 - sizes[j] / N) * (N - m) / (N - 1)
    assert abs(cov - want) < 5 * math.sqrt(var_i * var_j / reps) + 1e-9


def _degree_chi2(deg, rv, nbins_min=5):
    lo, hi = int(rv.ppf(1e-7)), int(rv.ppf(1 - 1e-7))
    x = np.clip(deg, lo, hi)
    obs = np.bincount(x - lo, minlength=hi - lo + 1).astype(np.float64)
    exp = np.array([rv.pmf(v) for v in range(lo, hi + 1)]) * len(deg)
    exp[0] += rv.cdf(lo - 1) * len(deg)
    exp[-1] += rv.sf(hi) * len(deg)
    keep = exp >= nbins_min
    o = np.concatenate([obs[keep], [obs[~keep].sum()]])
    e = np.concatenate([exp[keep], [exp[~keep].sum()]])
    if e[-1] < 1e-9:
        o, e = o[:-1], e[:-1]
    e *= o.sum() / e.sum()
    return stats.chisquare(o, e).pvalue


def test_degree_laws(kgref):
    n = 2**13
    # directed G(n,m): out-degree ~ Hyp(N, n-1, m); in-degree the same law
    m = 16 * n
    I = kgref.inst(n, m=m, directed=True, seed=21, chunks=16)
    E = kgref.generate(I)
    N = n * (n - 1)
    rv = stats.hypergeom(N, n - 1, m)
    assert _degree_chi2(np.bincount(E[:, 0], minlength=n), rv) > 1e-5
    assert _degree_chi2(np.bincount(E[:, 1], minlength=n), rv) > 1e-5
    # undirected G(n,m): degree ~ Hyp(N, n-1, m)
    I = kgref.inst(n, m=m, directed=False, seed=22, chunks=8)
    E = kgref.generate(I)
    N = n * (n - 1) // 2
    deg = np.bincount(E.ravel(), minlength=n)
    assert _degree_chi2(deg, stats.hypergeom(N, n - 1, m)) > 1e-5
    # G(n,p): degree ~ Bin(n-1, p)
    p = 24 / (n - 1)
    E = kgref.generate(kgref.inst(n, p=p, directed=False, seed=23, chunks=8))
    deg = np.bincount(E.ravel(), minlength=n)
    assert _degree_chi2(deg, stats.binom(n - 1, p)) > 1e-5


def test_tile_counts_sum_and_law(kgref):
    I = kgref.inst(2**16, m=2**20, directed=True, seed=1, chunks=64)
    s = kgref.tile_exponent(I)
    assert s == 22
    Nc = 1024 * (2**16 - 1)
    counts = kgref.chunk_counts(I)
    for c in [0, 17, 63]:
        tc = kgref.tile_counts(I, c, counts[c])
        assert tc.sum() == counts[c]
        assert len(tc) == -(-Nc // 2**s)              # ceil(N_c / 2^s) tiles, the last partial
    # tile 0 of chunk 0 across seeds ~ Hyp(N_c, S, K_c) given K_c: check mean
    vals = []
    for seed in range(300):
        J = kgref.inst(2**16, m=2**20, directed=True, seed=seed, chunks=64)
        Kc = kgref.chunk_count_path(J, 0)
        tc = kgref.tile_counts(J, 0, Kc)
        vals.append((tc[0] - Kc * 2**s / Nc) / math.sqrt(Kc * 2**s / Nc))
    assert abs(np.mean(vals)) < 5 / math.sqrt(300)


def test_gnp_geometric_skip_cross_check(kgref):
    """An independent G(n,p) sampler written here (Batagelj-Brandes style
    geometric skips over all slots, numpy's generator) must agree with the
    oracle in distribution: total edges and degree histogram (two-sample)."""
    n, p = 600, 0.02
    N = n * (n - 1) // 2
    rng = np.random.default_rng(77)
    tot_a, tot_b = [], []
    deg_a = np.zeros(n)
    deg_b = np.zeros(n)
    for s in range(300):
        E = kgref.generate(kgref.inst(n, p=p, directed=False, seed=500 + s, chunks=4))
        tot_a.append(len(E))
        deg_a += np.bincount(E.ravel(), minlength=n)
        pos, cnt = -1, 0
        idx = []
        while True:
            pos += int(rng.geometric(p))
            if pos >= N:
                break
            idx.append(pos)
        idx = np.array(idx, dtype=np.int64)
        # slot -> (u,v) over the strict upper triangle, row-major
        u = np.searchsorted(np.cumsum(np.arange(n - 1, 0, -1)), idx, side="right")
        deg_b += np.bincount(u, minlength=n)
        start = u * n - u * (u + 1) // 2
        v = u + 1 + (idx - start)
        deg_b += np.bincount(v, minlength=n)
        tot_b.append(len(idx))
    assert stats.ks_2samp(tot_a, tot_b).pvalue > 1e-4
    assert stats.ttest_ind(deg_a / 300, deg_b / 300).pvalue > 1e-4


def test_uneven_tile_tree_marginals(kgref):
    """n=100 directed, m=2000, one chunk: tiles of 2^12 slots -> sizes 4096,
    4096, 1708 (the root splits [0,2) | [2,3)).  Each tile count must follow
    Hyp(9900, size, 2000); a swapped split would move tile 2's mean from
    345.1 to 827.5."""
    I0 = kgref.inst(100, m=2000, directed=True, seed=1, chunks=1)
    assert kgref.tile_exponent(I0) == 12
    reps = 3000
    tc = np.zeros((reps, 3), dtype=np.int64)
    for s in range(reps):
        I = kgref.inst(100, m=2000, directed=True, seed=s, chunks=1)
        tc[s] = kgref.tile_counts(I, 0, 2000)
    assert np.all(tc.sum(axis=1) == 2000)
    for t, size in enumerate([4096, 4096, 1708]):
        rv = stats.hypergeom(9900, size, 2000)
        assert _degree_chi2(tc[:, t], rv) > 1e-5, t


@pytest.mark.parametrize("n,m,directed,P", [(100, 1500, True, 1), (100, 1500, True, 3),
                                             (200, 4000, False, 2), (200, 4000, False, 3)])
def test_slot_uniformity_multi_tile(kgref, n, m, directed, P):
    """Every slot is chosen with probability m/N (uniform m-subsets), across
    tile and chunk boundaries, including triangle and rectangle decoding."""
    N = n * (n - 1) // (1 if directed else 2)
    reps = 1500
    hits = np.zeros(n * n, dtype=np.int64)
    for s in range(reps):
        E = kgref.generate(kgref.inst(n, m=m, directed=directed, seed=7000 + s, chunks=P))
        hits[edge_key(E, n)] += 1
    valid = np.array([(u != v) and (directed or u < v) for u in range(n) for v in range(n)])
    assert hits[~valid].sum() == 0
    h = hits[valid]
    assert len(h) == N and h.sum() == m * reps
    assert stats.chisquare(h).pvalue > 1e-5

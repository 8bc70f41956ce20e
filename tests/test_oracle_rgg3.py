"""Pins of the oracle's three-dimensional random geometric graph (Sec.
2.1.2, Sec. 5 with d = 3) against facts outside the oracle: the all-pairs
definition of the graph (brute force over every pair, and exact rational
distances), the multinomial law of the octant split (means, variances,
covariances), the uniform law of the points, the closed-form mean edge count
of the unit cube, and the root-path recomputation of Sec. 5.1."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import kgref


def _brute(P, r):
    d2 = np.zeros((len(P), len(P)))
    # the oracle's order of operations: (dx^2 + dy^2) + dz^2, each rounded
    dx = P[:, 0][:, None] - P[:, 0][None, :]
    dy = P[:, 1][:, None] - P[:, 1][None, :]
    dz = P[:, 2][:, None] - P[:, 2][None, :]
    d2 = (dx * dx + dy * dy) + dz * dz
    adj = np.triu(d2 < r * r, 1)
    u, v = np.nonzero(adj)
    return np.stack([u, v], 1).astype(np.uint32)


@pytest.mark.parametrize("n,r,seed", [(2000, 0.1, 1), (1500, 0.05, 7), (300, 0.3, 2), (60, 0.6, 3),
                                      (4000, 0.04, 5), (3, 0.2, 1), (1, 0.5, 1), (0, 0.5, 1), (700, 0.0, 4),
                                      (500, 2.0, 9), (5000, 0.03, 6)])
def test_edges_equal_all_pairs(n, r, seed):
    P, E = kgref.rgg3d(n, r, seed)
    assert P.shape == (n, 3)
    assert np.array_equal(E, _brute(P, r))


def test_predicate_matches_exact_distance():
    """The binary64 test decides as exact rational arithmetic on the same
    coordinates for every pair not within 1e-9 of the radius."""
    n, r = 300, 0.2
    P, E = kgref.rgg3d(n, r, 11)
    have = set(map(tuple, E.tolist()))
    R2 = Fraction(r) * Fraction(r)
    F = [tuple(Fraction(float(c)) for c in p) for p in P]
    for u in range(n):
        for v in range(u + 1, n):
            d2 = sum((F[u][k] - F[v][k]) ** 2 for k in range(3))
            if abs(float(d2) - r * r) < 1e-9:
                continue
            assert (d2 < R2) == ((u, v) in have)


def test_level_rule():
    # cells of side 2^-L >= r and at most n of them; the benchmark radius
    # 0.55 (ln n / n)^(1/3) at n = 2^26 gives L = 8
    r26 = 0.55 * (math.log(2**26) / 2**26) ** (1.0 / 3.0)
    assert kgref.rgg3_level(2**26, r26) == 8
    assert kgref.rgg3_level(10**6, 0.5) == 1 and kgref.rgg3_level(10**6, 0.5000001) == 0
    assert kgref.rgg3_level(7, 0.01) == 0 and kgref.rgg3_level(8, 0.01) == 1 and kgref.rgg3_level(64, 0.01) == 2
    assert kgref.rgg3_level(2**32 - 1, 0.0) == kgref.RGG3_MAX_LEVEL
    for n, r in [(1000, 0.03), (10**5, 0.04), (777, 0.2)]:
        L = kgref.rgg3_level(n, r)
        assert 2.0**-L >= r and 8**L <= n
        assert L == kgref.RGG3_MAX_LEVEL or 2.0**-(L + 1) < r or 8**(L + 1) > n


def test_points_lie_in_their_cells_in_morton_order():
    n, r, seed = 5000, 0.1, 3
    L = kgref.rgg3_level(n, r)
    assert L == 3
    cells = kgref.rgg3_cells(n, r, seed)
    assert int(cells.sum()) == n
    P, _ = kgref.rgg3d(n, r, seed)
    h = 2.0**-L
    off = np.concatenate([[0], np.cumsum(cells)]).astype(np.int64)
    for z in range(1 << (3 * L)):
        c = [sum(((z >> (3 * i + d)) & 1) << i for i in range(L)) for d in range(3)]
        pts = P[off[z]:off[z + 1]]
        for d in range(3):
            assert np.all(pts[:, d] >= c[d] * h) and np.all(pts[:, d] <= (c[d] + 1) * h)


def test_cell_points_equal_the_whole_generator():
    n, r, seed = 3000, 0.1, 8
    cells = kgref.rgg3_cells(n, r, seed)
    P, _ = kgref.rgg3d(n, r, seed)
    off = np.concatenate([[0], np.cumsum(cells)]).astype(np.int64)
    for z in (0, 5, 77, len(cells) - 1):
        assert np.array_equal(kgref.rgg3_cell_points(n, r, seed, z, int(cells[z])), P[off[z]:off[z + 1]])


def test_root_path_recomputes_every_cell():
    """Sec. 5.1: a processor gets a cell's count from the cell's root path
    alone; it equals the count of the whole recursion for every cell."""
    for n, r, seed in [(3000, 0.1, 1), (100000, 0.04, 2), (20, 0.3, 5)]:
        cells = kgref.rgg3_cells(n, r, seed)
        for z in range(len(cells)):
            assert kgref.rgg3_cell_count_path(n, r, seed, z) == int(cells[z])


def test_octant_counts_are_multinomial():
    """L = 1: the eight octant counts are multinomial(n; 1/8 each): mean
    n/8, variance 7n/64, covariance -n/64 (a wrong split slot, a swapped
    octant or a conditional draw on the wrong half breaks the means or the
    covariance pattern)."""
    n, S = 1000, 3000
    X = np.array([kgref.rgg3_cells(n, 0.4, s) for s in range(S)], dtype=np.float64)
    assert X.shape == (S, 8)
    assert np.all(X.sum(1) == n)
    m = X.mean(0)
    C = np.cov(X.T)
    se_mean = math.sqrt(7 * n / 64 / S)
    assert np.all(np.abs(m - n / 8) < 5 * se_mean)
    var, cov = 7 * n / 64, -n / 64
    tol = 5 * var * math.sqrt(2.0 / S)
    for i in range(8):
        assert abs(C[i, i] - var) < tol
        for j in range(i + 1, 8):
            assert abs(C[i, j] - cov) < tol


def test_points_uniform():
    from scipy import stats
    P, _ = kgref.rgg3d(200000, 0.004, 13)
    for k in range(3):
        assert stats.kstest(P[:, k], "uniform").pvalue > 1e-4
    # independence of the coordinates: the eight octant counts
    q = (P[:, 0] >= 0.5).astype(int) + 2 * (P[:, 1] >= 0.5).astype(int) + 4 * (P[:, 2] >= 0.5).astype(int)
    cnt = np.bincount(q, minlength=8)
    assert stats.chisquare(cnt).pvalue > 1e-4


def test_mean_edge_count():
    """E[edges] = C(n,2) (4 pi r^3 / 3 - 3 pi r^4 / 2 + 8 r^5 / 5 - r^6 / 6)
    in the unit cube (r <= 1): the probability that two uniform points are
    closer than r, the integral of the product of the three coordinate
    differences' triangular densities over the ball."""
    n, r, S = 600, 0.15, 200
    mu = n * (n - 1) / 2 * (4 * math.pi * r**3 / 3 - 1.5 * math.pi * r**4 + 1.6 * r**5 - r**6 / 6)
    E = np.array([len(kgref.rgg3d(n, r, s)[1]) for s in range(S)], dtype=np.float64)
    se = E.std(ddof=1) / math.sqrt(S)
    assert abs(E.mean() - mu) < 5 * se

"""Pins of the oracle's two-dimensional random geometric graph (Sec. 2.1.2,
Sec. 5) against facts outside the oracle: the all-pairs definition of the
graph (brute force over every pair, and exact rational distances), the
multinomial law of the quadrant split (mean, variance, covariance), the
uniform law of the points, the closed-form mean edge count of the unit
square, and the root-path recomputation of Sec. 5.1 (a processor needing a
cell recomputes it alone)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import kgref


def _brute(P, r):
    x, y = P[:, 0], P[:, 1]
    dx = x[:, None] - x[None, :]
    dy = y[:, None] - y[None, :]
    adj = np.triu(dx * dx + dy * dy < r * r, 1)
    u, v = np.nonzero(adj)
    return np.stack([u, v], 1).astype(np.uint32)


@pytest.mark.parametrize("n,r,seed", [(2000, 0.05, 1), (1500, 0.02, 7), (300, 0.3, 2), (50, 0.6, 3),
                                      (4000, 0.011, 5), (3, 0.2, 1), (1, 0.5, 1), (0, 0.5, 1), (700, 0.0, 4),
                                      (600, 2.0, 9)])
def test_edges_equal_all_pairs(n, r, seed):
    P, E = kgref.rgg2d(n, r, seed)
    assert P.shape == (n, 2)
    assert np.array_equal(E, _brute(P, r))


def test_predicate_matches_exact_distance():
    """The binary64 test decides as exact rational arithmetic on the same
    coordinates for every pair not within 1e-9 of the radius."""
    n, r = 400, 0.09
    P, E = kgref.rgg2d(n, r, 11)
    have = set(map(tuple, E.tolist()))
    R2 = Fraction(r) * Fraction(r)
    F = [(Fraction(float(a)), Fraction(float(b))) for a, b in P]
    for u in range(n):
        for v in range(u + 1, n):
            d2 = (F[u][0] - F[v][0]) ** 2 + (F[u][1] - F[v][1]) ** 2
            if abs(float(d2) - r * r) < 1e-9:
                continue
            assert (d2 < R2) == ((u, v) in have)


def test_level_rule():
    # cells of side 2^-L >= r and at most n of them
    r26 = 0.55 * math.sqrt(math.log(2**26) / 2**26)
    assert kgref.rgg_level(2**26, r26) == 11
    assert kgref.rgg_level(10**6, 0.5) == 1 and kgref.rgg_level(10**6, 0.5000001) == 0
    assert kgref.rgg_level(3, 0.01) == 0 and kgref.rgg_level(4, 0.01) == 1 and kgref.rgg_level(16, 0.01) == 2
    assert kgref.rgg_level(2**32 - 1, 0.0) == kgref.RGG_MAX_LEVEL
    for n, r in [(1000, 0.03), (10**5, 0.004), (777, 0.2)]:
        L = kgref.rgg_level(n, r)
        assert 2.0**-L >= r and 4**L <= n
        assert L == kgref.RGG_MAX_LEVEL or 2.0**-(L + 1) < r or 4**(L + 1) > n


def test_points_lie_in_their_cells_in_morton_order():
    n, r, seed = 5000, 0.03, 3
    L = kgref.rgg_level(n, r)
    cells = kgref.rgg_cells(n, r, seed)
    assert int(cells.sum()) == n
    P, _ = kgref.rgg2d(n, r, seed)
    h = 2.0**-L
    off = np.concatenate([[0], np.cumsum(cells)]).astype(np.int64)
    for z in range(1 << (2 * L)):
        cx = sum(((z >> (2 * i)) & 1) << i for i in range(L))
        cy = sum(((z >> (2 * i + 1)) & 1) << i for i in range(L))
        pts = P[off[z]:off[z + 1]]
        assert np.all(pts[:, 0] >= cx * h) and np.all(pts[:, 0] <= (cx + 1) * h)
        assert np.all(pts[:, 1] >= cy * h) and np.all(pts[:, 1] <= (cy + 1) * h)


def test_root_path_recomputes_every_cell():
    """Sec. 5.1: a processor gets a cell's count from the cell's root path
    alone; it equals the count of the whole recursion for every cell."""
    for n, r, seed in [(3000, 0.04, 1), (100000, 0.01, 2), (20, 0.2, 5)]:
        cells = kgref.rgg_cells(n, r, seed)
        for z in range(len(cells)):
            assert kgref.rgg_cell_count_path(n, r, seed, z) == int(cells[z])


def test_quadrant_counts_are_multinomial():
    """L = 1: the four quadrant counts are multinomial(n; 1/4 each): mean
    n/4, variance 3n/16, covariance -n/16 (a wrong split slot or a swapped
    quadrant breaks the covariance pattern or the means)."""
    n, S = 1000, 3000
    X = np.array([kgref.rgg_cells(n, 0.4, s) for s in range(S)], dtype=np.float64)
    assert X.shape == (S, 4)
    assert np.all(X.sum(1) == n)
    m = X.mean(0)
    C = np.cov(X.T)
    se_mean = math.sqrt(3 * n / 16 / S)
    assert np.all(np.abs(m - n / 4) < 5 * se_mean)
    var, cov = 3 * n / 16, -n / 16
    # sample (co)variances: standard error about var * sqrt(2 / S)
    tol = 5 * var * math.sqrt(2.0 / S)
    for i in range(4):
        assert abs(C[i, i] - var) < tol
        for j in range(i + 1, 4):
            assert abs(C[i, j] - cov) < tol


def test_points_uniform():
    from scipy import stats
    P, _ = kgref.rgg2d(200000, 0.002, 13)
    for k in range(2):
        assert stats.kstest(P[:, k], "uniform").pvalue > 1e-4
    # independence of x and y: the four quadrant counts
    q = (P[:, 0] >= 0.5).astype(int) + 2 * (P[:, 1] >= 0.5).astype(int)
    cnt = np.bincount(q, minlength=4)
    assert stats.chisquare(cnt).pvalue > 1e-4


def test_mean_edge_count():
    """E[edges] = C(n,2) (pi r^2 - 8 r^3 / 3 + r^4 / 2) in the unit square."""
    n, r, S = 600, 0.08, 200
    mu = n * (n - 1) / 2 * (math.pi * r * r - 8 * r**3 / 3 + r**4 / 2)
    E = np.array([len(kgref.rgg2d(n, r, s)[1]) for s in range(S)], dtype=np.float64)
    se = E.std(ddof=1) / math.sqrt(S)
    assert abs(E.mean() - mu) < 5 * se

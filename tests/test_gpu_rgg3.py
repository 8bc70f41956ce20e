"""GPU parity of the three-dimensional random geometric graph (kg_rgg3d)
against the oracle: points bit for bit (as 64-bit patterns) and the edge list
element by element, at sizes that span many scan tiles, waves of vertices and
cells (including waves whose vertices spread over more than 64 cells), and at
the full benchmark size (n = 2^26, r = 0.55 (ln n / n)^(1/3)) on sampled
cells and vertices; plus the degenerate cases and the capacity contract."""
import math

import numpy as np
import pytest

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _np(t):
    import torch
    if t.dtype == torch.float64:
        return t.cpu().view(torch.int64).numpy().view(np.float64)
    return t.cpu().view(torch.int32).numpy().view(np.uint32)


def _r3(n):
    return 0.55 * (math.log(n) / n) ** (1.0 / 3.0)


CASES = [(0, 0.5, 1), (1, 0.5, 1), (2, 0.9, 3), (3, 0.2, 1), (60, 0.6, 3), (300, 0.3, 2), (2000, 0.1, 1),
         (4000, 0.04, 5), (700, 0.0, 4), (500, 2.0, 9), (5000, 0.02, 7), (100003, 0.02, 8), (200000, 0.015, 2),
         (1 << 20, _r3(1 << 20), 6)]


@pytest.mark.parametrize("n,r,seed", CASES)
def test_rgg3d_matches_oracle(kgref, n, r, seed):
    kg = require_gpu()
    print("rgg3d n=%d r=%g seed=%d" % (n, r, seed), flush=True)
    P, E = kg.rgg3d(n, r, seed)
    wantP, wantE = kgref.rgg3d(n, r, seed)
    gotP = _np(P)
    assert gotP.shape == wantP.shape
    assert np.array_equal(gotP.view(np.int64), wantP.view(np.int64))
    gotE = _np(E)
    assert gotE.shape == wantE.shape
    assert np.array_equal(gotE, wantE)


def test_rgg3d_capacity_contract(kgref):
    import torch
    kg = require_gpu()
    n, r, seed = 3000, 0.08, 12
    _, wantE = kgref.rgg3d(n, r, seed)
    E = len(wantE)
    # too small: nothing written, the total reported
    out = torch.full((E - 1, 2), 7, dtype=torch.int32, device="cuda").view(torch.uint32)
    P, out2, tot = kg.rgg3d(n, r, seed, out=out)
    torch.cuda.synchronize()
    assert int(tot.view(torch.int64).cpu()[0]) == E
    assert np.all(_np(out2) == 7)
    # exact fit
    out = torch.empty((E, 2), dtype=torch.uint32, device="cuda")
    P, out2, tot = kg.rgg3d(n, r, seed, out=out)
    torch.cuda.synchronize()
    assert np.array_equal(_np(out2), wantE)
    # a second call on the same buffers with a smaller graph leaves nothing stale
    n2 = 1000
    _, wantE2 = kgref.rgg3d(n2, r, seed + 1)
    P2, out3, tot2 = kg.rgg3d(n2, r, seed + 1, out=out)
    torch.cuda.synchronize()
    E2 = int(tot2.view(torch.int64).cpu()[0])
    assert E2 == len(wantE2)
    assert np.array_equal(_np(out3)[:E2], wantE2)


def test_rgg3d_argument_errors():
    kg = require_gpu()
    for n, r in [(10, -0.1), (10, float("nan"))]:
        with pytest.raises(kg.KgError):
            kg.rgg3d(n, r, 1)
    with pytest.raises(kg.KgError):
        kg.rgg3d_workspace_bytes(1 << 32, 0.001)
    with pytest.raises(kg.KgError):
        kg.rgg3d_workspace_bytes(10**6, 0.7)       # one cell of 10^6 points


def test_rgg3d_fullsize_sampled(kgref):
    """n = 2^26, r = 0.55 (ln n / n)^(1/3) (L = 8, 8^8 cells), the launch the
    benchmark times: sampled cells' points against the oracle bit for bit,
    sampled vertices' edge lists against a search of the 3 x 3 x 3 cell
    window on those points, and the invariants of the whole list."""
    import torch
    kg = require_gpu()
    n = 1 << 26
    r = _r3(n)
    seed = 1
    print("rgg3d full size n=2^26", flush=True)
    P, E = kg.rgg3d(n, r, seed)
    torch.cuda.synchronize()
    L = kgref.rgg3_level(n, r)
    assert L == 8
    cells = kgref.rgg3_cells(n, r, seed).astype(np.int64)
    off = np.concatenate([[0], np.cumsum(cells)])
    assert off[-1] == n
    Ph = _np(P)
    rng = np.random.default_rng(5)
    for z in rng.integers(0, len(cells), 300):
        want = kgref.rgg3_cell_points(n, r, seed, int(z), int(cells[z]))
        assert np.array_equal(Ph[off[z]:off[z + 1]].view(np.int64), want.view(np.int64)), int(z)
    print("  sampled cells match; checking %d edges" % E.shape[0], flush=True)
    Eh = _np(E)
    mu = kg.rgg3d_expected_edges(n, r)
    assert abs(len(Eh) - mu) < 0.01 * mu
    assert np.all(Eh[:, 0] < Eh[:, 1])
    key = Eh[:, 0].astype(np.uint64) << np.uint64(32) | Eh[:, 1].astype(np.uint64)
    assert np.all(key[1:] > key[:-1])
    G = 1 << L

    def cell_xyz(z):
        return [sum(((z >> (3 * i + d)) & 1) << i for i in range(L)) for d in range(3)]

    def morton(c):
        return sum(((c[d] >> i) & 1) << (3 * i + d) for i in range(L) for d in range(3))

    col0 = np.ascontiguousarray(Eh[:, 0])
    for u in rng.integers(0, n, 300):
        z = int(np.searchsorted(off, u, side="right") - 1)
        c = cell_xyz(z)
        cand = []
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    w = [c[0] + dx, c[1] + dy, c[2] + dz]
                    if all(0 <= t < G for t in w):
                        zz = morton(w)
                        cand.extend(range(off[zz], off[zz + 1]))
        cand = np.array(sorted(v for v in cand if v > u), dtype=np.int64)
        d = Ph[cand] - Ph[u]
        want = cand[(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2] < r * r]
        # a query of the column's own dtype: no cast of the whole column per call
        lo, hi = np.searchsorted(col0, np.uint32(u), "left"), np.searchsorted(col0, np.uint32(u), "right")
        assert np.array_equal(Eh[lo:hi, 1].astype(np.int64), want), int(u)

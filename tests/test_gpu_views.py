"""The per-PE view on the GPU (kg_pe_view, and views as kg_batch instances)
equals the oracle's view byte for byte (Sec. 4.1: a PE's row chunk; Sec. 4.2:
the chunk row and column of its section), for small shapes, G(n,p), the
headline undirected workload's sections, and all P views of a graph in one
batch."""
import numpy as np
import pytest

from gpu_util import require_gpu, to_np_u32, to_np_u64

pytestmark = pytest.mark.gpu

CASES = [(60, 0, 500, None, True, 5), (60, 0, 700, None, False, 5), (97, 1, 0, 0.05, False, 7),
         (3000, 0, 10**6, None, False, 13), (2**16, 0, 2**20, None, True, 64), (5000, 1, 0, 0.01, True, 33),
         (777, 0, 300000, None, False, 5)]


@pytest.mark.parametrize("n,model,m,p,directed,P", CASES)
def test_pe_view_equals_oracle(kg_mod, kgref, n, model, m, p, directed, P):
    import torch
    kg = kg_mod
    I = kgref.inst(n, m=m, p=p or 0.0, directed=directed, seed=5, chunks=P, model=model)
    for r in sorted({0, P // 2, P - 1}):
        got = kg.pe_view(n, r, P, directed=directed, m=m, p=p, seed=5)
        torch.cuda.synchronize()
        want = kgref.pe_view(I, r)
        assert np.array_equal(to_np_u32(got), want), (n, P, r)


def test_all_views_in_one_batch(kg_mod, kgref):
    import torch
    kg = kg_mod
    n, m, P = 3000, 400000, 9
    whole = kg.Instance(n, kg.GNM, False, m, 0.0, 8, P)
    views = [kg.Instance(n, kg.GNM, False, m, 0.0, 8, P, view=r + 1) for r in range(P)]
    arena, offs = kg.batch([whole] + views)
    torch.cuda.synchronize()
    A, O = to_np_u32(arena), to_np_u64(offs).astype(np.int64)
    I = kgref.inst(n, m=m, directed=False, seed=8, chunks=P)
    assert np.array_equal(A[O[0]:O[1]], kgref.generate(I))
    for r in range(P):
        assert np.array_equal(A[O[r + 1]:O[r + 2]], kgref.pe_view(I, r)), r


def test_pe_view_overflow_writes_nothing(kg_mod, kgref):
    import torch
    kg = kg_mod
    n, m, P, r = 3000, 10**6, 13, 4
    want = kgref.pe_view(kgref.inst(n, m=m, directed=False, seed=2, chunks=P), r)
    small = torch.full((len(want) - 1, 2), 0xABCD, dtype=torch.int32, device="cuda").view(torch.uint32)
    out, total = kg.pe_view(n, r, P, directed=False, m=m, seed=2, out=small)
    torch.cuda.synchronize()
    assert int(to_np_u64(total)[0]) == len(want)
    assert np.all(to_np_u32(out) == 0xABCD)


@pytest.mark.parametrize("r", [0, 100, 255])
def test_headline_sections(kg_mod, kgref, r):
    """Undirected n = 2^26, m = 2^31, P = 256: the view of section r (about
    2^24 edges) equals the oracle's."""
    import torch
    kg = kg_mod
    n, m, P = 2**26, 2**31, 256
    got = kg.pe_view(n, r, P, directed=False, m=m, seed=1)
    torch.cuda.synchronize()
    want = kgref.pe_view(kgref.inst(n, m=m, directed=False, seed=1, chunks=P), r)
    assert got.shape[0] == len(want)
    assert np.array_equal(to_np_u32(got), want)
    del got
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def kg_mod():
    return require_gpu()

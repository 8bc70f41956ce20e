"""The geometric-skip G(n,p) variant on the GPU (kg_gnp_skip) equals the
oracle's skip variant byte for byte: small and mid shapes (both waiting-time
forms, p = 0 and p = 1, directed and undirected, ragged tiles), the
overflow contract, and the directed 2^25 / 2^16-chunk workload on its first
and last chunks plus the device-side invariants."""
import numpy as np
import pytest

from gpu_util import require_gpu, to_np_u32, to_np_u64

pytestmark = pytest.mark.gpu

CASES = [(60, 0.05, True, 5), (97, 0.3, False, 7), (40, 0.8, True, 3), (50, 1.0, False, 4), (90, 0.0, True, 3),
         (2**12, 16 / (2**12 - 1), True, 64), (5000, 0.01, False, 7), (3000, 0.9, True, 2), (1, 0.5, True, 1),
         (2**16, 1e-5, True, 256), (20000, 2e-4, False, 200),
         # about 1440 successes per 4096-slot tile: most tiles fill the write
         # pass's LDS batch (1408 events) and are stored in two parts
         (5000, 0.3516, True, 3), (3000, 0.3516, False, 5),
         # failures just under the batch size when p is just above 1/2
         (4000, 0.5001, True, 2)]


@pytest.mark.parametrize("n,p,directed,P", CASES)
def test_skip_equals_oracle(kgs, kgref, n, p, directed, P):
    import torch
    got = kgs.gnp_skip(n, p, directed, 9, P)
    torch.cuda.synchronize()
    want = kgref.skip_generate(kgref.inst(n, p=p, directed=directed, seed=9, chunks=P, model=kgref.GNP))
    assert got.shape[0] == len(want)
    assert np.array_equal(to_np_u32(got), want)


def test_skip_overflow_writes_nothing(kgs, kgref):
    import torch
    n, p, P = 3000, 0.01, 7
    want = kgref.skip_generate(kgref.inst(n, p=p, directed=False, seed=2, chunks=P, model=kgref.GNP))
    small = torch.full((len(want) - 1, 2), 0xABCD, dtype=torch.int32, device="cuda").view(torch.uint32)
    out, total = kgs.gnp_skip(n, p, False, 2, P, out=small)
    torch.cuda.synchronize()
    assert int(to_np_u64(total)[0]) == len(want)
    assert np.all(to_np_u32(out) == 0xABCD)


def test_skip_directed_workload(kgs, kgref):
    """Directed n = 2^25, p = 16/(n-1), 2^16 chunks: the first and the last
    ten chunks equal the oracle's; the whole output is in range, loop-free,
    and ascending inside every chunk (each chunk is a row range)."""
    import torch
    n, P, seed = 2**25, 2**16, 1
    p = 16.0 / (n - 1)
    E = kgs.gnp_skip(n, p, True, seed, P)
    torch.cuda.synchronize()
    I = kgref.inst(n, p=p, directed=True, seed=seed, chunks=P, model=kgref.GNP)
    head = np.concatenate([kgref.skip_chunk_edges(I, c) for c in range(10)])
    tail = np.concatenate([kgref.skip_chunk_edges(I, c) for c in range(P - 10, P)])
    assert np.array_equal(to_np_u32(E[:len(head)]), head)
    assert np.array_equal(to_np_u32(E[E.shape[0] - len(tail):]), tail)
    Ei = E.view(torch.int32)
    u, v = Ei[:, 0].to(torch.int64), Ei[:, 1].to(torch.int64)
    assert int(u.min()) >= 0 and int(v.min()) >= 0 and int(u.max()) < n and int(v.max()) < n
    assert not bool((u == v).any())
    key = u * n + v
    assert bool((key[1:] > key[:-1]).all())       # directed chunks are row ranges: globally ascending
    # the edge count is binomial(N, p): within 6 standard deviations
    N = n * (n - 1)
    assert abs(E.shape[0] - N * p) < 6 * np.sqrt(N * p * (1 - p))


@pytest.mark.parametrize("n,p,directed,P", [(5000, 0.01, False, 7), (5000, 0.3516, True, 3),
                                             (4000, 0.5001, True, 2), (3000, 0.9, True, 2)])
def test_skip_paths_agree(kgs, kgref, n, p, directed, P):
    """The write pass decodes the count pass's stored positions when the
    workspace holds a row per tile, and generates the events again when it
    does not (a workspace of the plain G(n,p) size) or when a tile has more
    events than its row keeps (rows of 64 here, so nearly every tile): the
    same bytes, the oracle's, every way."""
    import torch
    want = kgref.skip_generate(kgref.inst(n, p=p, directed=directed, seed=4, chunks=P, model=kgref.GNP))
    inst = kgs.Instance(n, kgs.GNP, directed, 0, p, 4, P)
    small = torch.empty(kgs.workspace_bytes([inst]), dtype=torch.uint8, device="cuda")
    assert small.numel() < kgs.gnp_skip_workspace_bytes(n, p, directed, P)
    got_rows = kgs.gnp_skip(n, p, directed, 4, P)
    got_regen = kgs.gnp_skip(n, p, directed, 4, P, workspace=small)
    try:
        kgs.set_option(kgs._lib.KG_OPT_SKIP_ROW, 64)
        assert kgs.get_option(kgs._lib.KG_OPT_SKIP_ROW) == 64
        got_short = kgs.gnp_skip(n, p, directed, 4, P)
    finally:
        kgs.set_option(kgs._lib.KG_OPT_SKIP_ROW, 0)
    torch.cuda.synchronize()
    for what, got in (("rows", got_rows), ("regenerated", got_regen), ("rows of 64", got_short)):
        assert got.shape[0] == len(want), what
        assert np.array_equal(to_np_u32(got), want), what


@pytest.fixture(scope="module")
def kgs():
    return require_gpu()

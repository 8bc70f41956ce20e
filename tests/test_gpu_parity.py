"""Whole-generator parity: the HIP path's edge lists equal the oracle's byte
for byte (G(n,m): Sec. 4.1 directed, Sec. 4.2 undirected; G(n,p): Sec. 4.3),
over small exhaustive grids, the 2^16-vertex / 2^20-edge directed workload,
tiles spanning chunk boundaries and ragged last tiles, dense instances
(complement sampling), degenerate sizes, and every launch shape."""
import numpy as np
import pytest

from gpu_util import require_gpu, to_np_u32, to_np_u64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kg():
    return require_gpu()


def gpu_gnm(kg, n, m, directed, seed, P):
    import torch
    E = kg.gnm(n, m, directed=directed, seed=seed, chunks=P)
    torch.cuda.synchronize()
    return to_np_u32(E)


def gpu_gnp(kg, n, p, directed, seed, P):
    import torch
    E = kg.gnp(n, p, directed=directed, seed=seed, chunks=P)
    torch.cuda.synchronize()
    return to_np_u32(E)


def check_equal(got, want, what):
    assert got.shape == want.shape, (what, got.shape, want.shape)
    if not np.array_equal(got, want):
        bad = np.nonzero(np.any(got != want, axis=1))[0]
        raise AssertionError("%s: %d rows differ, first %d: got %s want %s"
                             % (what, len(bad), bad[0], got[bad[0]], want[bad[0]]))


SMALL = []
for directed in (True, False):
    for n in (1, 2, 3, 4, 5, 9, 40, 257):
        N = n * (n - 1) // (1 if directed else 2)
        for P in sorted({1, 2, 3, n}):
            if P > n:
                continue
            for m in sorted({0, 1, N // 3, N // 2, N - 1, N}):
                if 0 <= m <= N:
                    SMALL.append((n, m, directed, P))


@pytest.mark.parametrize("n,m,directed,P", SMALL)
def test_small_gnm(kg, kgref, n, m, directed, P):
    seed = 1000 + n * 7 + m + P
    got = gpu_gnm(kg, n, m, directed, seed, P)
    want = kgref.generate(kgref.inst(n, m=m, directed=directed, seed=seed, chunks=P))
    check_equal(got, want, "gnm n=%d m=%d dir=%d P=%d" % (n, m, directed, P))


MID = [
    # (n, m, directed, P): several tiles per chunk, ragged last tiles, tiles of
    # 2^9..2^12 slots, dense tiles (complement), non-power-of-two sections
    (2**16, 2**20, True, 64), (1000, 300000, True, 7), (1000, 998000, True, 3), (3000, 2 * 10**6, False, 13),
    (2**12, 2**16, False, 8), (5000, 10**6, False, 33), (777, 100000, False, 1), (777, 300000, False, 5),
    (2**14, 2**21, True, 1), (123456, 10**6, True, 1000), (2**17, 2**20, False, 256), (600, 179700, False, 2),
    (90, 8000, True, 90), (10**5, 3 * 10**6, False, 100),
    # tiles of 2^32 slots (keys use all 32 bits)
    (2**26, 2**20, False, 256), (2**26, 2**21, True, 64),
    # more than 4096 wave sums (the offset scan takes several rounds)
    (2**18 + 1000, 2**20, True, 2**18 + 1000), (2**16, 2**20, False, 730),
]


@pytest.mark.parametrize("n,m,directed,P", MID)
def test_mid_gnm(kg, kgref, n, m, directed, P):
    got = gpu_gnm(kg, n, m, directed, 7, P)
    want = kgref.generate(kgref.inst(n, m=m, directed=directed, seed=7, chunks=P))
    check_equal(got, want, "gnm n=%d m=%d dir=%d P=%d" % (n, m, directed, P))


GNP = [(1, 0.5, True, 1), (2, 0.5, False, 1), (50, 0.3, True, 5), (50, 0.7, False, 5), (300, 1.0, True, 3),
       (300, 0.0, False, 3), (2**12, 16 / (2**12 - 1), True, 64), (2**12, 64 / (2**12 - 1), False, 16),
       (5000, 0.01, False, 7), (3000, 0.9, True, 2), (2**16, 1e-5, True, 256), (20000, 2e-4, False, 200)]


@pytest.mark.parametrize("n,p,directed,P", GNP)
def test_gnp(kg, kgref, n, p, directed, P):
    got = gpu_gnp(kg, n, p, directed, 11, P)
    want = kgref.generate(kgref.inst(n, p=p, directed=directed, seed=11, chunks=P, model=1))
    check_equal(got, want, "gnp n=%d p=%g dir=%d P=%d" % (n, p, directed, P))


def test_small_config_directed(kg, kgref):
    """Directed G(n,m), n=2^16, m=2^20, 64 chunks, seed 1: identical bytes."""
    got = gpu_gnm(kg, 2**16, 2**20, True, 1, 64)
    want = kgref.generate(kgref.inst(2**16, m=2**20, directed=True, seed=1, chunks=64))
    check_equal(got, want, "directed n=2^16 m=2^20 P=64")


# Tiles expecting about 1115 samples (the top of the 560..1120 range): the
# register base case's widest sorts (18 and 20 keys per lane) and its fifth
# Philox round on most tiles.
UPPER = [(3000, 1224500, True, 1, 0), (3000, 1224500, True, 7, 0), (2500, 424900, False, 4, 0),
         (3000, 0.2722, True, 3, 1), (2000, 0.2722, False, 5, 1)]


@pytest.mark.parametrize("n,mp,directed,P,model", UPPER)
def test_tiles_near_the_upper_bound(kg, kgref, n, mp, directed, P, model):
    if model == 0:
        got = gpu_gnm(kg, n, mp, directed, 21, P)
        I = kgref.inst(n, m=mp, directed=directed, seed=21, chunks=P)
    else:
        got = gpu_gnp(kg, n, mp, directed, 21, P)
        I = kgref.inst(n, p=mp, directed=directed, seed=21, chunks=P, model=1)
    want = kgref.generate(I)
    check_equal(got, want, "upper n=%d %s dir=%d P=%d" % (n, mp, directed, P))


@pytest.mark.parametrize("cap", [128, 200, 512])
def test_leaf_capacity_does_not_change_bits(kg, kgref, cap):
    """Tiles larger than the LDS pass capacity go through key sub-ranges;
    the bytes must not change."""
    cases = [(2**16, 2**20, True, 64), (3000, 2 * 10**6, False, 13), (1000, 600000, True, 3)]
    try:
        kg.set_option(kg._lib.KG_OPT_LEAF_CAP, cap)
        for n, m, d, P in cases:
            got = gpu_gnm(kg, n, m, d, 5, P)
            want = kgref.generate(kgref.inst(n, m=m, directed=d, seed=5, chunks=P))
            check_equal(got, want, "cap=%d n=%d m=%d" % (cap, n, m))
    finally:
        kg.set_option(kg._lib.KG_OPT_LEAF_CAP, 0)


@pytest.mark.parametrize("sw,pw", [(1, 1), (3, 2), (32, 64)])
def test_launch_shape_does_not_change_bits(kg, sw, pw):
    """The tile -> workgroup mapping must not show in the output: grids of
    1, 3 and 32 sampler workgroups per compute unit (the last past the
    resident ones) take the tiles in ranges of other sizes and orders (one
    tile each, or 32 then 8 from the shared counter for the 2^15-tile job on
    the smallest grid) and must write the same bytes."""
    base = gpu_gnm(kg, 5000, 10**6, False, 3, 33)
    base2 = gpu_gnm(kg, 2**14, 2**21, True, 4, 1)
    base3 = gpu_gnm(kg, 2**17, 2**25, True, 8, 5)
    try:
        kg.set_option(kg._lib.KG_OPT_SAMPLE_WAVES, sw)
        kg.set_option(kg._lib.KG_OPT_PLAN_WAVES, pw)
        got = gpu_gnm(kg, 5000, 10**6, False, 3, 33)
        got2 = gpu_gnm(kg, 2**14, 2**21, True, 4, 1)
        got3 = gpu_gnm(kg, 2**17, 2**25, True, 8, 5)
    finally:
        kg.set_option(kg._lib.KG_OPT_SAMPLE_WAVES, 0)
        kg.set_option(kg._lib.KG_OPT_PLAN_WAVES, 0)
    check_equal(got, base, "launch shape %d/%d" % (sw, pw))
    check_equal(got2, base2, "launch shape %d/%d" % (sw, pw))
    check_equal(got3, base3, "launch shape %d/%d" % (sw, pw))


@pytest.mark.parametrize("n,directed,P,model", [(2**16, True, 64, 0), (2**26, False, 256, 0),
                                                (2**25, True, 2**16, 1), (2**25, False, 256, 1),
                                                (10**6, True, 999, 0), (10**5, False, 77, 1)])
def test_chunk_counts(kg, kgref, n, directed, P, model):
    """Per-chunk counts at the workload shapes (every chunk recomputes its own
    root path on the GPU; the oracle expands the whole tree)."""
    import torch
    if model == 0:
        m = {2**16: 2**20, 2**26: 2**31}.get(n, n * 8)
        inst = kg.Instance(n, kg.GNM, directed, m, 0.0, 1, P)
        ref = kgref.inst(n, m=m, directed=directed, seed=1, chunks=P, model=0)
    else:
        p = (16.0 if directed else 64.0) / (n - 1)
        inst = kg.Instance(n, kg.GNP, directed, 0, p, 1, P)
        ref = kgref.inst(n, p=p, directed=directed, seed=1, chunks=P, model=1)
    want = kgref.chunk_counts(ref)
    # the count kernel's lanes per chunk (launch shape only): automatic, then
    # each fixed choice
    try:
        for lanes in (0, 1, 2, 4, 8):
            kg.set_option(kg._lib.KG_OPT_COUNT_LANES, lanes)
            got = to_np_u64(kg.chunk_counts(inst))
            torch.cuda.synchronize()
            assert np.array_equal(got, want), "lanes per chunk %d" % lanes
    finally:
        kg.set_option(kg._lib.KG_OPT_COUNT_LANES, 0)


def test_gnp_count_and_overflow(kg, kgref):
    import torch
    n, p, P = 3000, 0.01, 7
    want = kgref.generate(kgref.inst(n, p=p, directed=False, seed=2, chunks=P, model=1))
    assert kg.gnp_count(n, p, False, 2, P) == len(want)
    small = torch.full((len(want) - 1, 2), 0xABCD, dtype=torch.int32, device="cuda").view(torch.uint32)
    out, total = kg.gnp(n, p, False, 2, P, out=small)
    torch.cuda.synchronize()
    assert int(to_np_u64(total)[0]) == len(want)
    assert np.all(to_np_u32(out) == 0xABCD)      # nothing written on overflow


def test_batch_equals_single_calls(kg, kgref):
    import torch
    rng = np.random.default_rng(12)
    insts = []
    for i in range(40):
        n = int(2 ** rng.uniform(3, 13))
        d = bool(rng.integers(0, 2))
        P = int(rng.integers(1, min(n, 40) + 1))
        seed = kg.instance_seed(1, i)
        N = n * (n - 1) // (1 if d else 2)
        if rng.uniform() < 0.5:
            m = int(min(N, n * rng.uniform(1, 20)))
            insts.append(kg.Instance(n, kg.GNM, d, m, 0.0, seed, P))
        else:
            insts.append(kg.Instance(n, kg.GNP, d, 0, float(rng.uniform(0, 0.2)), seed, P))
    arena, offs = kg.batch(insts)
    torch.cuda.synchronize()
    A, O = to_np_u32(arena), to_np_u64(offs).astype(np.int64)
    for i, I in enumerate(insts):
        ref = kgref.inst(I.n, m=I.m, p=I.p, directed=I.directed, seed=I.seed, chunks=I.chunks, model=I.model)
        want = kgref.generate(ref)
        check_equal(A[O[i]:O[i + 1]], want, "batch instance %d" % i)
    assert O[-1] == len(A)


def test_instance_seed_matches_oracle(kg, kgref):
    for base in (1, 2, 2**63 + 5):
        for i in (0, 1, 4095):
            assert kg.instance_seed(base, i) == kgref.instance_seed(base, i)

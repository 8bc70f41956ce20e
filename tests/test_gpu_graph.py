"""Stream capture: a batch recorded into a HIP graph (kg_batch_upload, then
kg_batch_launch under capture) and replayed rewrites exactly the bytes of an
eager kg_batch; so does a captured single-instance kg_gnm.  Every replay is
checked, with the program's own eager work and synchronisations between
replays, and the target is cleared before each replay."""
import numpy as np
import pytest

from gpu_util import require_gpu, to_np_u32, to_np_u64

pytestmark = pytest.mark.gpu


def _instances(kg, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(2 ** rng.uniform(4, 14))
        d = bool(rng.integers(0, 2))
        P = int(rng.integers(1, min(n, 24) + 1))
        N = n * (n - 1) // (1 if d else 2)
        s = kg.instance_seed(seed, i)
        if rng.uniform() < 0.5:
            out.append(kg.Instance(n, kg.GNM, d, int(min(N, n * rng.uniform(1, 30))), 0.0, s, P))
        else:
            out.append(kg.Instance(n, kg.GNP, d, 0, float(rng.uniform(0, 0.1)), s, P))
    return out


def test_batch_graph_replays_equal_eager(kgref):
    import torch
    kg = require_gpu()
    insts = _instances(kg, 48, 5)
    ref_arena, ref_offs = kg.batch(insts)
    torch.cuda.synchronize()
    A, O = to_np_u32(ref_arena), to_np_u64(ref_offs)
    # the eager batch itself against the oracle on a few instances
    for i in (0, 17, 47):
        I = insts[i]
        want = kgref.generate(kgref.inst(I.n, m=I.m, p=I.p, directed=I.directed, seed=I.seed, chunks=I.chunks,
                                         model=I.model))
        assert np.array_equal(A[O[i]:O[i + 1]], want), i
    arena = torch.empty_like(ref_arena)
    offs = torch.empty_like(ref_offs)
    ws = torch.empty(kg.workspace_bytes(insts), dtype=torch.uint8, device="cuda")
    g = kg.BatchGraph(insts, arena, offs, ws)
    other = _instances(kg, 9, 6)
    for rep in range(3):
        arena.fill_(0xFFFFFFFF)
        offs.zero_()
        g.replay()
        # eager work between replays, on its own buffers
        kg.batch(other)
        kg.gnm(3000, 100000, False, 10 + rep, 7)
        torch.cuda.synchronize()
        assert np.array_equal(to_np_u64(offs), O), rep
        assert np.array_equal(to_np_u32(arena), A), rep


def test_captured_gnm_replays_equal_eager():
    import torch
    kg = require_gpu()
    n, m, d, seed, P = 20000, 600000, False, 3, 40
    want = to_np_u32(kg.gnm(n, m, d, seed, P))
    out = torch.empty((m, 2), dtype=torch.uint32, device="cuda")
    ws = torch.empty(kg.workspace_bytes([kg.Instance(n, kg.GNM, d, m, 0.0, seed, P)]), dtype=torch.uint8,
                     device="cuda")
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=side):
        kg.gnm(n, m, d, seed, P, out=out, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        out.zero_()
        g.replay()
        kg.gnm(5000, 70000, True, rep, 3)
        torch.cuda.synchronize()
        assert np.array_equal(to_np_u32(out), want), rep


def test_capture_refuses_host_work():
    """Under capture, calls that would copy from the host, allocate or
    synchronise are refused before anything is enqueued; a valid launch in
    the same capture still records and replays correctly."""
    import torch
    kg = require_gpu()
    insts = _instances(kg, 6, 8)
    ref_arena, ref_offs = kg.batch(insts)
    torch.cuda.synchronize()
    arena = torch.empty_like(ref_arena)
    offs = torch.empty_like(ref_offs)
    ws = torch.empty(kg.workspace_bytes(insts), dtype=torch.uint8, device="cuda")
    kg.batch_upload(insts, ws)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    errors = []
    with torch.cuda.graph(g, stream=side):
        for call in (lambda: kg.batch(insts, arena=arena, offsets=offs, workspace=ws),
                     lambda: kg.gnp_count(1000, 0.01, True, 1, 4, workspace=ws),
                     lambda: kg.batch_upload(insts, ws)):
            try:
                call()
            except kg.KgError as e:
                errors.append(e.status)
        kg.batch_launch(insts, arena, offs, ws)
    torch.cuda.current_stream().wait_stream(side)
    assert errors == [kg._lib.KG_EINVAL] * 3
    arena.zero_()
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(arena.view(torch.int32), ref_arena.view(torch.int32))
    assert torch.equal(offs.view(torch.int64), ref_offs.view(torch.int64))


def test_captured_rgg2d_replays_equal_eager():
    """kg_rgg2d with a caller workspace only enqueues kernels: recorded into
    a graph and replayed, it rewrites the eager call's points and edges."""
    import torch
    kg = require_gpu()
    n, r, seed = 50000, 0.006, 4
    P0, E0 = kg.rgg2d(n, r, seed)
    torch.cuda.synchronize()
    wantP, wantE = P0.cpu().view(torch.int64).numpy(), to_np_u32(E0)
    pts = torch.empty_like(P0)
    out = torch.empty((E0.shape[0] + 16, 2), dtype=torch.uint32, device="cuda")
    tot = torch.zeros(1, dtype=torch.uint64, device="cuda")
    ws = torch.empty(kg.rgg2d_workspace_bytes(n, r), dtype=torch.uint8, device="cuda")
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=side):
        kg.rgg2d(n, r, seed, points=pts, out=out, total=tot, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        pts.zero_()
        out.zero_()
        tot.zero_()
        g.replay()
        kg.rgg2d(3000, 0.03, rep)      # eager work between replays, on its own buffers
        torch.cuda.synchronize()
        assert int(tot.view(torch.int64).cpu()[0]) == len(wantE), rep
        assert np.array_equal(pts.cpu().view(torch.int64).numpy(), wantP), rep
        assert np.array_equal(to_np_u32(out)[:len(wantE)], wantE), rep

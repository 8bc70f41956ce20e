"""The workspace contract of the C ABI on the device: a workspace registered
with kg_set_workspace serves calls that pass none (same bytes as an explicit
workspace), a registered buffer that is too small is refused with
KG_ENOSPC before anything is enqueued, removing the registration falls back
to the stream-ordered allocator, and a registered workspace lets a call be
recorded into a HIP graph."""
import numpy as np
import pytest

from gpu_util import require_gpu, to_np_u32

pytestmark = pytest.mark.gpu


def _stream(torch):
    return torch.cuda.current_stream().cuda_stream


def test_registered_workspace_serves_calls_without_one(kgref):
    import torch
    kg = require_gpu()
    L = kg._lib.lib()
    n, m, P, seed = 2**14, 2**18, 8, 5
    want = kgref.generate(kgref.inst(n, m=m, directed=True, seed=seed, chunks=P))
    need = kg.workspace_bytes([kg.Instance(n, kg.GNM, True, m, 0.0, seed, P)])
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    out = torch.empty((m, 2), dtype=torch.uint32, device="cuda")
    try:
        kg.set_workspace(ws)
        out.fill_(0xFFFFFFFF)
        assert L.kg_gnm(n, m, 1, seed, P, out.data_ptr(), m, None, 0, _stream(torch)) == kg._lib.KG_OK
        torch.cuda.synchronize()
        assert np.array_equal(to_np_u32(out), want)
        # G(n,p) through the same registration, against an explicit workspace
        p = 3.0 / n
        E = kg.gnp(n, p, False, seed, P)
        tot = torch.zeros(1, dtype=torch.uint64, device="cuda")
        got = torch.full_like(E, 0xFFFFFFFF)
        assert L.kg_gnp(n, p, 0, seed, P, got.data_ptr(), got.shape[0], tot.data_ptr(), None, 0,
                        _stream(torch)) == kg._lib.KG_OK
        torch.cuda.synchronize()
        assert int(tot.view(torch.int64).item()) == E.shape[0]
        assert torch.equal(got.view(torch.int32), E.view(torch.int32))
        # a registered buffer that is too small: refused, nothing enqueued
        small = ws[: (need // 2) & ~255]
        kg.set_workspace(small)
        out.fill_(0xFFFFFFFF)
        assert L.kg_gnm(n, m, 1, seed, P, out.data_ptr(), m, None, 0, _stream(torch)) == kg._lib.KG_ENOSPC
        torch.cuda.synchronize()
        assert bool((out.view(torch.int32) == -1).all())
    finally:
        kg.set_workspace(None)
    # no registration: the stream-ordered allocator
    out.fill_(0)
    assert L.kg_gnm(n, m, 1, seed, P, out.data_ptr(), m, None, 0, _stream(torch)) == kg._lib.KG_OK
    torch.cuda.synchronize()
    assert np.array_equal(to_np_u32(out), want)


def test_capture_with_registered_workspace(kgref):
    """Recorded with only a registered workspace, kg_gnp_skip and kg_pe_view
    replay the eager bytes (three replays, eager work in between); without
    a workspace the same capture is refused with KG_EINVAL."""
    import torch
    kg = require_gpu()
    L = kg._lib.lib()
    n, p, P, seed = 5000, 0.002, 6, 11
    inst = kg.Instance(n, kg.GNP, True, 0, p, seed, P)
    E_skip = kg.gnp_skip(n, p, True, seed, P)
    E_view = kg.pe_view(n, 2, P, directed=True, p=p, seed=seed)
    torch.cuda.synchronize()
    want = kgref.skip_generate(kgref.inst(n, p=p, directed=True, seed=seed, chunks=P, model=1))
    assert np.array_equal(to_np_u32(E_skip), want)
    ws = torch.empty(kg.workspace_bytes([inst]), dtype=torch.uint8, device="cuda")
    out_s = torch.empty((E_skip.shape[0] + 64, 2), dtype=torch.uint32, device="cuda")
    out_v = torch.empty((E_view.shape[0] + 64, 2), dtype=torch.uint32, device="cuda")
    tot_s = torch.zeros(1, dtype=torch.uint64, device="cuda")
    tot_v = torch.zeros(1, dtype=torch.uint64, device="cuda")
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    try:
        with torch.cuda.graph(g, stream=side):
            # refused while nothing is registered, before anything is enqueued
            assert L.kg_gnp_skip(n, p, 1, seed, P, out_s.data_ptr(), out_s.shape[0], tot_s.data_ptr(), None, 0,
                                 side.cuda_stream) == kg._lib.KG_EINVAL
            kg.set_workspace(ws)
            assert L.kg_gnp_skip(n, p, 1, seed, P, out_s.data_ptr(), out_s.shape[0], tot_s.data_ptr(), None, 0,
                                 side.cuda_stream) == kg._lib.KG_OK
            assert L.kg_pe_view(inst.c(), 2, out_v.data_ptr(), out_v.shape[0], tot_v.data_ptr(), None, 0,
                                side.cuda_stream) == kg._lib.KG_OK
        torch.cuda.current_stream().wait_stream(side)
    finally:
        kg.set_workspace(None)
    for rep in range(3):
        out_s.fill_(0xFFFFFFFF)
        out_v.fill_(0xFFFFFFFF)
        tot_s.zero_()
        tot_v.zero_()
        g.replay()
        kg.gnm(3000, 20000, False, 40 + rep, 3)
        torch.cuda.synchronize()
        assert int(tot_s.view(torch.int64).item()) == E_skip.shape[0], rep
        assert int(tot_v.view(torch.int64).item()) == E_view.shape[0], rep
        assert torch.equal(out_s[:E_skip.shape[0]].view(torch.int32), E_skip.view(torch.int32)), rep
        assert torch.equal(out_v[:E_view.shape[0]].view(torch.int32), E_view.view(torch.int32)), rep

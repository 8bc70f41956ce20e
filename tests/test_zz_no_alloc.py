"""kg_gnm_static, the entry point that allocates nothing (its workspace is the
library's static per-device scratch), against kg_gnm with a workspace of its
own: byte-equal output on two calls in a row, the second with a smaller
input (the scratch keeps the first call's contents), plus the oracle on the
smaller one."""
import numpy as np
import pytest

from gpu_util import require_gpu, to_np_u32

pytestmark = pytest.mark.gpu

# (n, m, directed, seed, P): the first call at the headline size (undirected
# n = 2^26, m = 2^31, P = 256: 65.3 MiB of the 96 MiB scratch), then a much
# smaller directed one
CALLS = [(2**26, 2**31, False, 3, 256), (2**14, 2**18, True, 5, 8)]


def _stream(torch):
    return torch.cuda.current_stream().cuda_stream


def test_static_scratch_equals_gnm_twice(kgref):
    import torch
    kg = require_gpu()
    L = kg._lib.lib()
    for i, (n, m, directed, seed, P) in enumerate(CALLS):
        print("kg_gnm_static call %d: n=%d m=%d directed=%d seed=%d P=%d" % (i, n, m, directed, seed, P),
              flush=True)
        inst = kg.Instance(n, kg.GNM, directed, m, 0.0, seed, P)
        need = kg.workspace_bytes([inst])
        assert need <= kg._lib.KG_STATIC_SCRATCH_BYTES
        got = torch.full((m, 2), 0xFFFFFFFF, dtype=torch.uint32, device="cuda")
        st = L.kg_gnm_static(n, m, int(directed), seed, P, got.data_ptr(), m, _stream(torch))
        assert st == kg._lib.KG_OK, kg._lib.strerror(st)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        want = torch.zeros((m, 2), dtype=torch.uint32, device="cuda")
        st = L.kg_gnm(n, m, int(directed), seed, P, want.data_ptr(), m, ws.data_ptr(), need, _stream(torch))
        assert st == kg._lib.KG_OK, kg._lib.strerror(st)
        torch.cuda.synchronize()
        assert torch.equal(got.view(torch.int32), want.view(torch.int32)), "call %d differs from kg_gnm" % i
        if m <= 2**20:
            ref = kgref.generate(kgref.inst(n, m=m, directed=directed, seed=seed, chunks=P))
            assert np.array_equal(to_np_u32(got), ref)
        del got, want, ws
        torch.cuda.empty_cache()

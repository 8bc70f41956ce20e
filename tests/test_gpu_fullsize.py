"""Parity at the full workload sizes, in the launch configuration bench.py
times: every chunk count equals the oracle's; the headline workload (all
2^31 edges, seeds 1-3) equals the oracle byte for byte; the G(n,p) workloads
on a spread of whole chunks; properties that hold at any size are checked
over the entire output on the device (count, id range, u < v when
undirected, ascending inside each chunk, no repeats)."""
import numpy as np
import pytest

from gpu_util import require_gpu, to_np_u32, to_np_u64

pytestmark = pytest.mark.gpu


def _check_whole_output(torch, E, offs, n, directed):
    """Invariants on the device, in slices (E is (edges, 2) uint32)."""
    Ei = E.view(torch.int32)                  # ids < 2^31 here: int32 order = uint32 order
    total = E.shape[0]
    step = 1 << 27
    bounds = torch.from_numpy(offs.astype(np.int64)).cuda()
    for a in range(0, total, step):
        b = min(total, a + step)
        u = Ei[a:b, 0].to(torch.int64)
        v = Ei[a:b, 1].to(torch.int64)
        assert int(u.min()) >= 0 and int(v.min()) >= 0
        assert int(u.max()) < n and int(v.max()) < n
        assert not bool((u == v).any())
        if not directed:
            assert bool((u < v).all())
        key = u * n + v
        del u, v
        # ascending inside chunks: a step down may only happen at a chunk start
        dif = key[1:] - key[:-1]
        bad = torch.nonzero(dif <= 0).flatten() + (a + 1)
        if bad.numel():
            starts = torch.isin(bad, bounds)
            assert bool(starts.all()), "order broken inside a chunk at %s" % bad[~starts][:5].tolist()
        del key, dif


def _compare_all_chunks(torch, kgref, E, I, counts, block=1024):
    """Every edge of E equals the oracle's, chunk block by chunk block (the
    oracle fills a host buffer with OpenMP over the chunks of a block)."""
    offs = np.concatenate([[0], np.cumsum(counts.astype(np.int64))])
    C = len(counts)
    buf = None
    threads = kgref.max_threads()
    for c0 in range(0, C, block):
        c1 = min(C, c0 + block)
        a, b = int(offs[c0]), int(offs[c1])
        want = kgref.generate_chunks(I, counts, c0, c1, out=buf, threads=threads)
        buf = want if buf is None or want.shape[0] > buf.shape[0] else buf
        got = E[a:b].view(torch.int32).cpu().numpy().view(np.uint32)
        if not np.array_equal(got, want):
            bad = np.nonzero(np.any(got != want, axis=1))[0]
            c = int(np.searchsorted(offs, a + bad[0], side="right") - 1)
            raise AssertionError("chunks [%d, %d): %d edges differ, first at edge %d (chunk %d): got %s want %s"
                                 % (c0, c1, len(bad), a + bad[0], c, got[bad[0]], want[bad[0]]))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_undirected_gnm_n26_m31(kgref, seed):
    """All 2^31 edges byte for byte against the oracle, then the device-side
    invariants over the whole output."""
    import torch
    kg = require_gpu()
    n, m, P = 2**26, 2**31, 256
    E = kg.gnm(n, m, False, seed, P)
    counts = to_np_u64(kg.chunk_counts(kg.Instance(n, kg.GNM, False, m, 0.0, seed, P)))
    torch.cuda.synchronize()
    I = kgref.inst(n, m=m, directed=False, seed=seed, chunks=P)
    want_counts = kgref.chunk_counts(I)
    assert np.array_equal(counts, want_counts)
    offs = np.concatenate([[0], np.cumsum(want_counts.astype(np.int64))])
    assert offs[-1] == m
    _compare_all_chunks(torch, kgref, E, I, want_counts)
    _check_whole_output(torch, E, offs, n, False)
    del E
    torch.cuda.empty_cache()


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("directed,P,deg", [(True, 2**16, 16.0), (False, 256, 64.0)])
def test_gnp_n25(kgref, directed, P, deg, seed):
    """Both G(n,p) workloads (directed n = 2^25, p = 16/(n-1), 2^16 chunks;
    undirected p = 64/(n-1), 256 sections): every chunk count and every edge
    byte for byte against the oracle, then the device-side invariants."""
    import torch
    kg = require_gpu()
    n = 2**25
    p = deg / (n - 1)
    print("gnp n=2^25 directed=%s P=%d seed=%d" % (directed, P, seed), flush=True)
    E = kg.gnp(n, p, directed, seed, P)
    counts = to_np_u64(kg.chunk_counts(kg.Instance(n, kg.GNP, directed, 0, p, seed, P)))
    torch.cuda.synchronize()
    I = kgref.inst(n, p=p, directed=directed, seed=seed, chunks=P, model=1)
    want_counts = kgref.chunk_counts(I)
    assert np.array_equal(counts, want_counts)
    offs = np.concatenate([[0], np.cumsum(want_counts.astype(np.int64))])
    assert offs[-1] == E.shape[0]
    _compare_all_chunks(torch, kgref, E, I, want_counts, block=4096 if directed else 1024)
    _check_whole_output(torch, E, offs, n, directed)
    del E
    torch.cuda.empty_cache()


def test_batched_workload_sample(kgref):
    """96 instances drawn by the batched workload's recipe (n log-uniform in
    [2^10, 2^22], mean degree in [2, 64], half directed, half G(n,m)) in one
    kg_batch pass: every instance equals its own single call, and every edge
    of every instance equals the oracle's (chunk blocks of each instance)."""
    import torch
    kg = require_gpu()
    from paper_1710_07565_amd import workloads
    specs = workloads.batch_instances(count=96, base_seed=1, seed_fn=kg.instance_seed)
    insts = [kg.Instance(s.n, s.model, s.directed, s.m, s.p, s.seed, s.chunks) for s in specs]
    arena, offs = kg.batch(insts)
    torch.cuda.synchronize()
    O = to_np_u64(offs).astype(np.int64)
    for i, (s, I) in enumerate(zip(specs, insts)):
        seg = arena[O[i]:O[i + 1]]
        if I.model == kg.GNM:
            alone = kg.gnm(I.n, I.m, I.directed, I.seed, I.chunks)
        else:
            alone = kg.gnp(I.n, I.p, I.directed, I.seed, I.chunks)
        assert torch.equal(seg.view(torch.int32), alone.view(torch.int32)), i
        del alone
        ref = kgref.inst(s.n, m=s.m, p=s.p, directed=s.directed, seed=s.seed, chunks=s.chunks, model=s.model)
        cnt = kgref.chunk_counts(ref)
        assert int(cnt.astype(np.int64).sum()) == O[i + 1] - O[i], i
        _compare_all_chunks(torch, kgref, seg, ref, cnt, block=64)
    del arena
    torch.cuda.empty_cache()

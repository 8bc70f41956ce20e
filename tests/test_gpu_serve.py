"""Serving (continuous batching): requests arrive over time, are admitted
under an HBM budget into shared kg_batch launches on several streams, and
every served edge list equals the same request generated alone, byte for
byte (and the oracle's on a sample)."""
import numpy as np
import pytest

from gpu_util import require_gpu, to_np_u32

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone(kgref):
    import torch
    kg = require_gpu()
    from paper_1710_07565_amd import serve, workloads
    stream = workloads.request_stream(rate_per_s=3000.0, duration_s=0.15, base_seed=3, seed_fn=kg.instance_seed,
                                      log2n=(6, 14), degree=(2.0, 24.0), rng_seed=5)
    assert len(stream) > 200
    got = {}

    def on_done(r):
        got[r.rid] = to_np_u32(r.edges)

    # a budget of a few requests forces admission to wait for releases
    srv = serve.Server(budget_bytes=2 * 2**20, streams=3, max_batch=16, on_done=on_done)
    reqs, stats = serve.run_stream(srv, stream, warmup_s=0.0)
    assert stats["requests"] == len(stream)
    assert len(got) + srv.rejected == len(stream)
    assert srv.used == 0 and not srv.inflight and not srv.queue
    batched = sum(1 for r in reqs if r.batch is None and r.rid in got)
    assert batched == len(got)
    for r in reqs:
        if r.rid not in got:
            continue
        s = r.spec
        if s.model == kg.GNM:
            alone = kg.gnm(s.n, s.m, s.directed, s.seed, s.chunks)
        else:
            alone = kg.gnp(s.n, s.p, s.directed, s.seed, s.chunks)
        torch.cuda.synchronize()
        assert np.array_equal(to_np_u32(alone), got[r.rid]), r.rid
    for r in reqs[::17]:
        if r.rid not in got:
            continue
        s = r.spec
        want = kgref.generate(kgref.inst(s.n, m=s.m, p=s.p, directed=s.directed, seed=s.seed, chunks=s.chunks,
                                         model=s.model))
        assert np.array_equal(want, got[r.rid]), r.rid


def test_overlapping_launches_and_budget_accounting():
    import torch
    kg = require_gpu()
    from paper_1710_07565_amd import serve, workloads
    specs = workloads.batch_instances(count=60, base_seed=9, seed_fn=kg.instance_seed, log2n=(10, 16),
                                      degree=(4.0, 16.0))
    srv = serve.Server(budget_bytes=1 << 30, streams=4, max_batch=5, keep=True)
    reqs = [srv.submit(s) for s in specs]
    srv.drain()
    assert all(r.done is not None and r.edges is not None for r in reqs)
    used = srv.used
    assert used > 0
    for r in reqs:
        srv.release(r)
    assert srv.used == 0
    torch.cuda.synchronize()


def _checksum_np(E):
    """The edge-list checksum kg_edge_hash documents, in numpy uint64
    arithmetic: sum of mix(i * 0x9E3779B97F4A7C15 + (u << 32 | v))."""
    E = E.astype(np.uint64)
    i = np.arange(E.shape[0], dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = i * np.uint64(0x9E3779B97F4A7C15) + ((E[:, 0] << np.uint64(32)) | E[:, 1])
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
        return int(z.sum(dtype=np.uint64))


def test_edge_hash_matches_its_definition():
    """kg_edge_hash on lists of 0, 1, 2, odd and even lengths, starting at
    16-byte and at odd 8-byte addresses, equals the documented sum."""
    import torch
    kg = require_gpu()
    E = kg.gnm(3000, 100001, True, 9, 5)
    A = to_np_u32(E)
    for a, b in [(0, 0), (0, 1), (1, 2), (0, 2), (1, 100001), (0, 100001), (3, 77777), (2, 50000)]:
        h = kg.edge_hash(E[a:b])
        torch.cuda.synchronize()
        assert int(h.view(torch.int64).item()) & (2**64 - 1) == _checksum_np(A[a:b]), (a, b)


def test_client_checks_every_request_on_the_device():
    """With verification on, every served request is checksummed on the
    device before its memory is released, G(n,m) lengths are exact, and the
    sampled requests generated alone give the same checksum."""
    import torch
    kg = require_gpu()
    from paper_1710_07565_amd import serve, workloads
    stream = workloads.request_stream(rate_per_s=2000.0, duration_s=0.2, base_seed=4, seed_fn=kg.instance_seed,
                                      log2n=(8, 15), degree=(4.0, 32.0), rng_seed=8)
    kept = {}

    def on_done(r):
        if r.rid % 7 == 0:
            kept[r.rid] = to_np_u32(r.edges)

    srv = serve.Server(budget_bytes=64 * 2**20, streams=3, max_batch=32, on_done=on_done, verify=True,
                       alone_every=5)
    reqs, stats = serve.run_stream(srv, stream, warmup_s=0.0)
    served = [r for r in reqs if r.nedges is not None]
    assert stats["verify_failures"] == 0, srv.verify_failures[:5]
    assert stats["verified"] == len(served) > 100
    assert stats["checked_alone"] > 10
    assert srv.used == 0 and not srv.verifying
    for r in served:
        if r.rid in kept:
            assert r.hash == _checksum_np(kept[r.rid]), r.rid

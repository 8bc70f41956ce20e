"""GPU parity on universes of 2^53 slots and more (Sec. 1: far beyond
binary64's exact integers; slot counts reach the variates rounded to
nearest): a directed G(n,m) with n = 2^27 + 9 (about 2^54 slots) byte for
byte over all of its 2^31 + 77 edges, a directed G(n,p) at n = 2^27 + 9 with
mean out-degree 16 on every chunk count and a spread of whole chunks, an
undirected G(n,m) at n = 2^27 + 1000 (just above 2^53 slots) on every chunk
count and sampled chunks, and the element-wise variates at N near 2^60."""
import numpy as np
import pytest

from gpu_util import require_gpu, to_np_u32, to_np_u64
from test_gpu_fullsize import _check_whole_output, _compare_all_chunks

pytestmark = pytest.mark.gpu


def test_directed_gnm_beyond_2_53(kgref):
    import torch
    kg = require_gpu()
    n, m, P, seed = 2**27 + 9, 2**31 + 77, 2**10, 5
    assert n * (n - 1) >= 2**53
    print("directed G(n,m) n=2^27+9 m=2^31+77 P=1024", flush=True)
    E = kg.gnm(n, m, True, seed, P)
    counts = to_np_u64(kg.chunk_counts(kg.Instance(n, kg.GNM, True, m, 0.0, seed, P)))
    torch.cuda.synchronize()
    I = kgref.inst(n, m=m, directed=True, seed=seed, chunks=P)
    want_counts = kgref.chunk_counts(I)
    assert np.array_equal(counts, want_counts)
    offs = np.concatenate([[0], np.cumsum(want_counts.astype(np.int64))])
    _compare_all_chunks(torch, kgref, E, I, want_counts, block=64)
    _check_whole_output(torch, E, offs, n, True)
    del E
    torch.cuda.empty_cache()


def test_directed_gnp_beyond_2_53(kgref):
    import torch
    kg = require_gpu()
    n, P, seed = 2**27 + 9, 2**10, 3
    p = 16.0 / (n - 1)
    print("directed G(n,p) n=2^27+9 d=16 P=1024", flush=True)
    E = kg.gnp(n, p, True, seed, P)
    counts = to_np_u64(kg.chunk_counts(kg.Instance(n, kg.GNP, True, 0, p, seed, P)))
    torch.cuda.synchronize()
    I = kgref.inst(n, p=p, directed=True, seed=seed, chunks=P)
    want_counts = kgref.chunk_counts(I)
    assert np.array_equal(counts, want_counts)
    offs = np.concatenate([[0], np.cumsum(want_counts.astype(np.int64))])
    assert E.shape[0] == int(offs[-1])
    rng = np.random.default_rng(2)
    for c in [0, 1, P // 2, P - 1] + [int(x) for x in rng.integers(0, P, 12)]:
        want = kgref.chunk_edges(I, c, int(want_counts[c]))
        got = to_np_u32(E[int(offs[c]):int(offs[c + 1])])
        assert np.array_equal(got, want), c
    _check_whole_output(torch, E, offs, n, True)
    del E
    torch.cuda.empty_cache()


def test_undirected_gnm_beyond_2_53(kgref):
    import torch
    kg = require_gpu()
    n, m, P, seed = 2**27 + 1000, 2**30 + 5, 64, 9
    assert n * (n - 1) // 2 >= 2**53
    print("undirected G(n,m) n=2^27+1000 m=2^30+5 P=64", flush=True)
    E = kg.gnm(n, m, False, seed, P)
    counts = to_np_u64(kg.chunk_counts(kg.Instance(n, kg.GNM, False, m, 0.0, seed, P)))
    torch.cuda.synchronize()
    I = kgref.inst(n, m=m, directed=False, seed=seed, chunks=P)
    want_counts = kgref.chunk_counts(I)
    assert np.array_equal(counts, want_counts)
    offs = np.concatenate([[0], np.cumsum(want_counts.astype(np.int64))])
    C = len(want_counts)
    rng = np.random.default_rng(4)
    # the first chunk (a diagonal triangle), the last, and random ones
    for c in [0, 1, C - 1] + [int(x) for x in rng.integers(0, C, 10)]:
        want = kgref.chunk_edges(I, c, int(want_counts[c]))
        got = to_np_u32(E[int(offs[c]):int(offs[c + 1])])
        assert np.array_equal(got, want), c
    _check_whole_output(torch, E, offs, n, False)
    del E
    torch.cuda.empty_cache()


def test_variates_beyond_2_53(kgref):
    """Hypergeometric and binomial variates with N between 2^53 and 2^63 on
    the device equal the oracle's, element by element (kg_eval records:
    N, K or p, k, seed, stream word, tag)."""
    import torch
    kg = require_gpu()
    rng = np.random.default_rng(11)
    n = 30000
    N = rng.integers(2**53, 2**63, n).astype(np.uint64)
    K = np.minimum((N.astype(np.float64) * rng.uniform(0.0, 1.0, n)).astype(np.uint64), N)
    k = np.where(rng.uniform(size=n) < 0.3, rng.integers(0, 17, n),
                 (2.0 ** rng.uniform(4, 40, n)).astype(np.int64)).astype(np.uint64)
    seeds = rng.integers(0, 2**63, n).astype(np.uint64)
    ab = rng.integers(0, 2**40, n).astype(np.uint64)
    rec = np.stack([N, K, k, seeds, ab, np.full(n, 4, np.uint64)], axis=1)
    got = kg.eval_device(5, torch.from_numpy(rec.view(np.int64)).cuda(), n, torch.int64, 1)
    torch.cuda.synchronize()
    got = got.cpu().numpy().view(np.uint64)
    want = kgref.eval_many(5, rec, np.uint64, 1)
    bad = np.nonzero(got[:, 0] != want[:, 0])[0]
    assert len(bad) == 0, rec[bad[:5]]
    # binomial: means from 2^-7 to 2^40 (waiting times and ratio of uniforms)
    mean = 2.0 ** rng.uniform(-7, 40, n)
    p = np.clip(mean / N.astype(np.float64), 0.0, 1.0)
    rec = np.stack([N, p.view(np.uint64), np.zeros(n, np.uint64), seeds, ab, np.full(n, 3, np.uint64)], axis=1)
    got = kg.eval_device(6, torch.from_numpy(rec.view(np.int64)).cuda(), n, torch.int64, 1)
    torch.cuda.synchronize()
    got = got.cpu().numpy().view(np.uint64)
    want = kgref.eval_many(6, rec, np.uint64, 1)
    bad = np.nonzero(got[:, 0] != want[:, 0])[0]
    assert len(bad) == 0, rec[bad[:5]]

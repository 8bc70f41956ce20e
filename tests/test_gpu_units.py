"""GPU building blocks against the oracle, element by element, bit for bit:
Philox4x32-10, log, log1p, ln k! differences, the hypergeometric and binomial
variates (Sec. 2.2, 4.3), and the binary64 sqrt / division the variates rely
on (checked for correct rounding with exact rational arithmetic)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kg():
    return require_gpu()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _eval(kg, fn, rec, dtype, width):
    import torch
    d = _dev(rec)
    out = kg.eval_device(fn, d, rec.shape[0], dtype, width)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_philox_bits(kg, kgref):
    import torch
    rng = np.random.default_rng(1)
    rec = rng.integers(0, 2**32, size=(200000, 6), dtype=np.uint64).astype(np.uint32)
    rec[:1000, 0] = np.arange(1000)           # structured counters (j, a, b, tag)
    rec[:1000, 3] = rng.integers(1, 7, 1000)
    got = _eval(kg, 1, rec.view(np.int32), torch.int32, 4).view(np.uint32)
    want = kgref.eval_many(1, rec, np.uint32, 4)
    assert np.array_equal(got, want)


def test_log_log1p_bits(kg, kgref):
    import torch
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.uniform(0, 1, 300000), np.exp(rng.uniform(-700, 700, 300000)),
                        rng.integers(1, 2**53, 200000).astype(np.float64),
                        1 + rng.uniform(-1e-3, 1e-3, 100000), [2.0**-1022, 1.0, 2.0, 1.4142135623730951]])
    got = _eval(kg, 2, x, torch.float64, 1)
    want = kgref.eval_many(2, x, np.float64, 1)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    y = np.concatenate([rng.uniform(-0.999, 5, 300000), -np.exp(rng.uniform(-60, -1, 100000)),
                        np.exp(rng.uniform(-60, 3, 100000)), [-0.25, 0.25, 0.0]])
    got = _eval(kg, 3, y, torch.float64, 1)
    want = kgref.eval_many(3, y, np.float64, 1)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def test_sqrt_and_division_correctly_rounded(kg):
    """The variates assume IEEE binary64 sqrt and / are correctly rounded on
    the device (they are on the host); check exactly with rationals."""
    import torch
    rng = np.random.default_rng(3)
    a = np.concatenate([np.exp(rng.uniform(-30, 80, 20000)), rng.integers(1, 2**53, 5000).astype(np.float64),
                        rng.uniform(0.5, 2.0, 5000)])
    b = np.concatenate([np.exp(rng.uniform(-30, 80, 20000)), rng.integers(1, 2**40, 5000).astype(np.float64),
                        rng.uniform(1.0, 3.0, 5000)])
    rec = np.stack([a, b], axis=1)
    got = _eval(kg, 7, rec, torch.float64, 2)
    # host binary64 is correctly rounded: bitwise equality with numpy
    assert np.array_equal(got[:, 0].view(np.uint64), np.sqrt(a).view(np.uint64))
    assert np.array_equal(got[:, 1].view(np.uint64), (a / b).view(np.uint64))
    # and an exact check on a sample: |r - sqrt(a)| <= ulp/2, |q - a/b| <= ulp/2
    for i in range(0, len(a), 97):
        r, q = float(got[i, 0]), float(got[i, 1])
        A, B = Fraction(float(a[i])), Fraction(float(b[i]))
        h = Fraction(math.ulp(r)) / 2
        assert (Fraction(r) - h) ** 2 <= A <= (Fraction(r) + h) ** 2
        assert abs(Fraction(q) - A / B) <= Fraction(math.ulp(q)) / 2


def test_lnf_diff_bits(kg, kgref):
    import torch
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.integers(0, 3000, 100000), rng.integers(0, 2**52, 100000),
                        rng.integers(0, 2**32, 50000)]).astype(np.uint64)
    d = np.concatenate([rng.integers(0, 3000, 100000), rng.integers(0, 10**6, 100000),
                        rng.integers(0, 2**31, 50000)]).astype(np.uint64)
    y = np.minimum(x + d, np.uint64(2**53 - 1))
    rec = np.stack([x, y], axis=1)
    rec[::2] = rec[::2, ::-1]
    got = _eval(kg, 4, rec.view(np.int64), torch.float64, 1)
    want = kgref.eval_many(4, rec, np.float64, 1)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def _hyp_records(rng, n):
    N = np.concatenate([rng.integers(1, 200, n // 4), rng.integers(1, 10**6, n // 4),
                        rng.integers(1, 2**40, n // 4), rng.integers(2**40, 2**53 - 1, n - 3 * (n // 4))])
    N = N.astype(np.uint64)
    K = (rng.uniform(0, 1, n) * N.astype(np.float64)).astype(np.uint64)
    k = (rng.uniform(0, 1, n) ** 3 * N.astype(np.float64)).astype(np.uint64)
    K = np.minimum(K, N)
    k = np.minimum(k, N)
    seed = rng.integers(0, 2**63, n).astype(np.uint64)
    ab = rng.integers(0, 2**63, n).astype(np.uint64)
    tag = rng.integers(1, 7, n).astype(np.uint64)
    return np.stack([N, K, k, seed, ab, tag], axis=1)


def test_hyp_bits(kg, kgref):
    import torch
    rng = np.random.default_rng(5)
    rec = _hyp_records(rng, 60000)
    # tree-shaped calls as the generator makes them: K ~ N/2, large k
    N = rng.integers(2**30, 2**52, 20000).astype(np.uint64)
    tree = np.stack([N, N // 2, (N.astype(np.float64) * 2.0**-21).astype(np.uint64),
                     rng.integers(0, 2**63, 20000).astype(np.uint64),
                     rng.integers(0, 2**40, 20000).astype(np.uint64), np.full(20000, 4, np.uint64)], axis=1)
    rec = np.concatenate([rec, tree])
    got = _eval(kg, 5, rec.view(np.int64), torch.int64, 1).view(np.uint64)
    want = kgref.eval_many(5, rec, np.uint64, 1)
    bad = np.nonzero(got[:, 0] != want[:, 0])[0]
    assert len(bad) == 0, rec[bad[:5]]


def test_bin_bits(kg, kgref):
    import torch
    rng = np.random.default_rng(6)
    n = 60000
    N = np.concatenate([rng.integers(0, 100, n // 3), rng.integers(0, 10**7, n // 3),
                        rng.integers(0, 2**52, n - 2 * (n // 3))]).astype(np.uint64)
    mean = np.exp(rng.uniform(-3, 14, n))
    p = np.clip(mean / np.maximum(N.astype(np.float64), 1.0), 0, 1)
    p[::17] = rng.uniform(0, 1, len(p[::17]))
    p[::101] = 0.0
    p[::103] = 1.0
    rec = np.stack([N, p.view(np.uint64), np.zeros(n, np.uint64), rng.integers(0, 2**63, n).astype(np.uint64),
                    rng.integers(0, 2**63, n).astype(np.uint64), np.full(n, 3, np.uint64)], axis=1)
    got = _eval(kg, 6, rec.view(np.int64), torch.int64, 1).view(np.uint64)
    want = kgref.eval_many(6, rec, np.uint64, 1)
    bad = np.nonzero(got[:, 0] != want[:, 0])[0]
    assert len(bad) == 0, rec[bad[:5]]

"""Pins of the oracle's hypergeometric and binomial variates (Sec. 2.2:
sample counts of sub-universes are hypergeometric; variates by
acceptance-rejection; Sec. 4.3: binomial chunk counts for G(n,p)).

Each law is checked against scipy's exact pmf by chi-square on fixed seeds,
special cases that reduce to a known answer, moments at the 2^51 scale of
the largest workload, and the ratio-of-uniforms envelope inequality."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

D1 = 2 * math.sqrt(2 / math.e)
D2 = 3 - 2 * math.sqrt(3 / math.e)


def chi2_pvalue(samples, pmf_fn, support):
    lo, hi = support
    xs = np.arange(lo, hi + 1)
    probs = np.array([pmf_fn(x) for x in xs])
    n = len(samples)
    counts = np.bincount(np.asarray(samples, dtype=np.int64) - lo, minlength=hi - lo + 1)
    assert counts.sum() == n and len(counts) == hi - lo + 1
    # merge bins of small expectation into neighbours
    exp = probs * n
    obs_b, exp_b = [], []
    acc_o = acc_e = 0.0
    for o, e in zip(counts, exp):
        acc_o += o
        acc_e += e
        if acc_e >= 8:
            obs_b.append(acc_o)
            exp_b.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0 or acc_o > 0:
        if exp_b:
            obs_b[-1] += acc_o
            exp_b[-1] += acc_e
        else:
            obs_b.append(acc_o)
            exp_b.append(acc_e)
    obs_b, exp_b = np.array(obs_b), np.array(exp_b)
    exp_b *= obs_b.sum() / exp_b.sum()
    if len(obs_b) < 2:
        return 1.0
    return stats.chisquare(obs_b, exp_b).pvalue


HYP_GRID = [
    # (N, K, k): direct simulation (k <= 16 after the symmetries), ratio of
    # uniforms, and every symmetry (k > N/2, K > N/2, k > K)
    (20, 7, 5), (50, 25, 10), (100, 90, 8), (100, 10, 95), (1000, 500, 16),
    (1000, 300, 200), (1000, 700, 900), (1000, 50, 400), (10**6, 3 * 10**5, 5000),
    (10**9, 10**8, 10**5), (64, 32, 32), (35, 17, 17), (2**20, 2**19, 2**10),
]


@pytest.mark.parametrize("N,K,k", HYP_GRID)
def test_hyp_matches_pmf(kgref, N, K, k):
    nsamp = 12000
    xs = [kgref.hyp(N, K, k, seed=7, a=i, b=3, tag=kgref.TAG_TTREE) for i in range(nsamp)]
    lo, hi = max(0, k - (N - K)), min(k, K)
    assert min(xs) >= lo and max(xs) <= hi
    rv = stats.hypergeom(N, K, k)
    mean, sd = rv.mean(), rv.std()
    lo2, hi2 = max(lo, int(mean - 12 * sd) - 1), min(hi, int(mean + 12 * sd) + 1)
    xs = np.clip(xs, lo2, hi2)
    pv = chi2_pvalue(xs, rv.pmf, (lo2, hi2))
    assert pv > 1e-5, pv


def test_hyp_special_cases(kgref):
    for N in [1, 2, 5, 100, 2**40]:
        for k in sorted({0, 1, N // 3, N // 2, N - 1, N}):
            assert kgref.hyp(N, 0, k, 1) == 0
            assert kgref.hyp(N, N, k, 1) == k
        for K in sorted({0, 1, N // 3, N - 1, N}):
            assert kgref.hyp(N, K, 0, 2) == 0
            assert kgref.hyp(N, K, N, 2) == K
    assert kgref.hyp(0, 0, 0, 1) == 0


@pytest.mark.parametrize("N,K,k", [(2**51 - 2**25, 2**50, 2**31), (2**51, 2**36, 2**31),
                                    (2**35, 2**34, 65536), (2**50, 3 * 2**48, 2**30 + 12345)])
def test_hyp_moments_at_scale(kgref, N, K, k):
    n = 3000
    xs = np.array([kgref.hyp(N, K, k, seed=11, a=i) for i in range(n)], dtype=np.float64)
    mu = k * K / N
    var = k * (K / N) * (1 - K / N) * (N - k) / (N - 1)
    z = (xs.mean() - mu) / math.sqrt(var / n)
    assert abs(z) < 5, z
    # sample variance: chi-square with n-1 dof, normal approximation
    r = xs.var(ddof=1) / var
    assert abs(r - 1) < 5 * math.sqrt(2 / (n - 1)), r


BIN_GRID = [(1, 0.5), (10, 0.3), (100, 0.05), (1000, 0.015), (200, 0.3), (10**5, 0.01),
            (10**4, 0.7), (50, 0.9), (2**40, 1e-11), (2**34, 16 / (2**25 - 1)), (3000, 0.5)]


@pytest.mark.parametrize("N,p", BIN_GRID)
def test_bin_matches_pmf(kgref, N, p):
    nsamp = 12000
    xs = [kgref.bin(N, p, seed=5, a=i) for i in range(nsamp)]
    assert min(xs) >= 0 and max(xs) <= N
    rv = stats.binom(N, p)
    mean, sd = rv.mean(), rv.std()
    lo2, hi2 = max(0, int(mean - 12 * sd) - 1), min(N, int(mean + 12 * sd) + 1)
    xs = np.clip(xs, lo2, hi2)
    assert chi2_pvalue(xs, rv.pmf, (lo2, hi2)) > 1e-5


def test_bin_special_cases(kgref):
    for N in [0, 1, 7, 2**52]:
        assert kgref.bin(N, 0.0, 1) == 0
        assert kgref.bin(N, 1.0, 1) == N
    assert kgref.bin(0, 0.5, 1) == 0


@pytest.mark.parametrize("N,p", [(2**51 - 2**25, 2**-20), (2**49, 64 / (2**25 - 1)), (2**40, 0.5)])
def test_bin_moments_at_scale(kgref, N, p):
    n = 3000
    xs = np.array([kgref.bin(N, p, seed=3, a=i) for i in range(n)], dtype=np.float64)
    mu, var = N * p, N * p * (1 - p)
    assert abs((xs.mean() - mu) / math.sqrt(var / n)) < 5
    assert abs(xs.var(ddof=1) / var - 1) < 5 * math.sqrt(2 / (n - 1))


def _envelope_ratio(xs, logf, mu, var):
    """Ratio-of-uniforms region {(u,v): u <= sqrt(f(floor(a + v/u))/f(M))}
    lies in [0,1] x [-h/2, h/2] iff sqrt(f(x)/f(M)) * max(|x-a|, |x+1-a|) <= h/2
    for every x of the support, with a = mu + 1/2 and h = D1 sqrt(var+1/2) + D2.
    Returns max over xs of the left side divided by h/2."""
    a = mu + 0.5
    h = D1 * math.sqrt(var + 0.5) + D2
    xs = np.asarray(xs, dtype=np.float64)
    logf = np.asarray(logf, dtype=np.float64)
    w = np.exp(0.5 * (logf - logf.max())) * np.maximum(np.abs(xs - a), np.abs(xs + 1 - a))
    return float(w.max() / (h / 2))


def test_hyp_envelope_exhaustive_small():
    worst = 0.0
    for N in range(34, 121):
        for K in range(17, N // 2 + 1):
            for k in range(17, K + 1):
                denom = math.comb(N, k)
                xs = range(0, k + 1)
                logf = [math.log(Fraction(math.comb(K, x) * math.comb(N - K, k - x), denom))
                        for x in xs]
                mu = k * K / N
                var = k * (K / N) * (1 - K / N) * (N - k) / (N - 1)
                worst = max(worst, _envelope_ratio(list(xs), logf, mu, var))
    assert worst < 1.0, worst


def test_hyp_envelope_sampled_large():
    rng = np.random.default_rng(9)
    worst = 0.0
    for _ in range(300):
        N = int(rng.integers(200, 10**7))
        K = int(rng.integers(17, N // 2 + 1))
        k = int(rng.integers(17, K + 1))
        rv = stats.hypergeom(N, K, k)
        mu, var = rv.mean(), rv.var()
        sd = math.sqrt(var)
        lo, hi = max(0, int(mu - 40 * sd) - 2), min(k, int(mu + 40 * sd) + 2)
        xs = np.arange(lo, hi + 1)
        worst = max(worst, _envelope_ratio(xs, rv.logpmf(xs), mu, var))
    assert worst < 1.0, worst


def test_bin_envelope():
    worst = 0.0
    for N in list(range(16, 400)) + [1000, 5000, 10**5, 10**7]:
        for p in [0.5, 0.45, 0.3, 0.2, 0.1, 0.05, 0.02, 16.0 / N, 17.0 / N, 0.5 - 1e-9]:
            if not (0 < p <= 0.5) or N * p < 16:
                continue
            rv = stats.binom(N, p)
            mu, var = N * p, N * p * (1 - p)
            sd = math.sqrt(var)
            lo, hi = max(0, int(mu - 40 * sd) - 2), min(N, int(mu + 40 * sd) + 2)
            xs = np.arange(lo, hi + 1)
            worst = max(worst, _envelope_ratio(xs, rv.logpmf(xs), mu, var))
    assert worst < 1.0, worst


def test_variates_depend_only_on_their_stream(kgref):
    # Same stream id, same value; a different id or tag, independent values.
    a = [kgref.hyp(10**6, 4 * 10**5, 3000, 42, a=i, tag=kgref.TAG_DTREE) for i in range(50)]
    b = [kgref.hyp(10**6, 4 * 10**5, 3000, 42, a=i, tag=kgref.TAG_DTREE) for i in range(50)]
    c = [kgref.hyp(10**6, 4 * 10**5, 3000, 42, a=i, tag=kgref.TAG_UTREE) for i in range(50)]
    assert a == b and a != c

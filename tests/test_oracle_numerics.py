"""Pins of the oracle's floating-point kernel: log, log1p, ln k! and stable
differences of ln k!, checked against 40-digit decimal arithmetic (which the
oracle does not use).  These feed the acceptance tests of the variates
(Sec. 2.2: acceptance-rejection samplers)."""
import math
from decimal import Decimal, getcontext

import numpy as np

getcontext().prec = 50


def dln(x):
    return Decimal(x).ln()


def ulps(got, exact):
    return abs(Decimal(got) - exact) / Decimal(math.ulp(float(exact)))


def test_log_special_values(kgref):
    assert kgref.log(1.0) == 0.0
    for k in range(-1000, 1000, 37):
        x = math.ldexp(1.0, k)
        assert ulps(kgref.log(x), dln(x)) <= 1
    # range ends the samplers reach: uniforms in (2^-53, 1), counts below 2^53
    for x in [2.0**-53, 0.5 * 2.0**-52, 1 - 2.0**-53, 2.0**53 - 1, 1.0 + 2.0**-52, math.sqrt(2.0),
              math.sqrt(0.5), 0.70710678118654746, 1.4142135623730954]:
        assert ulps(kgref.log(x), dln(x)) <= 2, x


def test_log_random_within_two_ulp(kgref):
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(0, 1, 3000), np.exp(rng.uniform(-40, 40, 3000)),
                         rng.integers(1, 2**53, 2000).astype(np.float64),
                         1.0 + rng.uniform(-1e-6, 1e-6, 1000)])
    worst = 0
    for x in xs:
        x = float(x)
        if x <= 0:
            continue
        e = ulps(kgref.log(x), dln(x))
        worst = max(worst, e)
    assert worst <= 2, worst


def test_log1p_random(kgref):
    rng = np.random.default_rng(2)
    xs = np.concatenate([-np.exp(rng.uniform(-50, math.log(0.5), 3000)),
                         np.exp(rng.uniform(-50, 10, 3000)), [-0.25, 0.25, -0.2499999, 0.2499999]])
    worst = 0
    for x in xs:
        x = float(x)
        exact = (Decimal(1) + Decimal(x)).ln()
        worst = max(worst, ulps(kgref.log1p(x), exact))
    assert worst <= 4, worst


def _lnf_exact_small(k):
    s = Decimal(0)
    for i in range(2, k + 1):
        s += Decimal(i).ln()
    return s


BERN = [Decimal(1) / 6, Decimal(-1) / 30, Decimal(1) / 42, Decimal(-1) / 30, Decimal(5) / 66,
        Decimal(-691) / 2730, Decimal(7) / 6]


def _lngamma_dec(z):
    """ln Gamma(z) for z >= 1000 from the full Stirling series in 50 digits."""
    z = Decimal(z)
    two_pi = 2 * Decimal("3.14159265358979323846264338327950288419716939937510")
    r = (z - Decimal("0.5")) * z.ln() - z + two_pi.ln() / 2
    zp = z
    z2 = z * z
    for k, b in enumerate(BERN, start=1):
        r += b / (2 * k * (2 * k - 1) * zp)
        zp *= z2
    return r


def _lnf_exact(k):
    if k < 1100:
        return _lnf_exact_small(k)
    return _lngamma_dec(k + 1)


def test_lnf_table_and_stirling(kgref):
    assert kgref.lnf(0) == 0.0 and kgref.lnf(1) == 0.0
    for k in [2, 3, 10, 100, 500, 1023, 1024]:
        assert abs(Decimal(kgref.lnf(k)) - _lnf_exact_small(k)) < Decimal("1e-9"), k
    for k in [1025, 2000, 10**5, 10**9, 2**40, 2**52]:
        ex = _lnf_exact(k)
        assert abs(Decimal(kgref.lnf(k)) - ex) / ex < Decimal("1e-13"), k
    # Gamma function values from the standard library agree to its accuracy
    for k in [5, 50, 5000]:
        assert math.isclose(kgref.lnf(k), math.lgamma(k + 1), rel_tol=1e-13)


def test_lnf_diff_large_arguments_stay_accurate(kgref):
    """Near 2^51 one ulp of ln k! is 16: only a stable difference keeps
    the acceptance ratio meaningful."""
    rng = np.random.default_rng(3)
    cases = [(2**51 - 5, 2**51 + 1000), (2**50, 2**50 + 1), (2**31, 2**31 + 70000),
             (1024, 5000), (10, 3000), (0, 2000), (1000, 1024), (700, 1030), (2**52, 2**52 - 77)]
    for _ in range(40):
        a = int(rng.integers(0, 2**52))
        d = int(rng.integers(1, 10**6))
        cases.append((a, a + d))
    for x, y in cases:
        got = Decimal(kgref.lnf_diff(x, y))
        ex = _lnf_exact(y) - _lnf_exact(x)
        tol = max(abs(ex) * Decimal("1e-14"), Decimal("2e-9"))
        assert abs(got - ex) <= tol, (x, y, float(got), float(ex))
        assert kgref.lnf_diff(y, x) == -kgref.lnf_diff(x, y)
    assert kgref.lnf_diff(12345, 12345) == 0.0

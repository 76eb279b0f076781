"""Pins of the rejection samplers' log-scale acceptance (BTRD and PTRS,
Hormann 1993) against exact log pmfs from mpmath, CPU only.

The chi-square tests cannot see an error of order 1e-6 in a log-scale test
that only a few percent of draws reach; these tests compare each decision
with the exact one at uniforms placed just beside the exact boundary."""
import math

import mpmath
import pytest

import oracle

mpmath.mp.dps = 50


def exact_fc(k):
    """log k! - [(k + 1/2) log(k+1) - (k+1) + log(2 pi)/2] at 50 digits."""
    k = mpmath.mpf(k)
    return mpmath.loggamma(k + 1) - ((k + mpmath.mpf(0.5)) * mpmath.log(k + 1) - (k + 1)
                                     + mpmath.log(2 * mpmath.pi) / 2)


@pytest.mark.parametrize("k", list(range(10)) + [10, 11, 12, 15, 20, 50, 137, 1000, 1e5, 1e7])
def test_stirling_tail_vs_mpmath(k):
    """Below 10 the oracle's fc is lgamma-exact; from 10 on it is the Stirling
    series 1/(12z) - 1/(360z^3) + 1/(1260z^5), z = k + 1, whose alternating
    remainder is bounded by the first dropped term 1/(1680 z^7)."""
    got = oracle.stirling_tail(k)
    ref = exact_fc(k)
    z = k + 1.0
    bound = 1e-14 if k < 10 else 1.0 / (1680.0 * z ** 7) + 4e-16 / z
    assert abs(got - float(ref)) <= bound, (k, got, float(ref))


def _log_binom_ratio(n, p, k, m):
    """log f(k) - log f(m), f the Binomial(n, p) pmf, at 50 digits (p is the
    double the sampler receives, taken exactly)."""
    n, p, k, m = (mpmath.mpf(v) for v in (n, p, k, m))
    q = 1 - p
    lf = lambda j: (mpmath.loggamma(n + 1) - mpmath.loggamma(j + 1) - mpmath.loggamma(n - j + 1)
                    + j * mpmath.log(p) + (n - j) * mpmath.log(q))
    return lf(k) - lf(m)


def _btrd_cases():
    """(n, p, k) with n p >= 10, p <= 1/2 and |k - m| > 15, with the exact log
    ratio above -20 (every rescaled uniform of a try can reach it).  The
    first rows are tries at k = 0 with small p, where the squeeze bounds
    t -+ rho are close to the exact ratio."""
    cases = [(1000, 0.02, 0), (2000, 0.01, 0), (10000, 0.002, 0), (500, 0.05, 1)]
    for n, p in [(21, 0.5), (40, 0.3), (60, 0.25), (100, 0.1), (200, 0.45), (300, 0.05),
                 (1000, 0.3), (5000, 0.01), (1e5, 0.37), (1e6, 0.001), (2e6, 0.5)]:
        m = math.floor((n + 1) * p)
        sd = math.sqrt(n * p * (1 - p))
        for d in (16, 17, 20, 25, 1.5 * sd, 2.5 * sd, 4 * sd, 5.5 * sd):
            for sgn in (-1, 1):
                k = m + sgn * math.ceil(d)
                if 0 <= k <= n and abs(k - m) > 15:
                    cases.append((n, p, k))
    return cases


@pytest.mark.parametrize("n,p,k", _btrd_cases())
def test_btrd_log_scale_decision_vs_exact_ratio(n, p, k):
    m = math.floor((n + 1) * p)
    L = _log_binom_ratio(n, p, k, m)
    if L < -20:
        pytest.skip("ratio below every reachable rescaled uniform")
    # the decision must be exact once v is 1e-9 (in log) away from the
    # boundary: rounding is ~1e-13 there and the Stirling remainder < 1e-10
    for delta in (-1e-5, -1e-7, -1e-8, -1e-9, 1e-9, 1e-8, 1e-7, 1e-5, 0.3, -0.3, 3.0, -3.0):
        v = float(mpmath.exp(L + delta))
        if not (0.0 < v):
            continue
        assert oracle.btrd_log_accept(n, p, k, v) == (delta < 0), (n, p, k, delta)


def _ptrs_cases():
    out = []
    for lam in (10.0, 10.5, 31.0, 100.0, 1234.5, 1e5):
        sl = math.sqrt(lam)
        for d in (-3.5, -2, -1, 0, 1, 2.5, 4):
            k = math.floor(lam + d * sl)
            if k >= 0:
                for us in (0.02, 0.1, 0.3, 0.49):
                    out.append((lam, us, k))
    return out


@pytest.mark.parametrize("lam,us,k", _ptrs_cases())
def test_ptrs_decision_vs_exact_pmf(lam, us, k):
    """PTRS accepts k when v * alpha / (a / us^2 + b) <= pmf(k).  The hat
    constants a, b, 1/alpha are Hormann's; the pmf side is checked against
    mpmath's exact log Poisson pmf."""
    b = 0.931 + 2.53 * math.sqrt(lam)
    a = -0.059 + 0.02483 * b
    inv_alpha = 1.1239 + 1.1328 / (b - 3.4)
    lam_m = mpmath.mpf(lam)
    log_pmf = -lam_m + k * mpmath.log(lam_m) - mpmath.loggamma(k + 1)
    log_hat = mpmath.log(mpmath.mpf(inv_alpha)) - mpmath.log(mpmath.mpf(a) / mpmath.mpf(us) ** 2 + mpmath.mpf(b))
    Lv = log_pmf - log_hat            # boundary for log v
    for delta in (-1e-6, -1e-8, 1e-8, 1e-6):
        v = float(mpmath.exp(Lv + delta))
        if not (0.0 < v < 1.0):
            continue
        assert oracle.ptrs_log_accept(lam, us, v, k) == (delta < 0), (lam, us, k, delta)

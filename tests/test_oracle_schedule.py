"""Pins of the noise schedule (Section IV-B): exact rational products."""
from fractions import Fraction

import numpy as np

from oracle import schedule


def _exact_alpha_bar(N, bmin, bmax):
    bmin, bmax = Fraction(bmin), Fraction(bmax)
    out, prod = [Fraction(1)], Fraction(1)
    for i in range(N):
        beta = bmin + (bmax - bmin) * Fraction(i, N - 1) if N > 1 else bmin
        prod *= 1 - beta
        out.append(prod)
    return out


def test_alpha_bar_matches_exact_rational_product():
    for N in (1, 2, 7, 100):
        ab = schedule.alpha_bar(N, 1e-4, 1e-2)
        ex = _exact_alpha_bar(N, "0.0001", "0.01")
        assert ab[0] == 1.0
        for i in range(N + 1):
            assert abs(ab[i] - float(ex[i])) <= 1e-14 * float(ex[i])


def test_endpoints_and_value_at_100_steps():
    b = schedule.betas(100, 1e-4, 1e-2)
    assert b[0] == 1e-4 and abs(b[-1] - 1e-2) < 1e-18
    ab = schedule.alpha_bar(100, 1e-4, 1e-2)
    # log alpha-bar_N = sum log(1 - beta) bracketed by -sum(beta) - sum(beta^2)/2 * (1 +- 0.1)
    s1, s2 = b.sum(), (b ** 2).sum()
    assert -s1 - 0.6 * s2 <= np.log(ab[-1]) <= -s1 - 0.5 * s2
    assert abs(ab[-1] - 0.6024803) < 5e-7


def test_step_scalars_relations():
    ms, sg, os_ = schedule.step_scalars(100, 1e-4, 1e-2)
    ex = _exact_alpha_bar(100, "0.0001", "0.01")
    for i in (1, 50, 100):
        a = float(ex[i])
        assert abs(ms[i] ** 2 * a - 1) < 1e-13
        assert abs(sg[i] ** 2 - (1 / a - 1)) < 1e-13
        assert abs(os_[i] ** 2 - float(ex[i - 1])) < 1e-13
    # sigma_1 = sqrt(beta_1 / (1 - beta_1)) since alpha-bar_1 = 1 - beta_1
    assert abs(sg[1] - np.sqrt(1e-4 / (1 - 1e-4))) < 1e-12 * sg[1]

"""The bounds behind the integrator's exp-free Poisson counts (the CDF
inversion of Sec. IV.B): for mu >= 0,
    e^-mu <= 1 - mu + mu^2/2,           e^-mu (1 + mu) >= 1 - mu^2/2,
    e^-mu (1 + mu) <= 1 - mu^2/2 + mu^3/3,   e^-mu (1 + mu + mu^2/2) >= 1 - mu^3/6,
checked at 50 significant digits, and the FP64 evaluation of each side within
the 2^-45 margin the kernel leaves."""
from decimal import Decimal, getcontext

import numpy as np

getcontext().prec = 50


def _mus():
    grid = [Decimal(k) / Decimal(1000) for k in range(1, 1001)]
    grid += [Decimal(10) ** Decimal(-e) for e in range(4, 16)]
    grid += [Decimal(1) - Decimal(10) ** Decimal(-e) for e in range(3, 12)]
    return grid


def test_cdf_bounds_hold_exactly():
    for mu in _mus():
        e = (-mu).exp()
        m2, m3 = mu * mu, mu * mu * mu
        assert e <= 1 - mu + m2 / 2
        assert e * (1 + mu) >= 1 - m2 / 2
        assert e * (1 + mu) <= 1 - m2 / 2 + m3 / 3
        assert e * (1 + mu + m2 / 2) >= 1 - m3 / 6


def test_fp64_bounds_within_margin():
    margin = 2.0 ** -45
    for mu_d in _mus():
        mu = float(mu_d)
        e = (-mu_d).exp()
        h, c = 0.5 * mu * mu, mu * (0.5 * mu * mu)
        exact = {
            "b0": 1 - mu_d + mu_d * mu_d / 2,
            "b1": 1 - mu_d * mu_d / 2,
            "b2": 1 - mu_d * mu_d / 2 + mu_d ** 3 / 3,
            "b3": 1 - mu_d ** 3 / 6,
        }
        fp = {"b0": (1.0 - mu) + h, "b1": 1.0 - h, "b2": (1.0 - h) + c * (2.0 / 3.0),
              "b3": 1.0 - c * (1.0 / 3.0)}
        for k in exact:
            assert abs(Decimal(fp[k]) - exact[k]) < Decimal(margin) / 8, (k, mu)
        # and the CDF terms the inversion would compute stay on their side
        assert Decimal(np.exp(-mu)) - e < Decimal(margin) / 8

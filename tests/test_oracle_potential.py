"""Pins of the pair potential, the switch and the rate bound (Sec. IV.A Eq. VdW,
Sec. V Coulomb split, Sec. IV.A bound L >= |chi W'|_inf)."""
import math

import numpy as np
import pytest
from scipy import optimize, special

KE = 332.0637


def _params(orc, coulomb, **kw):
    base = dict(charge=[-0.834, 0.417], eps=[0.152, 0.0], sigma=[3.15, 0.0], periodic=False,
                r_on=5.0, r_off=6.0, r_cut=9.0, coulomb=coulomb)
    base.update(kw)
    return orc.make_params(None, **base)


@pytest.mark.parametrize("coulomb", [0, 1])
def test_closed_forms(orc, coulomb):
    p = _params(orc, coulomb)
    a = 0.35
    for r in [1.0, 2.5, 3.15, 4.2, 8.0]:
        # H-H: Coulomb only
        u, du = orc.pair_u(p, 1, 1, r)
        g = 1.0 / r if coulomb == 0 else special.erfc(a * r) / r
        assert u == pytest.approx(KE * 0.417 * 0.417 * g, rel=1e-13)
        # O-O: Coulomb + LJ 4 eps [(s/r)^12 - (s/r)^6]
        u, du = orc.pair_u(p, 0, 0, r)
        g = 1.0 / r if coulomb == 0 else special.erfc(a * r) / r
        lj = 4 * 0.152 * ((3.15 / r) ** 12 - (3.15 / r) ** 6)
        assert u == pytest.approx(KE * 0.834**2 * g + lj, rel=1e-12)


def test_lj_minimum(orc):
    p = _params(orc, 0, charge=[0.0, 0.0])
    rmin = 2 ** (1 / 6) * 3.15
    u, du = orc.pair_u(p, 0, 0, rmin)
    assert u == pytest.approx(-0.152, rel=1e-12)
    assert abs(du) < 1e-12


@pytest.mark.parametrize("coulomb", [0, 1])
@pytest.mark.parametrize("ab", [(0, 0), (0, 1), (1, 1)])
def test_derivatives_against_finite_differences(orc, coulomb, ab):
    p = _params(orc, coulomb)
    h = 1e-5
    for r in [1.5, 2.8, 4.0, 6.5, 8.7]:
        u, du = orc.pair_u(p, *ab, r)
        fd = (orc.pair_u(p, *ab, r + h)[0] - orc.pair_u(p, *ab, r - h)[0]) / (2 * h)
        assert du == pytest.approx(fd, rel=1e-7, abs=1e-9)
        w, dw = orc.pair_wsf(p, *ab, r)
        fdw = (orc.pair_wsf(p, *ab, r + h)[0] - orc.pair_wsf(p, *ab, r - h)[0]) / (2 * h)
        assert dw == pytest.approx(fdw, rel=1e-7, abs=1e-9)


@pytest.mark.parametrize("coulomb", [0, 1])
def test_shifted_force_vanishes_at_cutoff(orc, coulomb):
    p = _params(orc, coulomb)
    for ab in [(0, 0), (0, 1), (1, 1)]:
        w, dw = orc.pair_wsf(p, *ab, 9.0 - 1e-9)
        assert abs(w) < 1e-9 and abs(dw) < 1e-9
        assert orc.pair_wsf(p, *ab, 9.0) == (0.0, 0.0)
        assert orc.pair_wsf(p, *ab, 12.0) == (0.0, 0.0)
        # W_sf - u differs from u by a linear function of r: second differences agree
        r, h = 4.0, 1e-3
        d2w = orc.pair_wsf(p, *ab, r + h)[0] - 2 * orc.pair_wsf(p, *ab, r)[0] + orc.pair_wsf(p, *ab, r - h)[0]
        d2u = orc.pair_u(p, *ab, r + h)[0] - 2 * orc.pair_u(p, *ab, r)[0] + orc.pair_u(p, *ab, r - h)[0]
        assert d2w == pytest.approx(d2u, rel=1e-6, abs=1e-12)


def test_switch_is_c2_and_monotone(orc):
    p = _params(orc, 0, r_on=5.0, r_off=6.0)
    assert orc.chi(p, 4.0) == 0.0 and orc.chi(p, 5.0) == 0.0
    assert orc.chi(p, 6.0) == 1.0 and orc.chi(p, 7.5) == 1.0
    assert orc.chi(p, 5.5) == pytest.approx(0.5, abs=1e-15)
    rs = np.linspace(5.0, 6.0, 1001)
    vals = np.array([orc.chi(p, r) for r in rs])
    assert np.all(np.diff(vals) >= 0)
    h = 1e-4
    for r0 in (5.0, 6.0):
        d1 = (orc.chi(p, r0 + h) - orc.chi(p, r0 - h)) / (2 * h)
        d2 = (orc.chi(p, r0 + h) - 2 * orc.chi(p, r0) + orc.chi(p, r0 - h)) / h**2
        assert abs(d1) < 1e-6 and abs(d2) < 1e-2  # O(h) second-derivative jump-free


@pytest.mark.parametrize("coulomb,r_on,r_off", [(0, 5.0, 6.0), (1, 6.0, 7.0), (1, 4.0, 5.0)])
def test_rate_bound_is_a_tight_upper_bound(orc, coulomb, r_on, r_off):
    p = _params(orc, coulomb, r_on=r_on, r_off=r_off)
    L_ab, L_a = orc.rate_bounds(p)
    for a in range(2):
        assert L_a[a] == pytest.approx(L_ab[a].max(), rel=0)
        for b in range(2):
            f = lambda r: abs(orc.chi(p, r) * orc.pair_wsf(p, a, b, r)[1])
            rs = np.linspace(r_on, 9.0, 20001)[:-1]
            vals = np.array([f(r) for r in rs])
            k = int(vals.argmax())
            lo, hi = rs[max(k - 1, 0)], rs[min(k + 1, len(rs) - 1)]
            res = optimize.minimize_scalar(lambda r: -f(r), bounds=(lo, hi), method="bounded",
                                           options=dict(xatol=1e-10))
            sup = max(vals.max(), -res.fun)
            assert L_ab[a, b] >= sup                       # a bound
            assert L_ab[a, b] <= sup * (1 + 1e-3) * (1 + 1e-7)  # and a tight one
            assert L_ab[a, b] == pytest.approx(L_ab[b, a], rel=1e-15)

"""Pins of the oracle's differentiable direct-space energy (Sec. V E_direct and
E_VdW with the full cutoff): central finite differences in positions and in the
per-type parameters, Euler homogeneity in the charges and in epsilon, and the
position gradient equal to the full pair gradient."""
import numpy as np
import pytest

from workloads import jitter_positions, water_box


@pytest.fixture(scope="module")
def setup(orc):
    sys = water_box(n_side=5, box_len=15.5, seed=5)
    p = orc.make_params(sys, r_cut=7.0)
    topo = orc.Topology.from_system(sys)
    q = jitter_positions(sys.pos, 0.05, seed=1)
    return sys, p, topo, q


def _with(orc, sys, base, **kw):
    ff = dict(charge=list(base.charge[:2]), eps=list(base.eps[:2]), sigma=list(base.sigma[:2]))
    ff.update(kw)
    return orc.make_params(sys, r_cut=base.r_cut, **ff)


def test_parameter_gradients_finite_differences(orc, setup):
    sys, p, topo, q = setup
    E, gq, gc, ge, gs = orc.direct_energy(p, topo, q)
    h = 1e-4
    for name, g, idx in [("charge", gc, 0), ("charge", gc, 1), ("eps", ge, 0), ("sigma", gs, 0)]:
        vals = list(getattr(p, name)[:2])
        vp, vm = list(vals), list(vals)
        vp[idx] += h
        vm[idx] -= h
        Ep = orc.direct_energy(_with(orc, sys, p, **{name: vp}), topo, q, grads=False)
        Em = orc.direct_energy(_with(orc, sys, p, **{name: vm}), topo, q, grads=False)
        assert g[idx] == pytest.approx((Ep - Em) / (2 * h), rel=1e-7)


def test_position_gradient(orc, setup):
    sys, p, topo, q = setup
    E, gq, *_ = orc.direct_energy(p, topo, q)
    np.testing.assert_allclose(gq, orc.gradient(p, topo, q, orc.G_FULL), rtol=1e-12, atol=1e-12)
    h = 1e-4
    rng = np.random.default_rng(0)
    for i in rng.choice(sys.n_atoms, 8, replace=False):
        for c in range(3):
            qp, qm = q.copy(), q.copy()
            qp[i, c] += h
            qm[i, c] -= h
            fd = (orc.direct_energy(p, topo, qp, grads=False)
                  - orc.direct_energy(p, topo, qm, grads=False)) / (2 * h)
            assert gq[i, c] == pytest.approx(fd, rel=1e-6, abs=1e-7)


def test_euler_homogeneity(orc, setup):
    sys, p, topo, q = setup
    E, gq, gc, ge, gs = orc.direct_energy(p, topo, q)
    e = orc.energies(p, topo, q, np.zeros_like(q))
    assert E == pytest.approx(e["pair"], rel=1e-12)
    # E_C is homogeneous of degree 2 in the charges, E_LJ of degree 1 in eps_O (eps_H = 0)
    assert gc[0] * p.charge[0] + gc[1] * p.charge[1] == pytest.approx(2 * e["coul"], rel=1e-10)
    assert ge[0] * p.eps[0] == pytest.approx(e["lj"], rel=1e-10)

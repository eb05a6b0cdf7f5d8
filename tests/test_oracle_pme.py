"""Pins of the oracle's reciprocal-space Ewald (Sec. V: SPME).

The plain reciprocal Ewald sum is pinned by the Madelung constant of rock
salt (with an independent real-space sum and the self term); smooth PME
converges to that sum as the mesh refines; its analytic gradient matches
finite differences of its energy; and for a lone excluded ion pair in a
growing box the reciprocal, self and exclusion terms cancel to the pair's
image interaction, which vanishes like 1/L^3."""
import math

import numpy as np
import pytest
from scipy import special

KE = 332.0637
MADELUNG_NACL = 1.747564594633


def _ions(orc, q, charges, L, alpha, K=None, order=5, excl=None):
    types = np.array([0 if c > 0 else 1 for c in charges], np.int32)
    p = orc.make_params(None, charge=[1.0, -1.0], eps=[0.0, 0.0], sigma=[0.0, 0.0],
                        periodic=True, box=[L] * 3, coulomb=1, ewald_alpha=alpha,
                        pme_grid=[K] * 3 if K else None, pme_order=order)
    topo = orc.Topology(types, np.ones(len(types)), excl=excl)
    return p, topo


def _real_space(q, charges, L, alpha, nimg=3):
    """sum over pairs and periodic images of k_e q_i q_j erfc(alpha r) / r (i<j
    in the cell, all i,j for image shifts != 0, halved)"""
    E = 0.0
    shifts = [np.array(s) * L for s in np.ndindex(2 * nimg + 1, 2 * nimg + 1, 2 * nimg + 1)]
    shifts = [s - nimg * L for s in shifts]
    for s in shifts:
        d = q[:, None, :] - q[None, :, :] + s
        r = np.linalg.norm(d, axis=-1)
        zero = np.all(s == 0)
        mask = ~np.eye(len(q), dtype=bool) if zero else np.ones((len(q), len(q)), bool)
        E += 0.5 * np.sum((KE * np.outer(charges, charges) * special.erfc(alpha * r) / np.where(mask, r, 1.0))[mask])
    return E


def test_madelung_constant_of_rock_salt(orc):
    a = 5.64                       # conventional cell; nearest neighbours at a/2
    n = 4                          # ions per edge (2 x 2 x 2 conventional cells)
    L = n * a / 2
    idx = np.array(list(np.ndindex(n, n, n)))
    q = idx * (a / 2)
    charges = np.where(idx.sum(1) % 2 == 0, 1.0, -1.0)
    alpha = 0.6
    p, topo = _ions(orc, q, charges, L, alpha)
    e_rec, _ = orc.ewald_recip(p, topo, q, 10, grad=False)
    e_self = -KE * alpha / math.sqrt(math.pi) * len(q)
    e_real = _real_space(q, charges, L, alpha)
    E = e_real + e_rec + e_self
    expect = -MADELUNG_NACL * KE * (len(q) / 2) / (a / 2)
    assert E == pytest.approx(expect, rel=1e-8)
    # the mesh sum reproduces it too, and its own self term agrees
    p.pme_grid[0] = p.pme_grid[1] = p.pme_grid[2] = 32
    (er, es, ex), _ = orc.pme(p, topo, q, grad=False)
    assert es == pytest.approx(e_self, rel=1e-14) and ex == 0.0
    assert e_real + er + es == pytest.approx(expect, rel=1e-6)


def test_mesh_converges_to_plain_sum(orc):
    rng = np.random.default_rng(0)
    L, n = 20.0, 60
    q = rng.uniform(0.0, L, (n, 3))
    charges = np.array([1.0, -1.0] * (n // 2))
    errs = []
    p0, topo = _ions(orc, q, charges, L, 0.35)
    E, g = orc.ewald_recip(p0, topo, q, 12)
    for K, tol_e, tol_g in ((16, 1e-3, 3e-3), (32, 1e-5, 1e-4), (48, 1e-6, 2e-5)):
        p, topo = _ions(orc, q, charges, L, 0.35, K=K)
        (er, _, _), gr = orc.pme(p, topo, q)
        errs.append(abs(er - E) / abs(E))
        assert errs[-1] < tol_e, (K, errs[-1])
        assert np.abs(gr - g).max() / np.abs(g).max() < tol_g, K
    assert errs[0] > errs[1] > errs[2]


@pytest.mark.parametrize("order", [4, 5, 6])
def test_gradient_matches_finite_differences(orc, order):
    from workloads import water_box
    s = water_box(n_side=4, box_len=12.4, seed=5)
    p = orc.make_params(s, ewald_alpha=0.45, pme_grid=[24, 24, 24], pme_order=order)
    topo = orc.Topology.from_system(s)
    (_, _, ex), g = orc.pme(p, topo, s.pos)
    assert ex > 0.0        # removes the attraction of the excluded O-H pairs (net of H-H)
    rng = np.random.default_rng(3)
    h = 1e-5
    for i in rng.choice(s.n_atoms, 6, replace=False):
        for c in range(3):
            qp, qm = s.pos.copy(), s.pos.copy()
            qp[i, c] += h
            qm[i, c] -= h
            ep = orc.pme(p, topo, qp, grad=False)[0]
            em = orc.pme(p, topo, qm, grad=False)[0]
            fd = ((ep[0] + ep[2]) - (em[0] + em[2])) / (2 * h)
            assert g[i, c] == pytest.approx(fd, rel=1e-6, abs=1e-6)


def test_lone_excluded_pair_cancels(orc):
    """A neutral excluded pair at distance 1 A: E_rec + E_self + E_excl is the
    interaction with its periodic images, decaying like 1/L^3."""
    vals = []
    for L in (15.0, 30.0):
        q = np.array([[L / 2, L / 2, L / 2], [L / 2 + 1.0, L / 2, L / 2]])
        p, topo = _ions(orc, q, np.array([1.0, -1.0]), L, 5.0 / L * 2.0, K=int(L) * 2,
                        excl=np.array([[0, 1]]))
        (er, es, ex), _ = orc.pme(p, topo, q, grad=False)
        vals.append(er + es + ex)
    # the image term of a dipole lattice ~ (dipole)^2 / L^3: shrinks ~8x
    assert abs(vals[1]) < abs(vals[0]) / 5
    assert abs(vals[1]) < 0.05


def test_respa_outer_step_conserves_energy(orc):
    """BAOAB without friction and with the mesh force as RESPA outer kicks
    (m = 2) or in every step (m = 0): the total energy, mesh terms included,
    stays put; a wrong sign or size of the outer kick would not."""
    from helpers import relaxed_box
    s = relaxed_box("b8")
    topo = orc.Topology.from_system(s)
    drifts = {}
    for m in (0, 2):
        p = orc.make_params(s, integrator=orc.BAOAB, dt=0.5, gamma=0.0, ewald_alpha=0.45,
                            r_cut=9.0, skin=2.0, pme_grid=[24, 24, 24], pme_order=5, respa_m=m)
        e0 = orc.energies(p, topo, s.pos, s.vel)
        o = orc.run(p, topo, s.pos, s.vel, 0, 60)
        assert o["status"] == 0, o["status_name"]
        e1 = orc.energies(p, topo, o["q"], o["v"])
        tot = lambda e: e["bond"] + e["angle"] + e["pair"] + e["kin"]
        drifts[m] = abs(tot(e1) - tot(e0))
        assert drifts[m] < 2e-3 * e0["kin"], (m, drifts[m], e0["kin"])
    # the reciprocal part is not negligible here: dropping it moves the energy more
    p = orc.make_params(s, integrator=orc.BAOAB, dt=0.5, gamma=0.0, ewald_alpha=0.45,
                        pme_grid=[24, 24, 24], pme_order=5, respa_m=2)
    (er, _, _), g = orc.pme(p, topo, s.pos)
    assert np.abs(g).max() > 1.0


def test_outer_nonbonded_with_one_inner_step_is_the_basic_scheme(orc):
    """BOUNCE-RESPA with the short pair force on the outer step (Sec. V) and
    m = 1: the outer half kicks and the inner B kicks add up to the basic
    scheme's kicks, so the trajectory and the jump events are the same up to
    rounding; with m = 2 they are not."""
    from helpers import relaxed_box
    s = relaxed_box("b8")
    topo = orc.Topology.from_system(s)
    kw = dict(integrator=orc.BOUNCE, dt=1.0, ewald_alpha=0.45, r_on=6.0, r_off=7.0, r_cut=9.0,
              skin=2.0, pme_grid=[16, 16, 16], pme_order=5)
    base = orc.run(orc.make_params(s, respa_m=0, **kw), topo, s.pos, s.vel, 0, 20, ev_cap=200000)
    one = orc.run(orc.make_params(s, respa_m=1, respa_outer=orc.OUTER_NONBONDED, **kw), topo, s.pos,
                  s.vel, 0, 20, ev_cap=200000)
    two = orc.run(orc.make_params(s, respa_m=2, respa_outer=orc.OUTER_NONBONDED, **kw), topo, s.pos,
                  s.vel, 0, 20, ev_cap=200000)
    for o in (base, one, two):
        assert o["status"] == 0, o["status_name"]
    assert base["n_events"] > 0
    assert np.abs(one["q"] - base["q"]).max() < 1e-9
    assert np.abs(one["v"] - base["v"]).max() < 1e-9
    key = lambda e: sorted(zip(e["step"], e["phase"], e["atom"], e["k"], e["partner"], e["accepted"]))
    assert key(one["events"]) == key(base["events"])
    assert np.abs(two["q"] - base["q"]).max() > 1e-6


@pytest.mark.parametrize("with_mesh", [False, True])
def test_outer_nonbonded_conserves_energy(orc, with_mesh):
    """BAOAB without friction, bonded forces on the inner step (0.5 fs) and the
    short-range pair force (plus the mesh force) on an outer step of m = 4:
    the total energy stays put, and moving the pair force to the outer step
    with the wrong sign or size of kick would not."""
    from helpers import relaxed_box
    s = relaxed_box("b8")
    topo = orc.Topology.from_system(s)
    mesh = dict(pme_grid=[24, 24, 24], pme_order=5) if with_mesh else {}
    p = orc.make_params(s, integrator=orc.BAOAB, dt=0.5, gamma=0.0, ewald_alpha=0.45, r_cut=9.0,
                        skin=2.0, respa_m=4, respa_outer=orc.OUTER_NONBONDED, rebuild_interval=8,
                        **mesh)
    e0 = orc.energies(p, topo, s.pos, s.vel)
    o = orc.run(p, topo, s.pos, s.vel, 0, 80)
    assert o["status"] == 0, o["status_name"]
    e1 = orc.energies(p, topo, o["q"], o["v"])
    tot = lambda e: e["bond"] + e["angle"] + e["pair"] + e["kin"]
    assert abs(tot(e1) - tot(e0)) < 2e-3 * e0["kin"], (tot(e1) - tot(e0), e0["kin"])


def test_mesh_outer_step_of_one_is_the_mesh_in_f0(orc):
    """The mesh force on an outer step of m = 1 (half kicks of dt/2 around every
    step) equals the mesh force in F_0 (the basic scheme) up to rounding, with
    the same jump events."""
    from helpers import relaxed_box
    s = relaxed_box("b8")
    topo = orc.Topology.from_system(s)
    kw = dict(integrator=orc.BOUNCE, dt=1.0, ewald_alpha=0.45, r_on=6.0, r_off=7.0, r_cut=9.0,
              skin=2.0, pme_grid=[16, 16, 16], pme_order=4)
    f0 = orc.run(orc.make_params(s, respa_m=0, **kw), topo, s.pos, s.vel, 0, 20, ev_cap=200000)
    one = orc.run(orc.make_params(s, respa_m=1, **kw), topo, s.pos, s.vel, 0, 20, ev_cap=200000)
    for o in (f0, one):
        assert o["status"] == 0, o["status_name"]
    assert f0["n_events"] > 0
    assert np.abs(one["q"] - f0["q"]).max() < 1e-9
    assert np.abs(one["v"] - f0["v"]).max() < 1e-9
    key = lambda e: sorted(zip(e["step"], e["phase"], e["atom"], e["k"], e["partner"], e["accepted"]))
    assert key(one["events"]) == key(f0["events"])

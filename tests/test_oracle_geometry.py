"""Pins of the oracle's canonical order, pair lists, gradients and energies.

Lists are checked against sets computed here with numpy (an independent
minimum-image distance computation); gradients against central finite
differences of the oracle's own energy, and against the force splitting of
Sec. IV.A (short + long = full)."""
import numpy as np
import pytest

from workloads import water_box, water_droplet


@pytest.fixture(scope="module")
def small_box():
    return water_box(n_side=6, box_len=18.6, seed=1)


@pytest.fixture(scope="module")
def droplet():
    return water_droplet(n_waters=64, seed=2)


def _numpy_pairs(sys, rmin, rmax):
    q = sys.pos
    d = q[:, None, :] - q[None, :, :]
    if sys.periodic:
        d -= sys.box * np.rint(d / sys.box)
    r2 = np.einsum("ijk,ijk->ij", d, d)
    ok = r2 < rmax * rmax
    if rmin > 0:
        ok &= r2 >= rmin * rmin
    np.fill_diagonal(ok, False)
    for a, b in sys.excl:
        ok[a, b] = ok[b, a] = False
    return ok


@pytest.mark.parametrize("which", ["box", "drop"])
@pytest.mark.parametrize("rmin,rmax", [(0.0, 9.0), (3.0, 11.0), (0.0, 8.0)])
def test_lists_equal_brute_force_sets(orc, small_box, droplet, which, rmin, rmax):
    sys = small_box if which == "box" else droplet
    p = orc.make_params(sys)
    topo = orc.Topology.from_system(sys)
    order, cell = orc.sort_order(p, sys.pos)
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    rp, col = orc.build_list(p, topo, sys.pos, rmin, rmax, order)
    ok = _numpy_pairs(sys, rmin, rmax)
    for i in range(sys.n_atoms):
        row = col[rp[i]:rp[i + 1]]
        assert set(row.tolist()) == set(np.nonzero(ok[i])[0].tolist())
        assert np.all(np.diff(rank[row]) > 0)  # canonical order: ascending sorted position
        # a single row computed alone is the same row
        if i % 37 == 0:
            assert np.array_equal(orc.list_row(p, topo, sys.pos, rmin, rmax, order, i), row)


def test_canonical_order_is_cell_then_id(orc, small_box, droplet):
    for sys in (small_box, droplet):
        p = orc.make_params(sys)
        order, cell = orc.sort_order(p, sys.pos)
        key = np.stack([cell[order], order], 1)
        assert np.all((np.diff(key[:, 0]) > 0) | ((np.diff(key[:, 0]) == 0) & (np.diff(key[:, 1]) > 0)))
        assert sorted(order.tolist()) == list(range(sys.n_atoms))
    # periodic cells: cell width = box / floor(box / cell_size); wrapped coordinates
    p = orc.make_params(small_box)
    order, cell = orc.sort_order(p, small_box.pos)
    n = int(np.floor(18.6 / small_box.cell_size))
    x = small_box.pos - 18.6 * np.floor(small_box.pos / 18.6)
    c = np.clip(np.floor(x / (18.6 / n)).astype(int), 0, n - 1)
    lin = (c[:, 0] * n + c[:, 1]) * n + c[:, 2]
    assert np.mean(lin == cell) > 0.999  # equal up to floor() ties at cell faces


def test_droplet_outside_grid_is_an_error(orc, droplet):
    p = orc.make_params(droplet)
    q = droplet.pos.copy()
    q[5] += 1000.0
    with pytest.raises(RuntimeError, match="GRID"):
        orc.sort_order(p, q)


def _etot(orc, p, topo, q, v):
    e = orc.energies(p, topo, q, v)
    return e["bond"] + e["angle"] + e["pair"]


@pytest.mark.parametrize("which", ["box", "drop"])
def test_gradient_matches_finite_differences(orc, small_box, droplet, which):
    sys = small_box if which == "box" else droplet
    p = orc.make_params(sys)
    topo = orc.Topology.from_system(sys)
    q = sys.pos
    g = orc.gradient(p, topo, q, orc.G_BONDED | orc.G_FULL)
    h = 1e-5
    rng = np.random.default_rng(3)
    for i in rng.choice(sys.n_atoms, 6, replace=False):
        for c in range(3):
            qp, qm = q.copy(), q.copy()
            qp[i, c] += h
            qm[i, c] -= h
            fd = (_etot(orc, p, topo, qp, sys.vel) - _etot(orc, p, topo, qm, sys.vel)) / (2 * h)
            assert g[i, c] == pytest.approx(fd, rel=2e-6, abs=2e-6)


def test_force_split_and_newton(orc, small_box):
    p = orc.make_params(small_box, r_on=4.0, r_off=5.5)
    topo = orc.Topology.from_system(small_box)
    q = small_box.pos
    gs = orc.gradient(p, topo, q, orc.G_SHORT)
    gl = orc.gradient(p, topo, q, orc.G_LONG)
    gf = orc.gradient(p, topo, q, orc.G_FULL)
    np.testing.assert_allclose(gs + gl, gf, rtol=1e-10, atol=1e-10)
    assert np.abs(gf.sum(0)).max() < 1e-9       # pair gradients sum to zero
    gb = orc.gradient(p, topo, q, orc.G_BONDED)
    assert np.abs(gb.sum(0)).max() < 1e-9
    # the single-atom variant agrees with the all-atom one
    for i in (0, 7, 300):
        np.testing.assert_allclose(orc.gradient_atom(p, topo, q, orc.G_SHORT | orc.G_BONDED, i),
                                   gs[i] + gb[i], rtol=1e-12, atol=1e-12)


def test_energy_terms_closed_forms(orc):
    # one water at its reference geometry has no bonded energy; a stretched one has k dx^2
    sys = water_droplet(n_waters=1, seed=0)
    p = orc.make_params(sys)
    topo = orc.Topology.from_system(sys)
    e = orc.energies(p, topo, sys.pos, np.zeros_like(sys.pos))
    assert abs(e["bond"]) < 1e-20 and abs(e["angle"]) < 1e-20 and e["pair"] == 0.0
    q = sys.pos.copy()
    d = q[1] - q[0]
    q[1] = q[0] + d * (1 + 0.1 / np.linalg.norm(d))
    e = orc.energies(p, topo, q, np.zeros_like(q))
    assert e["bond"] == pytest.approx(450.0 * 0.1**2, rel=1e-12)
    v = np.ones_like(q)
    e = orc.energies(p, topo, q, v)
    assert e["kin"] == pytest.approx(0.5 * sys.mass.sum() * 3 / 4.184e-4, rel=1e-14)


@pytest.mark.parametrize("dtheta", [0.05, -0.12, 0.3])
def test_angle_energy_and_gradient_closed_forms(orc, dtheta):
    """A water whose H2 is rotated about O in the molecular plane by dtheta
    keeps both bonds at r0 and has H-O-H = theta0 + dtheta: E_angle = k dtheta^2
    exactly (the harmonic angle term of flexible water, with k = 55 kcal/mol/rad^2
    and no factor 1/2), E_bond = 0, and the angle gradient on H2 is tangential
    with magnitude 2 k dtheta / r0 (dtheta/ds = 1/r0 along the arc)."""
    sys = water_droplet(n_waters=1, seed=0)
    p = orc.make_params(sys)
    topo = orc.Topology.from_system(sys)
    q = sys.pos.copy()
    o, h1, h2 = q[0], q[1], q[2]
    n = np.cross(h1 - o, h2 - o)
    n /= np.linalg.norm(n)
    # rotate H2 about the normal so that the angle opens by dtheta
    d = h2 - o
    c, s = np.cos(dtheta), np.sin(dtheta)
    rot = d * c + np.cross(n, d) * s + n * np.dot(n, d) * (1 - c)
    ang0 = np.arccos(np.dot(h1 - o, d) / (np.linalg.norm(h1 - o) * np.linalg.norm(d)))
    ang1 = np.arccos(np.dot(h1 - o, rot) / (np.linalg.norm(h1 - o) * np.linalg.norm(rot)))
    if abs(ang1 - ang0 - dtheta) > 1e-9:        # rotated the other way: flip the sense
        rot = d * c - np.cross(n, d) * s + n * np.dot(n, d) * (1 - c)
    q[2] = o + rot
    e = orc.energies(p, topo, q, np.zeros_like(q))
    assert e["bond"] == pytest.approx(0.0, abs=1e-20)
    assert e["angle"] == pytest.approx(55.0 * dtheta ** 2, rel=1e-10)
    g = orc.gradient(p, topo, q, orc.G_BONDED)
    r0 = np.linalg.norm(rot)
    assert np.linalg.norm(g[2]) == pytest.approx(2.0 * 55.0 * abs(dtheta) / r0, rel=1e-10)
    # tangential: orthogonal to the O-H2 bond, in the molecular plane
    assert abs(np.dot(g[2], rot)) < 1e-10 * np.linalg.norm(g[2]) * r0
    assert abs(np.dot(g[2], n)) < 1e-10 * np.linalg.norm(g[2])
    # opening the angle raises the energy: the gradient points along the opening direction
    opening = np.cross(n, rot) if np.dot(np.cross(n, rot), h1 - o) < 0 else -np.cross(n, rot)
    assert np.sign(np.dot(g[2], opening)) == np.sign(dtheta)

"""Pins of the per-type-pair rate bounds (Sec. V: the bound may depend on the
types of both atoms; Sec. II.B: independent Poisson clocks superpose, and each
proposal belongs to a mechanism with probability proportional to its bound).

Under RATE_PAIR a partner j of type b of an atom of type a carries the bound
L'_ab = Lq_ab * unit_a, with the integer weight Lq_ab = ceil(2^20 L_ab / L_a - 1e-4)
and unit_a = bound_scale L_a 2^-20; the proposal count has mean
beta |v| dt/2 sum_j L'_ab and partner j is picked with probability L'_ab / sum.  The thinned (accepted) process must be the same
as under RATE_ATOM, where every partner carries L_a = max_b L_ab."""
import math

import numpy as np
import pytest
from scipy import stats

KB, KE = 0.0019872041, 332.0637


def _droplet(orc, rate_mode, n_waters=64, seed=4, one_type=False):
    from workloads import water_droplet
    sys = water_droplet(n_waters=n_waters, seed=seed)
    if one_type:
        sys.atom_type = np.zeros_like(sys.atom_type)
        kw = dict(charge=[0.417], eps=[0.0], sigma=[0.0])
    else:
        kw = dict(charge=[-0.834, 0.417], eps=[0.0, 0.0], sigma=[0.0, 0.0])
    p = orc.make_params(sys, coulomb=orc.COUL_BARE, r_on=4.0, r_off=5.0, rate_mode=rate_mode, **kw)
    topo = orc.Topology.from_system(sys)
    order, _ = orc.sort_order(p, sys.pos)
    rp, col = orc.build_list(p, topo, sys.pos, p.r_on - p.skin, p.r_cut + p.skin, order)
    return sys, p, topo, rp, col


def _bounds(orc, p):
    """L'_ab = Lq_ab unit_a as the oracle uses them."""
    Lq, unit = orc.rate_weights(p)
    return Lq.astype(np.float64) * unit[:, None]


def test_weights_are_tight_integer_bounds(orc):
    for mode in (orc.RATE_ATOM, orc.RATE_PAIR):
        for scale in (1.0, 3.0):
            _, p, _, _, _ = _droplet(orc, mode)
            p.bound_scale = scale
            L_ab, L_a = orc.rate_bounds(p)
            Lq, unit = orc.rate_weights(p)
            one = 2 ** orc.WEIGHT_BITS
            np.testing.assert_array_equal(unit, scale * L_a / one)
            assert np.all(Lq.max(axis=1) == one)
            Lb = Lq * unit[:, None]
            if mode == orc.RATE_ATOM:
                assert np.all(Lq == one)
                np.testing.assert_array_equal(Lb, np.repeat((L_a * scale)[:, None], p.n_types, 1))
            else:
                # a bound on every pair type (up to the 1e-4-unit slack), at most one unit above it
                assert np.all(Lb >= scale * L_ab - 1e-4 * unit[:, None] * (1 + 1e-9))
                assert np.all(Lb - scale * L_ab <= unit[:, None] * (1 + 1e-12))
                # bare Coulomb with zero LJ: L_ab scales with |q_a q_b|
                np.testing.assert_allclose(L_ab / L_ab[0, 0],
                                           np.array([[1.0, 0.5], [0.5, 0.25]]), rtol=1e-3)


def test_single_type_pair_mode_equals_atom_mode(orc):
    """One type: every weight is 2^20 and the class is the whole row, so the
    two modes must draw the same partners and accept the same events."""
    outs = []
    for mode in (orc.RATE_ATOM, orc.RATE_PAIR):
        sys, p, topo, rp, col = _droplet(orc, mode, one_type=True)
        outs.append(orc.jump_halfstep(p, topo, sys.pos, sys.vel * 3.0, rp, col, step=2,
                                      phase=orc.PH_JB, ev_cap=10**6))
    a, b = outs
    assert a["counters"]["proposals"] > 1000
    assert np.array_equal(a["v"], b["v"])
    assert a["counters"] == b["counters"]
    assert np.array_equal(a["events"], b["events"])


def _pair_field(p, q, i, j, ti, tj):
    """chi W'_sf d/r for bare Coulomb with zero LJ, independently in numpy."""
    rc, ron, roff = p.r_cut, p.r_on, p.r_off
    d = q[i] - q[j]
    r = np.linalg.norm(d)
    if not (ron < r < rc):
        return np.zeros(3)
    qq = KE * p.charge[ti] * p.charge[tj]
    x = (r - ron) / (roff - ron)
    ch = 1.0 if x >= 1 else x ** 3 * (10 - 15 * x + 6 * x * x)
    return ch * (-qq / r ** 2 + qq / rc ** 2) * d / r


def test_pair_mode_compensator(orc):
    """Sum over logged proposals of lambda / L'_{a,type(j)} (each proposal with
    its own pair bound) matches the number of accepted events."""
    sys, p, topo, rp, col = _droplet(orc, orc.RATE_PAIR)
    Lb = _bounds(orc, p)
    tot, var, acc = 0.0, 0.0, 0
    v_in = sys.vel * 3.0
    for step in range(6):
        out = orc.jump_halfstep(p, topo, sys.pos, v_in, rp, col, step=step, phase=orc.PH_JA,
                                ev_cap=10**6)
        vv = v_in.copy()
        for e in out["events"]:
            i, j = int(e["atom"]), int(e["partner"])
            ti, tj = topo.type[i], topo.type[j]
            F = _pair_field(p, sys.pos, i, j, ti, tj)
            pr = max(0.0, vv[i] @ F) / (np.linalg.norm(vv[i]) * Lb[ti, tj])
            assert pr <= 1.0 + 1e-9
            if e["accepted"]:
                assert pr > 0
                vv[i] = vv[i] - 2 * (vv[i] @ F) / (F @ F) * F
                acc += 1
            tot += pr
            var += pr * (1 - pr)
        np.testing.assert_allclose(vv, out["v"], rtol=1e-12, atol=1e-15)
    assert acc > 200
    assert abs(acc - tot) < 5 * math.sqrt(var)


def test_pair_mode_proposal_counts_and_partner_classes(orc):
    """Proposals per atom have mean beta |v| dt/2 sum_j L'_{a,type(j)}, and the
    partner's class is b with probability n_b L'_ab / sum_b' n_b' L'_ab'."""
    sys, p, topo, rp, col = _droplet(orc, orc.RATE_PAIR, n_waters=100, seed=7)
    Lb = _bounds(orc, p)
    beta = 1.0 / (KB * p.temperature)
    v = sys.vel * 3.0
    n = topo.n
    ncls = np.zeros((n, 2))
    for i in range(n):
        ncls[i] = np.bincount(topo.type[col[rp[i]:rp[i + 1]]], minlength=2)
    rate = (ncls * Lb[topo.type]).sum(axis=1)               # sum_j L'_ij
    mu = beta * np.linalg.norm(v, axis=1) * rate * 0.5 * p.dt
    steps = 30
    per_cls = np.zeros((n, 2))
    total = 0
    for step in range(steps):
        out = orc.jump_halfstep(p, topo, sys.pos, v, rp, col, step=step, phase=orc.PH_JB,
                                ev_cap=10**6)
        ev = out["events"]
        total += len(ev)
        np.add.at(per_cls, (ev["atom"], topo.type[ev["partner"]]), 1)
    expect = steps * mu.sum()
    assert abs(total - expect) < 5 * math.sqrt(expect)
    # class frequencies, per atom type a
    for a in (0, 1):
        sel = topo.type == a
        # proposals of atom i land in class b with probability ncls_ib L'_ab / rate_i
        e_b = (steps * mu[sel, None] * ncls[sel] * Lb[a][None, :] / rate[sel, None]).sum(axis=0)
        o_b = per_cls[sel].sum(axis=0)
        chi2 = ((o_b - e_b) ** 2 / e_b).sum()
        assert stats.chi2.sf(chi2, 1) > 1e-4, (a, o_b, e_b)


def test_pair_mode_fewer_proposals_same_accepted_law(orc):
    """Both modes thin the same process: their accepted counts agree within
    sampling error while RATE_PAIR proposes in proportion to sum_j L'_ab."""
    res = {}
    for mode in (orc.RATE_ATOM, orc.RATE_PAIR):
        sys, p, topo, rp, col = _droplet(orc, mode, n_waters=100, seed=9)
        acc = prop = 0
        for step in range(40):
            out = orc.jump_halfstep(p, topo, sys.pos, sys.vel * 3.0, rp, col, step=step,
                                    phase=orc.PH_JA)
            acc += out["counters"]["accepted"]
            prop += out["counters"]["proposals"]
        res[mode] = (acc, prop, p, topo, rp, col)
    (a0, p0, pa, topo, rp, col), (a1, p1, pp, _, _, _) = res[orc.RATE_ATOM], res[orc.RATE_PAIR]
    assert a0 > 500
    assert abs(a0 - a1) < 5 * math.sqrt(a0 + a1)
    L_atom, L_pair = _bounds(orc, pa), _bounds(orc, pp)
    cls = [np.bincount(topo.type[col[rp[i]:rp[i + 1]]], minlength=2) for i in range(topo.n)]
    w0 = sum(c @ L_atom[topo.type[i]] for i, c in enumerate(cls))
    w1 = sum(c @ L_pair[topo.type[i]] for i, c in enumerate(cls))
    assert w1 < 0.75 * w0
    assert p1 / p0 == pytest.approx(w1 / w0, rel=0.05)

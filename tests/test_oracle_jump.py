"""Pins of the oracle's J step: reflection algebra (Eq. R_i), the exact law of
a single jump clock (Eq. S_i), Poisson proposal counts and thinning (Sec. III.D),
invariance of the accepted-event law under the bound, the compensator of the
accepted events, the mean-force identity behind L_J ~ L_B (Sec. III.C), and the
expected proposal count of the cost model (Sec. IV.C)."""
import math

import numpy as np
import pytest
from scipy import stats

KB, ACC, KE = 0.0019872041, 4.184e-4, 332.0637


def test_reflection_algebra(orc):
    rng = np.random.default_rng(0)
    for _ in range(200):
        v, F = rng.standard_normal(3), rng.standard_normal(3) * rng.uniform(0.01, 100)
        w = orc.reflect(v, F)
        assert np.linalg.norm(w) == pytest.approx(np.linalg.norm(v), rel=1e-14)
        assert w @ F == pytest.approx(-(v @ F), rel=1e-12, abs=1e-13 * np.linalg.norm(F))
        np.testing.assert_allclose(orc.reflect(w, F), v, rtol=1e-13, atol=1e-14)
        # component orthogonal to F is untouched
        n = F / np.linalg.norm(F)
        np.testing.assert_allclose(w - (w @ n) * n, v - (v @ n) * n, atol=1e-13)
    # mass-weighted form with a scalar mass M = m I reduces to the same map
    v, F, m = rng.standard_normal(3), rng.standard_normal(3), 15.999
    mw = v - 2 * (v @ F) / (F @ F / m) * F / m
    np.testing.assert_allclose(orc.reflect(v, F), mw, rtol=1e-13)


def _pairs(orc, n_pairs, r, v_first, charge=(-0.834,), bound_scale=1.0, coulomb=0,
           r_on=5.0, r_off=6.0):
    """n_pairs far-apart 2-atom systems of one type at separation r along x;
    atom 2k carries velocity v_first, its only candidate is atom 2k+1."""
    p = orc.make_params(None, charge=list(charge), eps=[0.0], sigma=[0.0], periodic=False,
                        coulomb=coulomb, r_on=r_on, r_off=r_off, r_cut=9.0,
                        bound_scale=bound_scale, dt=1.0)
    n = 2 * n_pairs
    q = np.zeros((n, 3))
    q[0::2, 0] = np.arange(n_pairs) * 100.0
    q[1::2, 0] = np.arange(n_pairs) * 100.0 - r      # d = q_i - q_j = +r x
    v = np.zeros((n, 3))
    v[0::2] = v_first
    topo = orc.Topology(np.zeros(n, np.int32), np.full(n, 15.999))
    row_ptr = np.arange(0, n + 1, dtype=np.int64)
    col = np.arange(n, dtype=np.int32) ^ 1
    return p, topo, q, v, row_ptr, col


def _grad_x(orc, p, r):
    return orc.chi(p, r) * orc.pair_wsf(p, 0, 0, r)[1]   # gradient on atom i along +x


def test_single_clock_exact_law(orc):
    r = 7.0
    vx = 0.05
    p, topo, q, v, rp, col = _pairs(orc, 20000, r, [vx, 0.01, -0.02])
    Fx = _grad_x(orc, p, r)
    assert Fx < 0  # bare Coulomb O-O repulsive: gradient points towards -x on i
    # choose the velocity sign so that v.F > 0 (uphill, non-zero rate)
    v[0::2, 0] = -vx
    beta = 1.0 / (KB * 300.0)
    lam = beta * max(0.0, v[0] @ np.array([Fx, 0, 0]))
    t = 0.5 * p.dt
    expect = 1.0 - math.exp(-lam * t)
    out = orc.jump_halfstep(p, topo, q, v, rp, col, step=3, phase=orc.PH_JA)
    assert out["status"] == 0
    moved = np.any(out["v"][0::2] != v[0::2], axis=1)
    n = moved.size
    se = math.sqrt(expect * (1 - expect) / n)
    assert abs(moved.mean() - expect) < 5 * se
    # a reflected velocity has the same norm and reversed v.F, so no second jump
    vr = out["v"][0::2][moved]
    np.testing.assert_allclose(np.linalg.norm(vr, axis=1), np.linalg.norm(v[0]), rtol=1e-14)
    assert np.all(vr[:, 0] * Fx < 0)
    # downhill (v.F < 0): rate zero, nothing ever accepted
    v2 = v.copy()
    v2[0::2, 0] = vx
    out2 = orc.jump_halfstep(p, topo, q, v2, rp, col, step=3, phase=orc.PH_JA)
    assert np.array_equal(out2["v"], v2)
    assert out2["counters"]["accepted"] == 0 and out2["counters"]["proposals"] > 0


def test_poisson_proposal_counts(orc):
    p, topo, q, v, rp, col = _pairs(orc, 20000, 7.0, [-0.05, 0.01, -0.02], bound_scale=40.0)
    _, L_a = orc.rate_bounds(p)
    beta = 1.0 / (KB * 300.0)
    mu = 1 * beta * np.linalg.norm(v[0]) * L_a[0] * 40.0 * 0.5 * p.dt
    out = orc.jump_halfstep(p, topo, q, v, rp, col, step=1, phase=orc.PH_JB, ev_cap=10**6)
    ev = out["events"]
    counts = np.bincount(ev["atom"] // 2, minlength=20000)
    kmax = int(stats.poisson.ppf(1 - 1e-6, mu))
    obs = np.array([(counts == k).sum() for k in range(kmax)] + [(counts >= kmax).sum()])
    pk = np.array([stats.poisson.pmf(k, mu) for k in range(kmax)] + [stats.poisson.sf(kmax - 1, mu)])
    exp = pk * counts.size
    keep = exp > 5
    chi2 = (((obs - exp) ** 2 / exp)[keep]).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4
    assert counts.mean() == pytest.approx(mu, rel=5 * math.sqrt(mu / counts.size) / mu)
    # proposals are numbered 1..M for each atom, in order
    for a in (0, 2, 4):
        ks = ev["k"][ev["atom"] == a]
        assert np.array_equal(ks, np.arange(1, ks.size + 1))


@pytest.mark.parametrize("scale", [2.0, 10.0])
def test_thinning_law_independent_of_bound(orc, scale):
    base = _pairs(orc, 30000, 6.5, [-0.06, 0.0, 0.03])
    p1, topo, q, v, rp, col = base
    o1 = orc.jump_halfstep(p1, topo, q, v, rp, col, step=5, phase=orc.PH_JA)
    p2 = _pairs(orc, 30000, 6.5, [-0.06, 0.0, 0.03], bound_scale=scale)[0]
    o2 = orc.jump_halfstep(p2, topo, q, v, rp, col, step=5, phase=orc.PH_JA)
    f1 = np.any(o1["v"][0::2] != v[0::2], axis=1).mean()
    f2 = np.any(o2["v"][0::2] != v[0::2], axis=1).mean()
    se = math.sqrt(f1 * (1 - f1) / 30000 * 2)
    assert abs(f1 - f2) < 5 * se
    r = o2["counters"]["proposals"] / o1["counters"]["proposals"]
    assert r == pytest.approx(scale, rel=0.05)


def _replay_compensator(orc, p, topo, q, v, rp, col, ev):
    """Sum of acceptance probabilities lambda/lambda* over the logged proposals,
    replaying each atom's chain with an independent numpy force evaluation."""
    from scipy import special
    _, L_a = orc.rate_bounds(p)
    L_a = L_a * p.bound_scale
    rc, ron, roff = p.r_cut, p.r_on, p.r_off
    charge = np.array(p.charge[:p.n_types])
    total_p, var, acc = 0.0, 0.0, 0
    vv = v.copy()
    for e in ev:
        i, j = int(e["atom"]), int(e["partner"])
        d = q[i] - q[j]
        r = np.linalg.norm(d)
        ti, tj = topo.type[i], topo.type[j]
        F = np.zeros(3)
        if ron < r < rc:
            qq = KE * charge[ti] * charge[tj]
            du = lambda x: -qq / x**2
            x = (r - ron) / (roff - ron)
            ch = 1.0 if x >= 1 else x**3 * (10 - 15 * x + 6 * x * x)
            F = ch * (du(r) - du(rc)) * d / r
        v0 = np.linalg.norm(vv[i])
        pr = max(0.0, vv[i] @ F) / (v0 * L_a[ti])
        assert pr <= 1.0 + 1e-9
        # the logged accept-test margin U |v| L - v.F and its scale |v| |F|:
        # accepted iff the margin is negative, and margin + v.F = U |v| L lies
        # in (0, |v| L)
        s = vv[i] @ F
        assert e["scale"] == pytest.approx(v0 * np.linalg.norm(F), rel=1e-9, abs=1e-300)
        assert (e["margin"] < 0) == bool(e["accepted"])
        ul = e["margin"] + s
        assert -1e-9 * v0 * L_a[ti] < ul < v0 * L_a[ti] * (1 + 1e-9)
        if e["accepted"]:
            assert pr > 0
            vv[i] = vv[i] - 2 * (vv[i] @ F) / (F @ F) * F
            acc += 1
        total_p += pr
        var += pr * (1 - pr)
    return total_p, var, acc


def test_compensator_of_accepted_events(orc):
    from workloads import water_droplet
    sys = water_droplet(n_waters=64, seed=4)
    p = orc.make_params(sys, charge=[-0.834, 0.417], eps=[0.0, 0.0], sigma=[0.0, 0.0],
                        coulomb=orc.COUL_BARE, r_on=4.0, r_off=5.0)
    topo = orc.Topology.from_system(sys)
    order, _ = orc.sort_order(p, sys.pos)
    rp, col = orc.build_list(p, topo, sys.pos, p.r_on - p.skin, p.r_cut + p.skin, order)
    tot, var, acc = 0.0, 0.0, 0
    for step in range(6):
        out = orc.jump_halfstep(p, topo, sys.pos, sys.vel * 3.0, rp, col, step=step,
                                phase=orc.PH_JA, ev_cap=10**6)
        a, b, c = _replay_compensator(orc, p, topo, sys.pos, sys.vel * 3.0, rp, col, out["events"])
        tot, var, acc = tot + a, var + b, acc + c
        assert c == out["counters"]["accepted"]
    assert acc > 200
    assert abs(acc - tot) < 5 * math.sqrt(var)


def test_mean_force_identity(orc):
    """For v ~ N(0, kT/m) at fixed q, E[dv] over a short J step equals the B-step
    kick -t F/m to first order in t (the jump generator reproduces L_B on average)."""
    n = 400000
    r = 6.2
    p, topo, q, v, rp, col = _pairs(orc, n, r, [0.0, 0.0, 0.0], charge=(-0.834,))
    m = 15.999
    sd = math.sqrt(KB * 300.0 * ACC / m)
    rng = np.random.default_rng(11)
    v[0::2] = rng.standard_normal((n, 3)) * sd
    Fx = _grad_x(orc, p, r)
    out = orc.jump_halfstep(p, topo, q, v, rp, col, step=0, phase=orc.PH_JA)
    dv = (out["v"][0::2] - v[0::2])[:, 0]
    t = 0.5 * p.dt
    expect = -t * ACC * Fx / m
    se = dv.std() / math.sqrt(n)
    assert abs(dv.mean() - expect) < 5 * se + 0.03 * abs(expect)


def test_expected_proposals_match_cost_model(orc):
    from workloads import water_box
    sys = water_box(n_side=6, box_len=18.6, seed=3)
    p = orc.make_params(sys, r_on=4.0, r_off=5.0, r_cut=8.0, skin=1.0)
    topo = orc.Topology.from_system(sys)
    order, _ = orc.sort_order(p, sys.pos)
    rp, col = orc.build_list(p, topo, sys.pos, p.r_on - p.skin, p.r_cut + p.skin, order)
    _, L_a = orc.rate_bounds(p)
    beta = 1.0 / (KB * 300.0)
    mu = np.diff(rp) * beta * np.linalg.norm(sys.vel, axis=1) * L_a[sys.atom_type] * 0.5 * p.dt
    tot = 0
    for step in range(20):
        out = orc.jump_halfstep(p, topo, sys.pos, sys.vel, rp, col, step=step, phase=orc.PH_JB)
        tot += out["counters"]["proposals"]
    expect = 20 * mu.sum()
    assert abs(tot - expect) < 5 * math.sqrt(expect)

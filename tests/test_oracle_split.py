"""Pins of the separate Coulomb and Lennard-Jones jump mechanisms (Sec. V: the
long-range Coulomb and van der Waals forces are both handled by jumps, with
bounds per pair of types and a switch per interaction; Sec. VI counts the VdW
jumps on their own; Sec. II.B: independent Poisson clocks superpose).

With jump_split each directed pair (i, j) carries two mechanisms: Coulomb,
field chi_C(r) q_i q_j k_e (g'(r) - g'(rc)) d/r with chi_C on [r_on, r_off], and
Lennard-Jones, field chi_V(r) (LJ'(r) - LJ'(rc)) d/r with chi_V on
[r_on_lj, r_off_lj], with the bounds L_C(a,b), L_V(a,b).  One Poisson count of
mean beta |v| dt/2 sum over (mechanism, partner) of the bounds, each proposal
picking (m, j) in proportion to its bound."""
import math

import numpy as np
import pytest
from scipy import stats

KB, KE = 0.0019872041, 332.0637
CHARGE, EPS, SIGMA = [-0.834, 0.417], [0.152, 0.0], [3.15, 0.0]


def _system(orc, n_waters=64, seed=4, charge=CHARGE, eps=EPS, split=1, rate_mode=None,
            win_c=(4.0, 5.0), win_v=(3.5, 4.5)):
    from workloads import water_droplet
    sys = water_droplet(n_waters=n_waters, seed=seed)
    p = orc.make_params(sys, coulomb=orc.COUL_BARE, r_on=win_c[0], r_off=win_c[1],
                        charge=list(charge), eps=list(eps), sigma=SIGMA, jump_split=split,
                        r_on_lj=win_v[0], r_off_lj=win_v[1],
                        rate_mode=orc.RATE_PAIR if rate_mode is None else rate_mode)
    topo = orc.Topology.from_system(sys)
    order, _ = orc.sort_order(p, sys.pos)
    rmin = min(win_c[0], win_v[0] if split else win_c[0]) - p.skin
    rp, col = orc.build_list(p, topo, sys.pos, rmin, p.r_cut + p.skin, order)
    return sys, p, topo, rp, col


def _smooth(lo, hi, r):
    x = (r - lo) / (hi - lo)
    return 0.0 if x <= 0 else (1.0 if x >= 1 else x ** 3 * (10 - 15 * x + 6 * x * x))


def _parts(p, a, b, r):
    """Coulomb and LJ parts of W'_sf (bare Coulomb), independently in numpy."""
    rc = p.r_cut
    qq = KE * p.charge[a] * p.charge[b]
    eps = math.sqrt(p.eps[a] * p.eps[b])
    sig = 0.5 * (p.sigma[a] + p.sigma[b])
    dlj = lambda x: 4 * eps * (-12 * sig ** 12 / x ** 13 + 6 * sig ** 6 / x ** 7)
    return qq * (-1 / r ** 2 + 1 / rc ** 2), dlj(r) - dlj(rc)


def _field(p, m, q, i, j, ti, tj):
    d = q[i] - q[j]
    r = np.linalg.norm(d)
    lo, hi = (p.r_on, p.r_off) if m == 0 else (p.r_on_lj, p.r_off_lj)
    if not (lo < r < p.r_cut):
        return np.zeros(3)
    wc, wv = _parts(p, ti, tj, r)
    return _smooth(lo, hi, r) * (wc if m == 0 else wv) * d / r


def _bounds(orc, p):
    """L'[a, m n_types + b] = Lq unit_a as the oracle uses them."""
    Lq, unit = orc.rate_weights(p)
    return Lq.astype(np.float64) * unit[:, None]


def test_bounds_per_mechanism(orc):
    _, p, _, _, _ = _system(orc)
    L, L_a = orc.rate_bounds(p)
    assert L.shape == (2, 2, 2)
    # no LJ between types with eps = 0: no Lennard-Jones bound
    assert L[1, 0, 1] == 0.0 and L[1, 1, 0] == 0.0 and L[1, 1, 1] == 0.0
    # brute force on a finer grid, independent field parts
    for m, (lo, hi) in enumerate(((p.r_on, p.r_off), (p.r_on_lj, p.r_off_lj))):
        r = np.arange(lo, p.r_cut, 2e-5)
        for a in range(2):
            for b in range(2):
                f = [abs(_smooth(lo, hi, x) * _parts(p, a, b, x)[m]) for x in r]
                mx = max(f)
                if mx == 0.0:
                    assert L[m, a, b] == 0.0
                    continue
                assert L[m, a, b] >= mx * (1 + 1e-3) * (1 - 1e-6)
                assert L[m, a, b] <= mx * (1 + 1e-3) * (1 + 1e-6)
    np.testing.assert_array_equal(L_a, L.max(axis=(0, 2)))
    Lb = _bounds(orc, p)
    for m in range(2):
        assert np.all(Lb[:, 2 * m:2 * m + 2] >= L[m] - 1e-4 * Lb.max(axis=1)[:, None] * 2 ** -20)


@pytest.mark.parametrize("without", ["lj", "coulomb"])
def test_split_reduces_to_the_combined_mechanism(orc, without):
    """Without LJ (eps = 0) only the Coulomb mechanism has a bound, and without
    charges only the LJ one; with the same switch window the split process is
    then the combined one (per-type-pair bounds): the same proposals, partners,
    accept decisions and, up to rounding, velocities."""
    charge = CHARGE if without == "lj" else [0.0, 0.0]
    eps = [0.0, 0.0] if without == "lj" else [5.0, 0.0]
    outs = []
    for split in (0, 1):
        sys, p, topo, rp, col = _system(orc, charge=charge, eps=eps, split=split,
                                        win_c=(4.0, 5.0), win_v=(4.0, 5.0))
        outs.append(orc.jump_halfstep(p, topo, sys.pos, sys.vel * 6.0, rp, col, step=3,
                                      phase=orc.PH_JA, ev_cap=10**6))
    a, b = outs
    assert a["counters"]["proposals"] > 100
    keys = ("step", "phase", "atom", "k", "partner", "accepted")
    for k in keys:
        np.testing.assert_array_equal(a["events"][k], b["events"][k])
    np.testing.assert_allclose(a["v"], b["v"], rtol=1e-12, atol=1e-15)
    assert a["counters"] == b["counters"]
    assert np.all(b["events"]["mech"] == (0 if without == "lj" else 1))


def test_split_compensator(orc):
    """Sum over logged proposals of lambda / L' with each proposal's own
    mechanism field and bound (independent numpy evaluation) matches the number
    of accepted events; replaying the reflections reproduces the velocities."""
    sys, p, topo, rp, col = _system(orc, eps=[1.5, 0.0])   # strong LJ: both mechanisms propose
    Lb = _bounds(orc, p)
    tot, var, acc, per_mech = 0.0, 0.0, 0, [0, 0]
    v_in = sys.vel * 3.0
    for step in range(6):
        out = orc.jump_halfstep(p, topo, sys.pos, v_in, rp, col, step=step, phase=orc.PH_JA,
                                ev_cap=10**6)
        vv = v_in.copy()
        for e in out["events"]:
            i, j, m = int(e["atom"]), int(e["partner"]), int(e["mech"])
            ti, tj = topo.type[i], topo.type[j]
            F = _field(p, m, sys.pos, i, j, ti, tj)
            pr = max(0.0, vv[i] @ F) / (np.linalg.norm(vv[i]) * Lb[ti, m * 2 + tj])
            assert pr <= 1.0 + 1e-9
            if e["accepted"]:
                assert pr > 0
                vv[i] = vv[i] - 2 * (vv[i] @ F) / (F @ F) * F
                acc += 1
            per_mech[m] += 1
            tot += pr
            var += pr * (1 - pr)
        np.testing.assert_allclose(vv, out["v"], rtol=1e-11, atol=1e-14)
    assert acc > 200 and min(per_mech) > 100
    assert abs(acc - tot) < 5 * math.sqrt(var)


def test_split_proposal_counts_and_classes(orc):
    """Proposals per atom have mean beta |v| dt/2 sum over (m, j) of L'; the
    proposal lands in class (m, b) with probability n_b L'_{m a b} / sum."""
    sys, p, topo, rp, col = _system(orc, n_waters=100, seed=7, eps=[1.5, 0.0])
    Lb = _bounds(orc, p)
    beta = 1.0 / (KB * p.temperature)
    v = sys.vel * 3.0
    n = topo.n
    nb = np.zeros((n, 2))
    for i in range(n):
        nb[i] = np.bincount(topo.type[col[rp[i]:rp[i + 1]]], minlength=2)
    ncls = np.concatenate([nb, nb], axis=1)                  # classes m * 2 + b
    rate = (ncls * Lb[topo.type]).sum(axis=1)
    mu = beta * np.linalg.norm(v, axis=1) * rate * 0.5 * p.dt
    steps = 30
    per_cls = np.zeros((n, 4))
    total = 0
    for step in range(steps):
        out = orc.jump_halfstep(p, topo, sys.pos, v, rp, col, step=step, phase=orc.PH_JB,
                                ev_cap=10**6)
        ev = out["events"]
        total += len(ev)
        np.add.at(per_cls, (ev["atom"], ev["mech"] * 2 + topo.type[ev["partner"]]), 1)
    expect = steps * mu.sum()
    assert abs(total - expect) < 5 * math.sqrt(expect)
    for a in (0, 1):
        sel = topo.type == a
        e_c = (steps * mu[sel, None] * ncls[sel] * Lb[a][None, :] / rate[sel, None]).sum(axis=0)
        o_c = per_cls[sel].sum(axis=0)
        keep = e_c > 0
        assert np.all(o_c[~keep] == 0)          # no proposal of a class without a bound
        chi2 = ((o_c[keep] - e_c[keep]) ** 2 / e_c[keep]).sum()
        assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4, (a, o_c, e_c)


def test_split_gradient_parts(orc):
    """Short-range and long-range gradients with a window per interaction:
    SHORT + LONG = FULL, and SHORT = sum_j [(1 - chi_C) W'_C + (1 - chi_V) W'_V] d/r
    (independent numpy sum) on a small droplet."""
    sys, p, topo, _, _ = _system(orc, n_waters=27, seed=2, eps=[1.5, 0.0])
    q = sys.pos
    gs = orc.gradient(p, topo, q, orc.G_SHORT)
    gl = orc.gradient(p, topo, q, orc.G_LONG)
    gf = orc.gradient(p, topo, q, orc.G_FULL)
    np.testing.assert_allclose(gs + gl, gf, rtol=1e-10, atol=1e-10)
    excl = {(int(a), int(b)) for a, b in sys.excl} | {(int(b), int(a)) for a, b in sys.excl}
    ref = np.zeros_like(q)
    for i in range(topo.n):
        for j in range(topo.n):
            if i == j or (i, j) in excl:
                continue
            d = q[i] - q[j]
            r = np.linalg.norm(d)
            if r >= p.r_cut:
                continue
            wc, wv = _parts(p, topo.type[i], topo.type[j], r)
            s = 0.0
            if r < p.r_off:
                s += (1 - _smooth(p.r_on, p.r_off, r)) * wc
            if r < p.r_off_lj:
                s += (1 - _smooth(p.r_on_lj, p.r_off_lj, r)) * wv
            ref[i] += s * d / r
    np.testing.assert_allclose(gs, ref, rtol=1e-9, atol=1e-9)

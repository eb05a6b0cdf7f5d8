"""Pins of the oracle's integrator (Sec. III.C splitting, Sec. IV.B B J A O A J B):
reduction to BAOAB when no pair is long-range, BAOAB's exact configurational
sampling of a harmonic potential, canonical invariants of a small Lennard-Jones
gas against an independent Metropolis Monte Carlo, and bitwise determinism /
resume of the counter-based random stream."""
import math

import numpy as np
import pytest

from workloads import water_box, water_droplet

KB, ACC = 0.0019872041, 4.184e-4


def test_bounce_without_long_range_is_baoab_bitwise(orc):
    sys = water_droplet(n_waters=27, seed=7)
    topo = orc.Topology.from_system(sys)
    # r' >= rc + s: every candidate list is empty and chi = 0 below the cutoff
    pb = orc.make_params(sys, integrator=orc.BOUNCE, r_on=11.5, r_off=12.0, r_cut=9.0, skin=2.0)
    pa = orc.make_params(sys, integrator=orc.BAOAB, r_cut=9.0, skin=2.0)
    ob = orc.run(pb, topo, sys.pos, sys.vel, 0, 30)
    oa = orc.run(pa, topo, sys.pos, sys.vel, 0, 30)
    assert ob["status"] == 0 and oa["status"] == 0
    assert ob["counters"]["proposals"] == 0
    assert np.array_equal(ob["q"], oa["q"]) and np.array_equal(ob["v"], oa["v"])


def test_run_is_deterministic_and_resumable(orc):
    sys = water_droplet(n_waters=40, seed=8)
    topo = orc.Topology.from_system(sys)
    p = orc.make_params(sys, rebuild_interval=10)
    a = orc.run(p, topo, sys.pos, sys.vel, 0, 40, ev_cap=10**6)
    b = orc.run(p, topo, sys.pos, sys.vel, 0, 40, ev_cap=10**6)
    assert np.array_equal(a["q"], b["q"]) and np.array_equal(a["v"], b["v"])
    assert np.array_equal(a["events"], b["events"])
    c1 = orc.run(p, topo, sys.pos, sys.vel, 0, 20)
    c2 = orc.run(p, topo, c1["q"], c1["v"], 20, 20)
    assert np.array_equal(a["q"], c2["q"]) and np.array_equal(a["v"], c2["v"])
    assert a["counters"]["proposals"] > 0 and a["counters"]["accepted"] > 0


def test_skin_violation_is_reported(orc):
    sys = water_droplet(n_waters=8, seed=9)
    topo = orc.Topology.from_system(sys)
    p = orc.make_params(sys, skin=0.01, rebuild_interval=1000)
    out = orc.run(p, topo, sys.pos, sys.vel, 0, 50)
    assert out["status_name"] == "SKIN"


def test_baoab_harmonic_configurational_sampling(orc):
    """E = k |q1 - q2|^2 (a bond with r0 = 0) is harmonic in Cartesian space;
    BAOAB samples its configurations exactly: <|d|^2> = 3 / (2 beta k)."""
    npair = 400
    q = np.zeros((2 * npair, 3))
    q[0::2, 0] = np.arange(npair) * 50.0
    q[1::2, 0] = np.arange(npair) * 50.0 + 0.3
    bonds = np.stack([np.arange(0, 2 * npair, 2), np.arange(1, 2 * npair, 2)], 1)
    k = 20.0
    topo = orc.Topology(np.zeros(2 * npair, np.int32), np.tile([16.0, 1.008], npair), bonds,
                        np.full(npair, k), np.zeros(npair), excl=bonds)
    grid = dict(grid_origin=[-100.0, -100.0, -100.0], grid_dims=[npair + 4, 4, 4], cell_size=50.0)
    p = orc.make_params(None, integrator=orc.BAOAB, charge=[0.0], eps=[0.0], sigma=[0.0],
                        periodic=False, dt=2.0, gamma=0.05, r_cut=1.0, skin=1e3,
                        rebuild_interval=10**9, **grid)
    v = np.zeros_like(q)
    o = orc.run(p, topo, q, v, 0, 500)
    assert o["status"] == 0
    qq, vv = o["q"], o["v"]
    samples = []
    for blk in range(40):
        o = orc.run(p, topo, qq, vv, 500 + 100 * blk, 100)
        assert o["status"] == 0
        qq, vv = o["q"], o["v"]
        d = qq[0::2] - qq[1::2]
        samples.append(np.einsum("ij,ij->i", d, d).mean())
    s = np.array(samples)
    beta = 1.0 / (KB * 300.0)
    expect = 3.0 / (2.0 * beta * k)
    assert abs(s.mean() - expect) < 5 * s.std(ddof=1) / math.sqrt(s.size) + 0.002 * expect


def _lj_gas(n_side=3, box=15.0, seed=0):
    rng = np.random.default_rng(seed)
    g = (np.arange(n_side) + 0.5) * box / n_side
    q = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    q += rng.normal(0, 0.2, q.shape)
    return q


def _mc_mean_energy(q0, box, eps, sig, rc, beta, sweeps, seed):
    """Independent Metropolis Monte Carlo of the shifted-force LJ gas."""
    rng = np.random.default_rng(seed)
    n = q0.shape[0]

    def wsf(r):
        u = lambda x: 4 * eps * ((sig / x) ** 12 - (sig / x) ** 6)
        du = lambda x: 4 * eps * (-12 * (sig / x) ** 12 + 6 * (sig / x) ** 6) / x
        return np.where(r < rc, u(r) - u(rc) - (r - rc) * du(rc), 0.0)

    def e_atom(q, i):
        d = q[i] - q
        d -= box * np.rint(d / box)
        r = np.sqrt(np.einsum("ij,ij->i", d, d))
        r[i] = 10 * rc
        return wsf(r).sum()

    q = q0.copy()
    es = []
    step = 0.6
    for s in range(sweeps):
        for i in range(n):
            old = q[i].copy()
            e0 = e_atom(q, i)
            q[i] = old + rng.uniform(-step, step, 3)
            e1 = e_atom(q, i)
            if rng.random() >= math.exp(min(0.0, -beta * (e1 - e0))):
                q[i] = old
        if s >= sweeps // 5:
            d = q[:, None] - q[None]
            d -= box * np.rint(d / box)
            r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
            r[np.arange(n), np.arange(n)] = 10 * rc
            es.append(0.5 * wsf(r).sum())
    return np.array(es)


@pytest.mark.slow
def test_lj_gas_canonical_invariants(orc):
    """Small periodic LJ gas (27 argon-like atoms, supercritical): BOUNCE with
    long-range jumps active keeps <T_kin> = T and reproduces the canonical mean
    potential energy of an independent Metropolis Monte Carlo."""
    box, eps, sig, rc, mass, T = 15.0, 0.238, 3.4, 7.0, 39.948, 300.0
    q0 = _lj_gas(3, box)
    n = q0.shape[0]
    topo = orc.Topology(np.zeros(n, np.int32), np.full(n, mass))
    p = orc.make_params(None, integrator=orc.BOUNCE, charge=[0.0], eps=[eps], sigma=[sig],
                        periodic=True, box=[box] * 3, cell_size=5.0, coulomb=orc.COUL_BARE,
                        dt=2.0, gamma=0.01, temperature=T, r_on=3.6, r_off=4.4, r_cut=rc,
                        skin=0.5, rebuild_interval=2, seed=1)
    rng = np.random.default_rng(2)
    v = rng.standard_normal((n, 3)) * math.sqrt(KB * T * ACC / mass)
    q = q0.copy()
    o = orc.run(p, topo, q, v, 0, 2000)
    q, v = o["q"], o["v"]
    epot, tkin = [], []
    props = acc = 0
    for blk in range(300):
        o = orc.run(p, topo, q, v, 2000 + 100 * blk, 100)
        assert o["status"] == 0
        q, v = o["q"], o["v"]
        props += o["counters"]["proposals"]
        acc += o["counters"]["accepted"]
        e = orc.energies(p, topo, q, v)
        epot.append(e["pair"])
        tkin.append(e["tkin"])
    epot, tkin = np.array(epot), np.array(tkin)
    assert acc > 1000  # the jump mechanism is active
    se_t = tkin.std(ddof=1) / math.sqrt(tkin.size)
    assert abs(tkin.mean() - T) < 5 * se_t + 0.01 * T
    beta = 1.0 / (KB * T)
    mc = _mc_mean_energy(q0, box, eps, sig, rc, beta, 3000, seed=3)
    se_e = math.hypot(epot.std(ddof=1) / math.sqrt(epot.size / 2),
                      mc.std(ddof=1) / math.sqrt(mc.size / 20))
    assert abs(epot.mean() - mc.mean()) < 5 * se_e + 0.02 * abs(mc.mean())

"""GPU parity of the separate Coulomb and Lennard-Jones jump mechanisms
(jump_split, Sec. V / Sec. VI) against the oracle: bounds and integer weights,
lists with the two windows, short- and long-range gradients, FP64 jump
half-steps and trajectories with identical events (mechanism included), and
the FP32 event log up to a near-tie."""
import numpy as np
import pytest

from helpers import (BOX, DROPLET, event_keys, first_divergence, gpu_sim, oracle_params,
                     rel_err, relaxed_box, relaxed_droplet)
from workloads import jitter_positions

pytestmark = pytest.mark.gpu

# droplets: Coulomb window 5/6 A (bare), Lennard-Jones window 4/5 A; boxes:
# Coulomb 6/7 A (erfc), Lennard-Jones 5/6 A
DROP_S = dict(DROPLET, jump_split=1, r_on_lj=4.0, r_off_lj=5.0)
BOX_S = dict(BOX, jump_split=1, r_on_lj=5.0, r_off_lj=6.0)
KEYS = ("step", "phase", "atom", "k", "partner", "accepted", "mech")


@pytest.fixture(scope="module")
def droplet():
    return relaxed_droplet("c0")


@pytest.fixture(scope="module")
def box():
    return relaxed_box("b8")


def _sys(droplet, box, which):
    return (droplet, DROP_S) if which == "drop" else (box, BOX_S)


@pytest.mark.parametrize("which", ["drop", "box"])
def test_bounds_and_weights(orc, droplet, box, which):
    sys, cfg = _sys(droplet, box, which)
    sim = gpu_sim(sys, cfg)
    lab, la = sim.rate_bounds()
    p = oracle_params(orc, sys, cfg)
    olab, ola = orc.rate_bounds(p)
    assert lab.shape == (2, 2, 2)
    np.testing.assert_allclose(lab, olab, rtol=1e-12, atol=0)
    np.testing.assert_allclose(la, ola, rtol=1e-12)
    lq, unit = sim.rate_weights()
    olq, ounit = orc.rate_weights(p)
    assert np.array_equal(lq, olq)
    np.testing.assert_allclose(unit, ounit, rtol=1e-12)


@pytest.mark.parametrize("which", ["drop", "box"])
def test_lists_bit_exact(orc, droplet, box, which):
    import paper_2002_07109_amd as B
    sys, cfg = _sys(droplet, box, which)
    sim = gpu_sim(sys, cfg, fp64=True)
    sim.jump_halfstep(0, B.PH_JA)
    p = oracle_params(orc, sys, cfg)
    topo = orc.Topology.from_system(sys)
    order, _ = orc.sort_order(p, sys.pos)
    r_short = max(cfg["r_off"], cfg["r_off_lj"])
    r_long = min(cfg["r_on"], cfg["r_on_lj"])
    for which_list, (rmin, rmax) in [(B.LIST_FORCE, (0.0, r_short + cfg["skin"])),
                                     (B.LIST_CAND, (r_long - cfg["skin"],
                                                    cfg["r_cut"] + cfg["skin"]))]:
        grp, gcol = sim.get_list(which_list)
        orp, ocol = orc.build_list(p, topo, sys.pos, rmin, rmax, order)
        assert np.array_equal(grp, orp)
        assert np.array_equal(gcol, ocol)


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("which", ["drop", "box"])
def test_gradients(orc, droplet, box, which, fp64):
    import paper_2002_07109_amd as B
    sys, cfg = _sys(droplet, box, which)
    sim = gpu_sim(sys, cfg, fp64=fp64)
    q = jitter_positions(sys.pos, 0.05, seed=11)
    sim.set_state(pos=q)
    p = oracle_params(orc, sys, cfg)
    topo = orc.Topology.from_system(sys)
    tol = 1e-11 if fp64 else 1e-5
    for gbit, obit in [(B.G_SHORT, orc.G_SHORT), (B.G_LONG, orc.G_LONG), (B.G_FULL, orc.G_FULL),
                       (B.G_STEP, orc.G_SHORT)]:
        g = sim.gradient(gbit).cpu().numpy()
        err = rel_err(g, orc.gradient(p, topo, q, obit))
        print(f"{which} fp64={fp64} part {gbit}: {err:.3e}")
        assert err < tol, (gbit, err)


@pytest.mark.parametrize("which", ["drop", "box"])
def test_jump_halfstep_events_bit_exact(orc, droplet, box, which):
    import paper_2002_07109_amd as B
    sys, cfg = _sys(droplet, box, which)
    cfg = dict(cfg, r_on=4.0, r_off=5.0, r_on_lj=3.5, r_off_lj=4.5)     # many proposals
    sim = gpu_sim(sys, cfg, fp64=True, log_events=True, event_capacity=4_000_000)
    p = oracle_params(orc, sys, cfg)
    topo = orc.Topology.from_system(sys)
    order, _ = orc.sort_order(p, sys.pos)
    rp, col = orc.build_list(p, topo, sys.pos, 3.5 - cfg["skin"], cfg["r_cut"] + cfg["skin"], order)
    v = sys.vel.copy()
    all_o = []
    for step, phase in [(0, B.PH_JA), (0, B.PH_JB), (7, B.PH_JA)]:
        sim.jump_halfstep(step, phase)
        out = orc.jump_halfstep(p, topo, sys.pos, v, rp, col, step, phase, ev_cap=4_000_000)
        assert out["status"] == 0
        v = out["v"]
        all_o.append(out["events"])
        np.testing.assert_allclose(sim.vel.cpu().numpy(), v, rtol=0, atol=1e-14)
    ev, n = sim.events()
    o = np.concatenate(all_o)
    assert n == o.size and n > 1000
    assert np.array_equal(event_keys(ev, KEYS), event_keys(o, KEYS))
    assert (o["mech"] == 1).sum() > 0 and (o["mech"] == 0).sum() > 100


@pytest.mark.parametrize("which,nsteps", [("drop", 100), ("box", 100)])
def test_trajectory_fp64(orc, droplet, box, which, nsteps):
    sys, cfg = _sys(droplet, box, which)
    sim = gpu_sim(sys, cfg, fp64=True, log_events=True, event_capacity=4_000_000, use_graph=True)
    sim.step(nsteps)
    sim.sync()
    o = orc.run(oracle_params(orc, sys, cfg), orc.Topology.from_system(sys), sys.pos, sys.vel, 0,
                nsteps, ev_cap=4_000_000)
    assert o["status"] == 0, o["status_name"]
    assert np.abs(sim.pos.cpu().numpy() - o["q"]).max() <= 1e-6
    assert np.abs(sim.vel.cpu().numpy() - o["v"]).max() <= 1e-6
    ev, n = sim.events()
    assert n == o["n_events"] and n > 0
    assert np.array_equal(event_keys(ev, KEYS), event_keys(o["events"], KEYS))
    c = sim.counters()
    assert c["proposals"] == o["counters"]["proposals"] and c["bound_violations"] == 0


@pytest.mark.parametrize("which", ["drop", "box"])
def test_fp32_events_follow_oracle(orc, droplet, box, which):
    sys, cfg = _sys(droplet, box, which)
    sim = gpu_sim(sys, cfg, fp64=False, log_events=True, event_capacity=4_000_000, use_graph=True)
    sim.step(50)
    sim.sync()
    o = orc.run(oracle_params(orc, sys, cfg), orc.Topology.from_system(sys), sys.pos, sys.vel, 0,
                50, ev_cap=4_000_000)
    assert o["status"] == 0
    ev, n = sim.events()
    div = first_divergence(ev, o["events"])
    print(f"{which}: {n} events (oracle {o['n_events']}), first divergence {div}")
    if div is None:
        assert n == o["n_events"]
        return
    for atom, k, oe in div[2]:
        assert oe is not None
        assert abs(oe["margin"]) < 1e-5 * oe["scale"], (atom, k)

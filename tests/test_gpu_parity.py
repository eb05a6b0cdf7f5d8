"""GPU path (through the C ABI) against the FP64 oracle on the same seeded inputs.

Tolerances (max_i |dF_i| / RMS_i |F_i| for per-atom vectors, each force part
against its own RMS): FP64 pair arithmetic 1e-11 (summation order only), FP32
pair arithmetic 1e-5; pair energies in FP32 within 2e-6 of the sum over pairs of
|u_pair|.  Lists and, in FP64, jump events are compared bit for bit; FP32 event
logs must match the oracle until the first accept test whose oracle margin is a
near-tie (|U |v| L - v.F| < 1e-5 |v| |F|)."""
import math

import numpy as np
import pytest

from helpers import (BOX, DROPLET, FF, event_keys, first_divergence, gpu_sim, oracle_params,
                     rel_err, relaxed_box, relaxed_droplet, sum_abs_pair_energy)
from workloads import jitter_positions, water_box, water_droplet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def droplet():
    return relaxed_droplet("c0")


@pytest.fixture(scope="module")
def box():
    return relaxed_box("b8")


def _sys(droplet, box, which):
    return (droplet, DROPLET) if which == "drop" else (box, BOX)


@pytest.mark.parametrize("which", ["drop", "box"])
def test_rate_bounds_match_oracle(orc, droplet, box, which):
    sys, cfg = _sys(droplet, box, which)
    sim = gpu_sim(sys, cfg)
    lab, la = sim.rate_bounds()
    olab, ola = orc.rate_bounds(oracle_params(orc, sys, cfg))
    np.testing.assert_allclose(lab, olab, rtol=1e-12)
    np.testing.assert_allclose(la, ola, rtol=1e-12)


@pytest.mark.parametrize("which", ["drop", "box"])
def test_lists_bit_exact(orc, droplet, box, which):
    import paper_2002_07109_amd as B
    sys, cfg = _sys(droplet, box, which)
    sim = gpu_sim(sys, cfg, fp64=True)
    sim.jump_halfstep(0, B.PH_JA)       # builds the lists at q_0 (velocities change only)
    p = oracle_params(orc, sys, cfg)
    topo = orc.Topology.from_system(sys)
    order, _ = orc.sort_order(p, sys.pos)
    for which_list, (rmin, rmax) in [(B.LIST_FORCE, (0.0, cfg["r_off"] + cfg["skin"])),
                                     (B.LIST_CAND, (cfg["r_on"] - cfg["skin"],
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
    q = jitter_positions(sys.pos, 0.05, seed=11)      # bonds and angles off their minima
    sim.set_state(pos=q)
    p = oracle_params(orc, sys, cfg)
    topo = orc.Topology.from_system(sys)
    tol = 1e-11 if fp64 else 1e-5
    # each part's error against that part's own RMS
    for gbit, obit in [(B.G_SHORT, orc.G_SHORT), (B.G_LONG, orc.G_LONG), (B.G_FULL, orc.G_FULL),
                       (B.G_BONDED, orc.G_BONDED), (B.G_BONDED | B.G_SHORT,
                                                    orc.G_BONDED | orc.G_SHORT)]:
        g = sim.gradient(gbit).cpu().numpy()
        o = orc.gradient(p, topo, q, obit)
        err = rel_err(g, o)
        print(f"{which} fp64={fp64} part {gbit}: max|dF|/RMS|F| = {err:.3e}")
        assert err < (1e-13 if gbit == B.G_BONDED else tol), (gbit, err)


@pytest.mark.parametrize("integrator", [0, 1])
@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("which", ["drop", "box"])
def test_step_pair_force(orc, droplet, box, which, fp64, integrator):
    """The pair part of F_0 exactly as the integrator computes it (its own
    force list and pair kernel: with FP32 pair arithmetic over the fixed-point
    position mirror) against the oracle's SHORT (BOUNCE) or
    FULL (BAOAB) pair gradient: from a fresh build at jittered positions, and
    after 7 steps with the list and position mirrors the steps maintained (the
    oracle at its own positions after the same 7 steps)."""
    import paper_2002_07109_amd as B
    sys, cfg = _sys(droplet, box, which)
    cfg = dict(cfg, integrator=integrator)
    p = oracle_params(orc, sys, cfg)
    topo = orc.Topology.from_system(sys)
    obit = orc.G_SHORT if integrator == 0 else orc.G_FULL
    sim = gpu_sim(sys, cfg, fp64=fp64)
    q = jitter_positions(sys.pos, 0.05, seed=11)
    sim.set_state(pos=q)
    g = sim.gradient(B.G_STEP).cpu().numpy()
    err = rel_err(g, orc.gradient(p, topo, q, obit))
    print(f"{which} fp64={fp64} integrator={integrator}: step pair force {err:.3e}")
    assert err < (1e-11 if fp64 else 1e-5), err
    sim = gpu_sim(sys, cfg, fp64=fp64)
    sim.step(7)
    sim.sync()
    g7 = sim.gradient(B.G_STEP).cpu().numpy()
    o7 = orc.run(p, topo, sys.pos, sys.vel, 0, 7)
    assert o7["status"] == 0
    err7 = rel_err(g7, orc.gradient(p, topo, o7["q"], obit))
    print(f"  after 7 steps: {err7:.3e}")
    assert err7 < (1e-10 if fp64 else 1e-5), err7


@pytest.mark.parametrize("which", ["drop", "box"])
def test_energies(orc, droplet, box, which):
    sys, cfg = _sys(droplet, box, which)
    sim = gpu_sim(sys, cfg, fp64=True)
    e = sim.energies()[0]
    o = orc.energies(oracle_params(orc, sys, cfg), orc.Topology.from_system(sys), sys.pos, sys.vel)
    for k in ("bond", "angle", "coul", "lj", "pair", "kin", "tkin"):
        assert e[k] == pytest.approx(o[k], rel=1e-11, abs=1e-9), k
    # FP32 pair energies: ~1e-7 relative per pair; the total cancels pair
    # energies of either sign, so the bound is taken against the sum of |u_pair|
    sim32 = gpu_sim(sys, cfg, fp64=False)
    e32 = sim32.energies()[0]
    p = oracle_params(orc, sys, cfg)
    sabs = sum_abs_pair_energy(orc, p, orc.Topology.from_system(sys), sys.pos,
                               sys.box if sys.periodic else None)
    err = abs(e32["pair"] - o["pair"]) / sabs
    print(f"{which}: FP32 pair energy error {err:.3e} of sum |u_pair| = {sabs:.1f}")
    assert err < 2e-6, err


@pytest.mark.parametrize("which", ["drop", "box"])
def test_jump_halfstep_events_bit_exact(orc, droplet, box, which):
    import paper_2002_07109_amd as B
    sys, cfg = _sys(droplet, box, which)
    cfg = dict(cfg, r_on=4.0, r_off=5.0)           # many proposals
    sim = gpu_sim(sys, cfg, fp64=True, log_events=True, event_capacity=4_000_000)
    p = oracle_params(orc, sys, cfg)
    topo = orc.Topology.from_system(sys)
    order, _ = orc.sort_order(p, sys.pos)
    rp, col = orc.build_list(p, topo, sys.pos, cfg["r_on"] - cfg["skin"],
                             cfg["r_cut"] + cfg["skin"], order)
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
    assert np.array_equal(event_keys(ev), event_keys(o))
    assert sim.counters()["accepted"] == int(o["accepted"].sum())


def _traj(orc, sys, cfg, nsteps, fp64, use_graph=False):
    sim = gpu_sim(sys, cfg, fp64=fp64, log_events=True, event_capacity=4_000_000,
                  use_graph=use_graph)
    sim.step(nsteps)
    sim.sync()
    p = oracle_params(orc, sys, cfg)
    o = orc.run(p, orc.Topology.from_system(sys), sys.pos, sys.vel, 0, nsteps, ev_cap=4_000_000)
    assert o["status"] == 0, o["status_name"]
    return sim, o


@pytest.mark.parametrize("which,nsteps", [("drop", 200), ("box", 100)])
def test_trajectory_fp64(orc, droplet, box, which, nsteps):
    sys, cfg = _sys(droplet, box, which)
    sim, o = _traj(orc, sys, cfg, nsteps, fp64=True)
    dq = np.abs(sim.pos.cpu().numpy() - o["q"]).max()
    dv = np.abs(sim.vel.cpu().numpy() - o["v"]).max()
    assert dq <= 1e-6, dq
    assert dv <= 1e-6, dv
    ev, n = sim.events()
    assert n == o["n_events"]
    assert np.array_equal(event_keys(ev), event_keys(o["events"]))
    c = sim.counters()
    assert c["proposals"] == o["counters"]["proposals"]
    assert c["accepted"] == o["counters"]["accepted"]
    assert c["bound_violations"] == 0


@pytest.mark.parametrize("integrator", [0, 1])
def test_trajectory_past_the_far_part_gate(orc, box, integrator):
    """With a 1.2 A skin, over a hundred atoms move more than a quarter skin
    within one rebuild interval (checked on the oracle first), so the force
    rows' far parts come back into the pair sum part-way through each
    interval: the trajectory and the jump events still follow the oracle."""
    cfg = dict(BOX, skin=1.2, integrator=integrator)
    p = oracle_params(orc, box, cfg)
    o10 = orc.run(p, orc.Topology.from_system(box), box.pos, box.vel, 0, cfg["rebuild_interval"])
    moved = np.sqrt(((o10["q"] - box.pos) ** 2).sum(axis=1))
    assert (moved >= 0.5 * (0.5 * cfg["skin"] - 1e-3)).sum() > 50
    sim, o = _traj(orc, box, cfg, 60, fp64=True)
    assert np.abs(sim.pos.cpu().numpy() - o["q"]).max() <= 1e-6
    assert np.abs(sim.vel.cpu().numpy() - o["v"]).max() <= 1e-6
    if integrator == 0:
        ev, n = sim.events()
        assert n == o["n_events"] and n > 0
        assert np.array_equal(event_keys(ev), event_keys(o["events"]))


def test_trajectory_baoab_fp64(orc, droplet):
    cfg = dict(DROPLET, integrator=1, dt=1.0)
    sim, o = _traj(orc, droplet, cfg, 100, fp64=True)
    assert np.abs(sim.pos.cpu().numpy() - o["q"]).max() <= 1e-6


def assert_fp32_events_follow_oracle(ev, o_events, tol=1e-5):
    """FP32 pair arithmetic in the jump field: the event log equals the FP64
    oracle's until the first half-step where they differ, and there every
    atom's first differing proposal is a near-tie of the oracle's accept test,
    |U |v| L - v.F| < tol |v| |F| (FP32 rounding moves v.F by ~1e-7 |v| |F|).
    Returns (number of identical leading events, the divergence or None)."""
    div = first_divergence(ev, o_events)
    if div is None:
        return len(o_events), None
    step, phase, atoms = div
    for atom, k, oe in atoms:
        assert oe is not None, f"step {step} phase {phase} atom {atom}: proposal count differs"
        rel = abs(oe["margin"]) / oe["scale"] if oe["scale"] > 0 else np.inf
        assert rel < tol, (step, phase, atom, k, rel)
    before = int(np.sum(o_events["step"] * 4 + o_events["phase"] < step * 4 + phase))
    return before, div


@pytest.mark.parametrize("which", ["drop", "box"])
def test_trajectory_fp32_events_and_positions(orc, droplet, box, which):
    """FP32 pair arithmetic (fixed-point position mirror) on the proposal-heavy droplet
    (~3,000 proposals a step) and on the periodic box: the event log follows
    the FP64 oracle up to its first near-tie, and positions after 100 steps
    stay close."""
    sys, cfg = _sys(droplet, box, which)
    sim, o = _traj(orc, sys, cfg, 100, fp64=False)
    dq = np.abs(sim.pos.cpu().numpy() - o["q"]).max()
    ev, n = sim.events()
    same, div = assert_fp32_events_follow_oracle(ev, o["events"])
    print(f"FP32 vs FP64 oracle after 100 steps: max |dq| = {dq:.3e} A; events {n} vs "
          f"{o['n_events']}; identical leading events {same}; first divergence {div}")
    if div is None:
        assert n == o["n_events"]
        assert dq < 1e-4, dq
    else:
        assert dq < 1e-2, dq


@pytest.mark.parametrize("which", ["drop", "box"])
def test_graph_replay_equals_direct_launches(orc, droplet, box, which):
    sys, cfg = _sys(droplet, box, which)
    sa = gpu_sim(sys, cfg, fp64=False, use_graph=False)
    sb = gpu_sim(sys, cfg, fp64=False, use_graph=True)
    for sim in (sa, sb):
        sim.step(35)
        sim.sync()
    assert np.array_equal(sa.pos.cpu().numpy(), sb.pos.cpu().numpy())
    assert np.array_equal(sa.vel.cpu().numpy(), sb.vel.cpu().numpy())


def test_deterministic_and_resumable(box):
    a = gpu_sim(box, BOX)
    a.step(40)
    a.sync()
    b = gpu_sim(box, BOX)
    b.step(20)
    b.sync()
    b.step(20)
    b.sync()
    assert np.array_equal(a.pos.cpu().numpy(), b.pos.cpu().numpy())
    assert np.array_equal(a.vel.cpu().numpy(), b.vel.cpu().numpy())


def test_replicas_match_independent_oracle_runs(orc):
    systems = [relaxed_droplet(name) for name in ("r0", "r1", "r2")]
    sim = gpu_sim(systems, DROPLET, fp64=True, log_events=True, event_capacity=2_000_000)
    sim.step(30)
    sim.sync()
    pos = sim.pos.cpu().numpy()
    for r, s in enumerate(systems):
        o = orc.run(oracle_params(orc, s, DROPLET, replica=r), orc.Topology.from_system(s),
                    s.pos, s.vel, 0, 30)
        assert o["status"] == 0
        b, e = sim.offsets[r], sim.offsets[r + 1]
        assert np.abs(pos[b:e] - o["q"]).max() <= 1e-6
        assert sim.counters(r)["proposals"] == o["counters"]["proposals"]


def test_device_conditions_are_reported(droplet):
    import paper_2002_07109_amd as B
    sim = gpu_sim(droplet, dict(DROPLET, skin=0.02, rebuild_interval=1000, dt=1.0))
    sim.step(60)
    with pytest.raises(B.BounceError) as e:
        sim.sync()
    assert e.value.status == -4


def test_autotuner_picks_a_lane_count_and_keeps_results(orc, box):
    import paper_2002_07109_amd as B
    sim = gpu_sim(box, BOX, fp64=True)
    g0 = sim.gradient(B.G_SHORT).cpu().numpy()
    lanes, times = sim.autotune(reps=3)
    assert lanes in (4, 8, 16, 32) and all(t > 0 for t in times.values())
    g1 = sim.gradient(B.G_SHORT).cpu().numpy()
    assert rel_err(g1, g0) < 1e-13
    sim.step(20)
    sim.sync()


def test_replicas_graph_replay_equals_direct_launches():
    systems = [relaxed_droplet(name) for name in ("r0", "r1", "r2")]
    sa = gpu_sim(systems, DROPLET, fp64=False, use_graph=False)
    sb = gpu_sim(systems, DROPLET, fp64=False, use_graph=True)
    for sim in (sa, sb):
        sim.step(25)
        sim.sync()
    assert np.array_equal(sa.pos.cpu().numpy(), sb.pos.cpu().numpy())
    assert np.array_equal(sa.vel.cpu().numpy(), sb.vel.cpu().numpy())
    for r in range(3):
        assert sa.counters(r)["proposals"] == sb.counters(r)["proposals"]


def test_profiling_kinds_keep_or_advance_the_trajectory(box):
    """Kinds 0 and 2 of bounce_profile_kernel leave the trajectory as it was,
    kind 1 keeps positions and velocities; kind 3 advances the trajectory by
    reps + 1 steps exactly as bounce_step would."""
    a = gpu_sim(box, BOX, fp64=True)
    b = gpu_sim(box, BOX, fp64=True)
    c = gpu_sim(box, BOX, fp64=True)
    for sim in (a, b, c):
        sim.step(5)
        sim.sync()
    pos0, vel0 = a.pos.cpu().numpy().copy(), a.vel.cpu().numpy().copy()
    assert c.profile_kernel(1, 2) > 0.0
    assert np.array_equal(c.pos.cpu().numpy(), pos0)
    assert np.array_equal(c.vel.cpu().numpy(), vel0)
    for kind in (0, 2):
        assert a.profile_kernel(kind, 3) > 0.0
    assert np.array_equal(a.pos.cpu().numpy(), pos0)
    assert np.array_equal(a.vel.cpu().numpy(), vel0)
    assert a.profile_kernel(3, 4) > 0.0
    b.step(5)
    b.sync()
    assert a.get_step() == b.get_step() == 10
    assert np.array_equal(a.pos.cpu().numpy(), b.pos.cpu().numpy())
    assert np.array_equal(a.vel.cpu().numpy(), b.vel.cpu().numpy())

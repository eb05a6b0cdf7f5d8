"""GPU parity of the reciprocal-space Ewald sum by smooth PME and of the RESPA
outer step (Sec. V) against the oracle's plain-DFT mesh sum: energy parts,
gradients, energies, trajectories with the mesh force in F_0 (respa_m = 0) or
as outer half kicks every m steps, and graph replay."""
import numpy as np
import pytest

from helpers import (BOX, DROPLET, event_keys, gpu_sim, oracle_params, rel_err, relaxed_box,
                     relaxed_droplet)
from workloads import jitter_positions

pytestmark = pytest.mark.gpu

MESH = dict(BOX, pme_grid=(32, 32, 32), pme_order=5)


@pytest.fixture(scope="module")
def box():
    return relaxed_box("b8")


@pytest.mark.parametrize("order,grid", [(4, (32, 32, 32)), (5, (32, 32, 32)), (6, (32, 32, 32)),
                                        (5, (16, 32, 64)), (4, (8, 8, 8)), (6, (8, 16, 8))])
def test_mesh_energy_and_gradient(orc, box, order, grid):
    import paper_2002_07109_amd as B
    cfg = dict(MESH, pme_order=order, pme_grid=grid)
    sim = gpu_sim(box, cfg, fp64=True)
    q = jitter_positions(box.pos, 0.05, seed=11)
    sim.set_state(pos=q)
    p = oracle_params(orc, box, cfg)
    topo = orc.Topology.from_system(box)
    (er, es, ex), go = orc.pme(p, topo, q)
    e = sim.pme_energy()
    assert e[0] == pytest.approx(er, rel=1e-10)
    assert e[1] == pytest.approx(es, rel=1e-13)
    assert e[2] == pytest.approx(ex, rel=1e-12)
    g = sim.gradient(B.G_RECIP).cpu().numpy()
    assert rel_err(g, go) < 1e-10
    # combined with the real-space part, summed into one output
    g2 = sim.gradient(B.G_FULL | B.G_RECIP).cpu().numpy()
    o2 = orc.gradient(p, topo, q, orc.G_FULL | orc.G_RECIP)
    assert rel_err(g2, o2) < 1e-10


def test_energies_include_mesh_terms(orc, box):
    sim = gpu_sim(box, MESH, fp64=True)
    e = sim.energies()[0]
    o = orc.energies(oracle_params(orc, box, MESH), orc.Topology.from_system(box), box.pos, box.vel)
    for k in ("bond", "angle", "coul", "lj", "pair", "kin"):
        assert e[k] == pytest.approx(o[k], rel=1e-10, abs=1e-8), k
    plain = gpu_sim(box, BOX, fp64=True).energies()[0]
    assert e["coul"] - plain["coul"] == pytest.approx(sum(sim.pme_energy()), rel=1e-12)


@pytest.mark.parametrize("integrator", [0, 1])
@pytest.mark.parametrize("respa_m", [0, 2, 5])
def test_trajectory_with_mesh(orc, box, respa_m, integrator):
    cfg = dict(MESH, respa_m=respa_m, integrator=integrator)
    nsteps = 60
    sim = gpu_sim(box, cfg, fp64=True, log_events=True, event_capacity=4_000_000)
    sim.step(nsteps)
    sim.sync()
    o = orc.run(oracle_params(orc, box, cfg), orc.Topology.from_system(box), box.pos, box.vel, 0,
                nsteps, ev_cap=4_000_000)
    assert o["status"] == 0, o["status_name"]
    dq = np.abs(sim.pos.cpu().numpy() - o["q"]).max()
    dv = np.abs(sim.vel.cpu().numpy() - o["v"]).max()
    assert dq <= 1e-6 and dv <= 1e-6, (dq, dv)
    if integrator == 0:
        ev, n = sim.events()
        assert n == o["n_events"] and n > 0
        assert np.array_equal(event_keys(ev), event_keys(o["events"]))


def test_outer_kick_matters(orc, box):
    """The mesh force moves the trajectory: without it (or with the outer
    kicks at the wrong steps) the run leaves the oracle's."""
    cfg = dict(MESH, respa_m=2)
    a = gpu_sim(box, cfg, fp64=True)
    b = gpu_sim(box, dict(cfg, respa_m=5), fp64=True)
    c = gpu_sim(box, BOX, fp64=True)
    for s in (a, b, c):
        s.step(20)
        s.sync()
    qa, qb, qc = (s.pos.cpu().numpy() for s in (a, b, c))
    assert np.abs(qa - qb).max() > 1e-5 and np.abs(qa - qc).max() > 1e-5


@pytest.mark.parametrize("respa_m", [0, 2])
def test_graph_replay_and_resume_are_bit_exact(box, respa_m):
    cfg = dict(MESH, respa_m=respa_m)
    sa = gpu_sim(box, cfg, fp64=False, use_graph=False)
    sb = gpu_sim(box, cfg, fp64=False, use_graph=True)
    for sim in (sa, sb):
        sim.step(35)
        sim.sync()
    assert np.array_equal(sa.pos.cpu().numpy(), sb.pos.cpu().numpy())
    assert np.array_equal(sa.vel.cpu().numpy(), sb.vel.cpu().numpy())
    # stopping and restarting at any step gives the same bits
    sc = gpu_sim(box, cfg, fp64=False, use_graph=True)
    for k in (3, 7, 25):
        sc.step(k)
    sc.sync()
    assert np.array_equal(sc.pos.cpu().numpy(), sb.pos.cpu().numpy())


def test_mesh_needs_one_periodic_replica(box):
    import paper_2002_07109_amd as B
    with pytest.raises(B.BounceError):
        gpu_sim([box, box], MESH)


@pytest.mark.parametrize("case", ["box_mesh_m2", "box_mesh_m5", "box_m2", "drop_m2", "box_baoab_m5",
                                  "box_mesh_m2_pairbounds"])
def test_trajectory_with_outer_nonbonded(orc, box, case):
    """BOUNCE-RESPA with the short-range pair force (and the mesh force) on the
    outer step (Sec. V): FP64 trajectory and jump events against the oracle."""
    if case.startswith("drop"):
        sys, cfg = relaxed_droplet("c0"), dict(DROPLET)
    else:
        sys, cfg = box, dict(MESH if "mesh" in case else BOX)
    cfg.update(respa_outer=1, respa_m=5 if case.endswith("m5") else 2)
    if "baoab" in case:
        cfg["integrator"] = 1
    if "pairbounds" in case:
        cfg["rate_mode"] = 1
    nsteps = 60
    sim = gpu_sim(sys, cfg, fp64=True, log_events=True, event_capacity=4_000_000)
    sim.step(nsteps)
    sim.sync()
    o = orc.run(oracle_params(orc, sys, cfg), orc.Topology.from_system(sys), sys.pos, sys.vel, 0,
                nsteps, ev_cap=4_000_000)
    assert o["status"] == 0, o["status_name"]
    dq = np.abs(sim.pos.cpu().numpy() - o["q"]).max()
    dv = np.abs(sim.vel.cpu().numpy() - o["v"]).max()
    assert dq <= 1e-6 and dv <= 1e-6, (dq, dv)
    if cfg["integrator"] == 0:
        ev, n = sim.events()
        assert n == o["n_events"] and n > 0
        assert np.array_equal(event_keys(ev), event_keys(o["events"]))


def test_outer_nonbonded_graph_replay_is_bit_exact(box):
    cfg = dict(MESH, respa_m=2, respa_outer=1)
    sa = gpu_sim(box, cfg, fp64=False, use_graph=False)
    sb = gpu_sim(box, cfg, fp64=False, use_graph=True)
    for sim in (sa, sb):
        sim.step(35)
        sim.sync()
    assert np.array_equal(sa.pos.cpu().numpy(), sb.pos.cpu().numpy())
    assert np.array_equal(sa.vel.cpu().numpy(), sb.vel.cpu().numpy())


@pytest.mark.parametrize("respa_outer", [0, 1])
def test_mesh_timing_leaves_the_trajectory(box, respa_outer):
    """Timing the mesh sum (it writes the outer-gradient buffer) between steps,
    also in the middle of an outer step, changes nothing: every outer kick
    recomputes that buffer first."""
    cfg = dict(MESH, respa_m=5, respa_outer=respa_outer)
    a = gpu_sim(box, cfg, fp64=False, use_graph=True)
    b = gpu_sim(box, cfg, fp64=False, use_graph=True)
    a.step(23)
    for k in (7, 9, 7):
        b.step(k)
        b.profile_kernel(4, 3)
    for s in (a, b):
        s.sync()
    assert np.array_equal(a.pos.cpu().numpy(), b.pos.cpu().numpy())
    assert np.array_equal(a.vel.cpu().numpy(), b.vel.cpu().numpy())


def test_outer_nonbonded_replicas_match_independent_oracle_runs(orc):
    """Several droplets in one context with the short-range pair force on the
    outer step: each replica follows its own oracle run."""
    cfg = dict(DROPLET, respa_m=2, respa_outer=1)
    systems = [relaxed_droplet(name) for name in ("r0", "r1", "r2")]
    sim = gpu_sim(systems, cfg, fp64=True, use_graph=True)
    sim.step(30)
    sim.sync()
    pos = sim.pos.cpu().numpy()
    for r, s in enumerate(systems):
        o = orc.run(oracle_params(orc, s, cfg, replica=r), orc.Topology.from_system(s), s.pos, s.vel,
                    0, 30)
        assert o["status"] == 0, o["status_name"]
        b, e = sim.offsets[r], sim.offsets[r + 1]
        assert np.abs(pos[b:e] - o["q"]).max() <= 1e-6
        assert sim.counters(r)["proposals"] == o["counters"]["proposals"]

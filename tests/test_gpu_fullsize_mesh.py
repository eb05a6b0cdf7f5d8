"""GPU path at the mesh workload's full size (the 96,000-atom periodic water box,
32,000 waters in a 98 A cube, smooth PME on a 64^3 mesh with order-5 splines,
alpha = 0.35/A) against the oracle: the mesh energy terms and the whole
reciprocal-space gradient (the oracle's plain-DFT mesh sum takes about a second
here), a 16-step FP64 trajectory of the BOUNCE-RESPA scheme with the short-range
pair and mesh forces on the outer step (positions, velocities and every jump
event against the oracle), and a short run of the benchmark's configuration."""
import numpy as np
import pytest

from helpers import BOX, event_keys, gpu_sim, oracle_params
from workloads import jitter_positions, water_box

pytestmark = pytest.mark.gpu

C3 = dict(BOX, ewald_alpha=0.35, r_on=7.0, r_off=8.0, pme_grid=(64, 64, 64), pme_order=5)


@pytest.fixture(scope="module")
def c3():
    return water_box(n_side=32, box_len=98.0, seed=3, remove=768)


def test_c3_mesh_energy_and_gradient(orc, c3):
    import paper_2002_07109_amd as B
    assert c3.n_atoms == 96000
    sim = gpu_sim(c3, C3, fp64=False, use_graph=True)
    q = jitter_positions(c3.pos, 0.05, seed=12)
    sim.set_state(pos=q)
    p = oracle_params(orc, c3, C3)
    topo = orc.Topology.from_system(c3)
    (er, es, ex), go = orc.pme(p, topo, q)
    e = sim.pme_energy()
    assert e[0] == pytest.approx(er, rel=1e-10)
    assert e[1] == pytest.approx(es, rel=1e-13)
    assert e[2] == pytest.approx(ex, rel=1e-12)
    g = sim.gradient(B.G_RECIP).cpu().numpy()
    rms = np.sqrt(np.mean(np.sum(go * go, 1)))
    err = np.max(np.linalg.norm(g - go, axis=1)) / rms
    assert err < 1e-9, err


def test_c3_bench_configuration_runs(c3):
    """Relax the lattice start (BAOAB, strong friction), then run BOUNCE-RESPA
    with the short-range pair and mesh forces on a 2 fs outer step, as timed."""
    sim = gpu_sim(c3, dict(C3, integrator=1, gamma=0.05), fp64=False, use_graph=True)
    sim.step(300)
    sim.sync()
    pos, vel = sim.pos.cpu().numpy(), sim.vel.cpu().numpy()
    sim = gpu_sim(c3, dict(C3, respa_m=2, respa_outer=1), fp64=False, use_graph=True)
    sim.set_state(pos=pos, vel=vel, step=0)
    sim.step(100)
    sim.sync()
    c = sim.counters()
    e = sim.energies()[0]
    assert c["proposals"] > 0 and c["bound_violations"] == 0
    assert np.isfinite(e["coul"]) and 100.0 < e["tkin"] < 2000.0


def test_c3_trajectory_fp64_respa_with_mesh(orc, c3):
    """16 steps of 0.5 fs from the lattice start (at 1 fs the start's hot spots
    move an atom half the skin within 20 steps, in both implementations), outer
    step m = 2 with the short-range pair force and the mesh force, FP64."""
    cfg = dict(C3, integrator=0, dt=0.5, respa_m=2, respa_outer=1)
    nsteps = 16
    sim = gpu_sim(c3, cfg, fp64=True, log_events=True, event_capacity=1_000_000, use_graph=True)
    sim.step(nsteps)
    sim.sync()
    o = orc.run(oracle_params(orc, c3, cfg), orc.Topology.from_system(c3), c3.pos, c3.vel, 0, nsteps,
                ev_cap=1_000_000)
    assert o["status"] == 0, o["status_name"]
    dq = np.abs(sim.pos.cpu().numpy() - o["q"]).max()
    dv = np.abs(sim.vel.cpu().numpy() - o["v"]).max()
    ev, n = sim.events()
    print(f"96k mesh box, {nsteps} FP64 RESPA steps: max |dq| {dq:.3e} A, max |dv| {dv:.3e} A/fs, "
          f"{n} events (oracle {o['n_events']})")
    assert dq <= 1e-6 and dv <= 1e-6
    assert n == o["n_events"] and n > 0
    assert np.array_equal(event_keys(ev), event_keys(o["events"]))
    c = sim.counters()
    assert c["proposals"] == o["counters"]["proposals"] and c["accepted"] == o["counters"]["accepted"]

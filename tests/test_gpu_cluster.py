"""The cluster-pair (tile) form of the F_0 pair force (pair_kernel = 4 or 8):
clusters of consecutive sorted atoms, a bounding-box cluster list per list
build, one pair per lane.  It must give the integrator's pair force within the
FP32 tolerance of the oracle (each part against its own RMS, 1e-5), agree with
the atom-row kernel within that same tolerance (the two round differently: the
rows form r^2 in mirror units when the unit is the same on all axes, the tiles
in A; each lands within ~3.5e-6 of the oracle), and carry FP32 trajectories
whose event logs follow the FP64 oracle up to a near-tie, as the row kernel's do."""
import numpy as np
import pytest

from helpers import BOX, DROPLET, gpu_sim, oracle_params, rel_err, relaxed_box, relaxed_box24k, relaxed_droplet
from test_gpu_parity import assert_fp32_events_follow_oracle
from workloads import jitter_positions

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def droplet():
    return relaxed_droplet("c0")


@pytest.fixture(scope="module")
def box():
    return relaxed_box("b8")


def _sys(droplet, box, which):
    return (droplet, DROPLET) if which == "drop" else (box, BOX)


@pytest.mark.parametrize("cl", [4, 8])
@pytest.mark.parametrize("integrator", [0, 1], ids=["bounce", "baoab"])
@pytest.mark.parametrize("which", ["drop", "box"])
def test_cluster_step_pair_force(orc, droplet, box, which, integrator, cl):
    import paper_2002_07109_amd as B
    sys, cfg = _sys(droplet, box, which)
    cfg = dict(cfg, integrator=integrator, pair_kernel=cl)
    p = oracle_params(orc, sys, cfg)
    topo = orc.Topology.from_system(sys)
    obit = orc.G_SHORT if integrator == 0 else orc.G_FULL
    sim = gpu_sim(sys, cfg)
    q = jitter_positions(sys.pos, 0.05, seed=11)
    sim.set_state(pos=q)
    g = sim.gradient(B.G_STEP).cpu().numpy()
    err = rel_err(g, orc.gradient(p, topo, q, obit))
    print(f"{which} cl={cl} integrator={integrator}: cluster pair force {err:.3e}")
    assert err < 1e-5, err
    # after 7 steps: the cluster lists of the step-0 build, positions moved
    sim = gpu_sim(sys, cfg)
    sim.step(7)
    sim.sync()
    g7 = sim.gradient(B.G_STEP).cpu().numpy()
    o7 = orc.run(p, topo, sys.pos, sys.vel, 0, 7)
    assert o7["status"] == 0
    err7 = rel_err(g7, orc.gradient(p, topo, o7["q"], obit))
    print(f"  after 7 steps: {err7:.3e}")
    assert err7 < 1e-5, err7


def test_cluster_step_pair_force_with_separate_mechanisms(orc, box):
    """The tiles with separate Coulomb and Lennard-Jones windows in F_0."""
    import paper_2002_07109_amd as B
    cfg = dict(BOX, jump_split=1, r_on_lj=5.0, r_off_lj=6.0, pair_kernel=4)
    p = oracle_params(orc, box, cfg)
    q = jitter_positions(box.pos, 0.05, seed=13)
    sim = gpu_sim(box, cfg)
    sim.set_state(pos=q)
    g = sim.gradient(B.G_STEP).cpu().numpy()
    err = rel_err(g, orc.gradient(p, orc.Topology.from_system(box), q, orc.G_SHORT))
    print(f"split mechanisms, cluster tiles: {err:.3e}")
    assert err < 1e-5, err


def test_cluster_tiles_on_uneven_replicas():
    """Eight droplets of uneven size in one context: each replica's clusters
    and cluster lists stay within the replica; the tiles agree with the rows."""
    import paper_2002_07109_amd as B
    from workloads import droplet_batch
    systems = droplet_batch(64)[:8]
    g = {}
    for k in (0, 4):
        sim = gpu_sim(systems, dict(DROPLET, pair_kernel=k))
        g[k] = sim.gradient(B.G_STEP).cpu().numpy()
        sim.close()
    err = rel_err(g[4], g[0])
    print(f"8 droplets: cluster vs row kernel {err:.3e}")
    assert err < 1e-5, err


@pytest.mark.parametrize("cl", [4, 8])
def test_cluster_and_row_kernels_agree_at_full_size(cl):
    """The 24,000-atom box: the same pairs, summed in another order."""
    import paper_2002_07109_amd as B
    c1 = relaxed_box24k()
    g = {}
    for k in (0, cl):
        sim = gpu_sim(c1, dict(BOX, pair_kernel=k))
        g[k] = sim.gradient(B.G_STEP).cpu().numpy()
        sim.close()
    err = rel_err(g[cl], g[0])
    print(f"cl={cl}: cluster vs row kernel {err:.3e}")
    assert err < 1e-5, err


@pytest.mark.parametrize("which", ["drop", "box"])
def test_cluster_trajectory_fp32_events(orc, droplet, box, which):
    sys, cfg = _sys(droplet, box, which)
    cfg = dict(cfg, pair_kernel=8)
    nsteps = 40
    sim = gpu_sim(sys, cfg, log_events=True, event_capacity=4_000_000, use_graph=True)
    sim.step(nsteps)
    sim.sync()
    o = orc.run(oracle_params(orc, sys, cfg), orc.Topology.from_system(sys), sys.pos, sys.vel, 0, nsteps,
                ev_cap=4_000_000)
    assert o["status"] == 0
    ev, n = sim.events()
    same, div = assert_fp32_events_follow_oracle(ev, o["events"])
    dq = np.abs(sim.pos.cpu().numpy() - o["q"]).max()
    print(f"{which}: {nsteps} steps, max |dq| = {dq:.3e} A, identical leading events {same} of "
          f"{o['n_events']}, first divergence {div}")
    if div is None:
        assert dq < 1e-4

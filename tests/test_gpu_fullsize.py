"""GPU path at the benchmark's full size (the 24,000-atom periodic water box,
FP32 pair arithmetic, graph replay) against the oracle: sampled per-atom
gradients, candidate-list rows and one J half-step of sampled atoms; a whole
100-step FP64 trajectory with its event log; the FP32 benchmark configuration's
event log over 10 steps; and the differentiable direct energy (autograd) on 10
jittered geometries against the oracle and against finite differences of the
GPU energy."""
import numpy as np
import pytest

from helpers import BOX, FF, event_keys, first_divergence, gpu_sim, oracle_params, relaxed_box24k
from workloads import jitter_positions, water_box

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    return water_box(n_side=20, box_len=62.0, seed=0)


@pytest.fixture(scope="module")
def sample(c1):
    rng = np.random.default_rng(42)
    return np.sort(rng.choice(c1.n_atoms, 96, replace=False))


@pytest.mark.parametrize("fp64", [False, True])
def test_c1_gradients_sampled(orc, c1, sample, fp64):
    import paper_2002_07109_amd as B
    sim = gpu_sim(c1, BOX, fp64=fp64, use_graph=True)
    p = oracle_params(orc, c1, BOX)
    topo = orc.Topology.from_system(c1)
    tol = 1e-11 if fp64 else 1e-5
    # each part's error against that part's own RMS over the sample
    for gbit, obit in [(B.G_SHORT | B.G_BONDED, orc.G_SHORT | orc.G_BONDED),
                       (B.G_LONG, orc.G_LONG), (B.G_FULL, orc.G_FULL)]:
        g = sim.gradient(gbit).cpu().numpy()[sample]
        o = np.stack([orc.gradient_atom(p, topo, c1.pos, obit, int(i)) for i in sample])
        rms = np.sqrt(np.mean(np.sum(o * o, 1)))
        err = np.max(np.linalg.norm(g - o, axis=1)) / rms
        print(f"fp64={fp64} part {gbit}: max|dF|/RMS|F| = {err:.3e}")
        assert err < tol, (gbit, err)


@pytest.mark.parametrize("integrator", [0, 1])
@pytest.mark.parametrize("fp64", [False, True])
def test_c1_step_pair_force_sampled(orc, sample, fp64, integrator):
    """The integrator's own pair part of F_0 (the fixed-point mirror in FP32) at full
    size after 5 steps from the relaxed box, on the sampled atoms, against the
    oracle at its own positions after the same 5 steps: BOUNCE's short-range
    force and BAOAB's full one."""
    import paper_2002_07109_amd as B
    c1 = relaxed_box24k()
    cfg = dict(BOX, integrator=integrator)
    sim = gpu_sim(c1, cfg, fp64=fp64, use_graph=True)
    sim.step(5)
    sim.sync()
    g = sim.gradient(B.G_STEP).cpu().numpy()[sample]
    p = oracle_params(orc, c1, cfg)
    topo = orc.Topology.from_system(c1)
    o5 = orc.run(p, topo, c1.pos, c1.vel, 0, 5)
    assert o5["status"] == 0
    obit = orc.G_SHORT if integrator == 0 else orc.G_FULL
    o = np.stack([orc.gradient_atom(p, topo, o5["q"], obit, int(i)) for i in sample])
    rms = np.sqrt(np.mean(np.sum(o * o, 1)))
    err = np.max(np.linalg.norm(g - o, axis=1)) / rms
    print(f"24k step pair force fp64={fp64}: {err:.3e}")
    assert err < (1e-10 if fp64 else 1e-5), err


def test_c1_candidate_rows_bit_exact(orc, c1, sample):
    import paper_2002_07109_amd as B
    sim = gpu_sim(c1, BOX, fp64=False)
    sim.jump_halfstep(0, B.PH_JA)
    rp, col = sim.get_list(B.LIST_CAND)
    frp, fcol = sim.get_list(B.LIST_FORCE)
    p = oracle_params(orc, c1, BOX)
    topo = orc.Topology.from_system(c1)
    order, _ = orc.sort_order(p, c1.pos)
    for i in sample:
        o = orc.list_row(p, topo, c1.pos, BOX["r_on"] - BOX["skin"], BOX["r_cut"] + BOX["skin"],
                         order, int(i))
        assert np.array_equal(col[rp[i]:rp[i + 1]], o)
        of = orc.list_row(p, topo, c1.pos, 0.0, BOX["r_off"] + BOX["skin"], order, int(i))
        assert np.array_equal(fcol[frp[i]:frp[i + 1]], of)


def test_c1_jump_events_sampled_fp64(orc, c1, sample):
    import paper_2002_07109_amd as B
    cfg = dict(BOX, r_on=4.0, r_off=5.0)
    sim = gpu_sim(c1, cfg, fp64=True, log_events=True, event_capacity=2_000_000)
    sim.jump_halfstep(3, B.PH_JB)
    ev, n = sim.events()
    p = oracle_params(orc, c1, cfg)
    topo = orc.Topology.from_system(c1)
    order, _ = orc.sort_order(p, c1.pos)
    rp = np.zeros(c1.n_atoms + 1, np.int64)
    rows = {}
    for i in sample:
        rows[int(i)] = orc.list_row(p, topo, c1.pos, cfg["r_on"] - cfg["skin"],
                                    cfg["r_cut"] + cfg["skin"], order, int(i))
    counts = np.zeros(c1.n_atoms, np.int64)
    for i, r in rows.items():
        counts[i] = r.size
    rp[1:] = np.cumsum(counts)
    col = np.concatenate([rows[int(i)] for i in sample]).astype(np.int32)
    out = orc.jump_halfstep(p, topo, c1.pos, c1.vel, rp, col, 3, B.PH_JB, ev_cap=1_000_000)
    mine = ev[np.isin(ev["atom"], sample)]
    assert out["events"].size > 50
    assert np.array_equal(event_keys(mine), event_keys(out["events"]))
    np.testing.assert_allclose(sim.vel.cpu().numpy()[sample], out["v"][sample], rtol=0, atol=1e-14)


def test_c1_bench_configuration_runs(c1):
    # relax the hot lattice start on the GPU first (strong friction), then run
    # the benchmark's configuration
    sim = gpu_sim(c1, dict(BOX, integrator=1, gamma=0.05), fp64=False, use_graph=True)
    sim.step(300)
    sim.sync()
    pos, vel = sim.pos.cpu().numpy(), sim.vel.cpu().numpy()
    sim = gpu_sim(c1, BOX, fp64=False, use_graph=True)
    sim.set_state(pos=pos, vel=vel, step=0)
    sim.step(200)
    sim.sync()
    c = sim.counters()
    e = sim.energies()[0]
    assert c["proposals"] > 0 and c["bound_violations"] == 0
    assert np.isfinite(e["pair"]) and 100.0 < e["tkin"] < 2000.0


@pytest.mark.timeout(900)
def test_c1_trajectory_fp64_100_steps(orc):
    """The whole 24,000-atom box (from its oracle-relaxed state), 100 steps of
    B J A O A J B with FP64 pair arithmetic and the K = 10 step graph (ten list
    rebuilds, each interval running past the far-part gate), against the
    oracle: positions and velocities within 1e-6, the event logs and the
    counters identical."""
    c1 = relaxed_box24k()
    sim = gpu_sim(c1, BOX, fp64=True, log_events=True, event_capacity=2_000_000, use_graph=True)
    sim.step(100)
    sim.sync()
    p = oracle_params(orc, c1, BOX)
    o = orc.run(p, orc.Topology.from_system(c1), c1.pos, c1.vel, 0, 100, ev_cap=2_000_000)
    assert o["status"] == 0, o["status_name"]
    dq = np.abs(sim.pos.cpu().numpy() - o["q"]).max()
    dv = np.abs(sim.vel.cpu().numpy() - o["v"]).max()
    moved = np.sqrt(((o["q"] - c1.pos) ** 2).sum(1)).max()
    ev, n = sim.events()
    print(f"24k box, 100 FP64 steps: max |dq| {dq:.3e} A, max |dv| {dv:.3e} A/fs, "
          f"{n} events, largest displacement {moved:.2f} A")
    assert dq <= 1e-6 and dv <= 1e-6, (dq, dv)
    assert n == o["n_events"] and n > 1000
    assert np.array_equal(event_keys(ev), event_keys(o["events"]))
    c = sim.counters()
    assert c["proposals"] == o["counters"]["proposals"]
    assert c["accepted"] == o["counters"]["accepted"]
    assert c["bound_violations"] == 0


@pytest.mark.timeout(600)
def test_c1_fp32_events_follow_oracle(orc, c1):
    """The benchmark's configuration (FP32 pair arithmetic, graph replay), 10
    steps: the event log equals the FP64 oracle's until the first half-step where
    they differ, and there every differing atom's first proposal is a near-tie of
    the oracle's accept test, |U |v| L - v.F| < 1e-5 |v| |F|."""
    sim = gpu_sim(c1, BOX, fp64=False, log_events=True, event_capacity=500_000, use_graph=True)
    sim.step(10)
    sim.sync()
    p = oracle_params(orc, c1, BOX)
    o = orc.run(p, orc.Topology.from_system(c1), c1.pos, c1.vel, 0, 10, ev_cap=500_000)
    assert o["status"] == 0
    ev, n = sim.events()
    assert o["n_events"] > 1000
    div = first_divergence(ev, o["events"])
    print(f"24k box, 10 FP32 steps: {n} events (oracle {o['n_events']}), first divergence {div}")
    if div is None:
        assert n == o["n_events"]
        return
    step, phase, atoms = div
    for atom, k, oe in atoms:
        assert oe is not None, (step, phase, atom, "proposal count differs")
        assert abs(oe["margin"]) < 1e-5 * oe["scale"], (step, phase, atom, k)


C4_SEEDS = list(range(10))
C4_PARAMS = np.concatenate([FF["charge"], FF["eps"], FF["sigma"]])


def _c4_check(orc, c1, q, tp, fp64, eps=None, sigma=None):
    import torch
    import paper_2002_07109_amd as B
    sim = gpu_sim(c1, BOX, fp64=fp64)
    pos = torch.tensor(q, dtype=torch.float64, device="cuda:0", requires_grad=True)
    par = torch.tensor(tp, dtype=torch.float64, device="cuda:0", requires_grad=True)
    E = B.DirectEnergy.apply(pos, par, sim)
    E.backward()
    p = orc.make_params(c1, integrator=BOX["integrator"], coulomb=BOX["coulomb"],
                        r_on=BOX["r_on"], r_off=BOX["r_off"], r_cut=BOX["r_cut"],
                        skin=BOX["skin"], ewald_alpha=BOX["ewald_alpha"], eps=eps, sigma=sigma)
    topo = orc.Topology.from_system(c1)
    oE, ogq, ogc, oge, ogs = orc.direct_energy(p, topo, q)
    tol = 1e-11 if fp64 else 1e-5
    assert float(E.detach()) == pytest.approx(oE, rel=tol)
    gq = pos.grad.cpu().numpy()
    rms = np.sqrt(np.mean(np.sum(ogq * ogq, 1)))
    err = np.max(np.linalg.norm(gq - ogq, axis=1)) / rms
    assert err < tol, err
    return par.grad.cpu().numpy(), (ogc, oge, ogs), tol


@pytest.mark.parametrize("seed", C4_SEEDS)
def test_c4_direct_energy_autograd(orc, c1, seed):
    """FP32 pair arithmetic on 10 jittered geometries (sigma = 0.05 A): energy,
    position gradient and the gradients w.r.t. Q_O, Q_H, eps_O and sigma_O
    against the FP64 oracle (eps_H = 0 leaves d/deps_H undefined under
    Lorentz-Berthelot mixing)."""
    q = jitter_positions(c1.pos, 0.05, seed=seed)
    gp, (ogc, oge, ogs), tol = _c4_check(orc, c1, q, C4_PARAMS, fp64=False)
    for k, ref in [(0, ogc[0]), (1, ogc[1]), (2, oge[0]), (4, ogs[0])]:
        assert gp[k] == pytest.approx(ref, rel=10 * tol), k


def test_c4_direct_energy_autograd_fp64(orc, c1):
    q = jitter_positions(c1.pos, 0.05, seed=1)
    gp, (ogc, oge, ogs), tol = _c4_check(orc, c1, q, C4_PARAMS, fp64=True)
    for k, ref in [(0, ogc[0]), (1, ogc[1]), (2, oge[0]), (4, ogs[0])]:
        assert gp[k] == pytest.approx(ref, rel=10 * tol), k


def test_c4_all_six_parameter_gradients_with_lj_on_h(orc, c1):
    """With Lennard-Jones on H as well (eps_H = 0.02 kcal/mol, sigma_H = 1.2 A)
    every per-type gradient is defined: all six against the FP64 oracle."""
    eps, sigma = np.array([0.152, 0.02]), np.array([3.15, 1.2])
    tp = np.concatenate([FF["charge"], eps, sigma])
    q = jitter_positions(c1.pos, 0.05, seed=4)
    for fp64 in (True, False):
        gp, (ogc, oge, ogs), tol = _c4_check(orc, c1, q, tp, fp64=fp64, eps=eps, sigma=sigma)
        ref = np.concatenate([ogc, oge, ogs])
        for k in range(6):
            assert gp[k] == pytest.approx(ref[k], rel=10 * tol, abs=tol * np.abs(ref).max()), k


@pytest.mark.parametrize("seed", C4_SEEDS)
def test_c4_backward_matches_finite_differences_of_gpu_energy(c1, seed):
    """Central differences (h = 1e-4) of the FP64 GPU energy against its
    hand-written backward: 4 parameters and 6 random coordinates per geometry."""
    import torch
    import paper_2002_07109_amd as B
    q = jitter_positions(c1.pos, 0.05, seed=seed)
    sim = gpu_sim(c1, BOX, fp64=True)
    tp = C4_PARAMS
    pos = torch.tensor(q, dtype=torch.float64, device="cuda:0", requires_grad=True)
    par = torch.tensor(tp, dtype=torch.float64, device="cuda:0", requires_grad=True)
    E = B.DirectEnergy.apply(pos, par, sim)
    E.backward()
    h = 1e-4

    def energy(qq, pp):
        with torch.no_grad():
            return float(B.DirectEnergy.apply(torch.tensor(qq, dtype=torch.float64, device="cuda:0"),
                                              torch.tensor(pp, dtype=torch.float64,
                                                           device="cuda:0"), sim))
    for k in (0, 1, 2, 4):
        pp, pm = tp.copy(), tp.copy()
        pp[k] += h
        pm[k] -= h
        fd = (energy(q, pp) - energy(q, pm)) / (2 * h)
        assert float(par.grad[k]) == pytest.approx(fd, rel=1e-6)
    rng = np.random.default_rng(100 + seed)
    for i in rng.choice(c1.n_atoms, 6, replace=False):
        for c in range(3):
            qp, qm = q.copy(), q.copy()
            qp[i, c] += h
            qm[i, c] -= h
            fd = (energy(qp, tp) - energy(qm, tp)) / (2 * h)
            assert float(pos.grad[i, c]) == pytest.approx(fd, rel=1e-5, abs=1e-5)

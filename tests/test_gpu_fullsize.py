"""GPU path at the benchmark's full size (the 24,000-atom periodic water box,
FP32 pair arithmetic, graph replay) against the oracle on sampled outputs the
oracle computes one by one: per-atom gradients, candidate-list rows, and one J
half-step of sampled atoms; plus the differentiable direct energy (autograd)
against the oracle and against finite differences of the GPU energy."""
import numpy as np
import pytest

from helpers import BOX, FF, event_keys, gpu_sim, oracle_params
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
    # errors of each part against the scale of the whole force on the sample
    total = np.stack([orc.gradient_atom(p, topo, c1.pos, orc.G_BONDED | orc.G_FULL, int(i))
                      for i in sample])
    rms = np.sqrt(np.mean(np.sum(total * total, 1)))
    for gbit, obit in [(B.G_SHORT | B.G_BONDED, orc.G_SHORT | orc.G_BONDED),
                       (B.G_LONG, orc.G_LONG), (B.G_FULL, orc.G_FULL)]:
        g = sim.gradient(gbit).cpu().numpy()[sample]
        o = np.stack([orc.gradient_atom(p, topo, c1.pos, obit, int(i)) for i in sample])
        err = np.max(np.linalg.norm(g - o, axis=1)) / rms
        assert err < tol, (gbit, err)


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


@pytest.mark.parametrize("fp64,seed", [(False, 0), (True, 1)])
def test_c4_direct_energy_autograd(orc, c1, seed, fp64):
    import torch
    import paper_2002_07109_amd as B
    q = jitter_positions(c1.pos, 0.05, seed=seed)
    sim = gpu_sim(c1, BOX, fp64=fp64)
    tp = np.concatenate([FF["charge"], FF["eps"], FF["sigma"]])
    pos = torch.tensor(q, dtype=torch.float64, device="cuda:0", requires_grad=True)
    par = torch.tensor(tp, dtype=torch.float64, device="cuda:0", requires_grad=True)
    E = B.DirectEnergy.apply(pos, par, sim)
    E.backward()
    p = oracle_params(orc, c1, BOX)
    topo = orc.Topology.from_system(c1)
    oE, ogq, ogc, oge, ogs = orc.direct_energy(p, topo, q)
    tol = 1e-11 if fp64 else 1e-5
    assert float(E) == pytest.approx(oE, rel=tol)
    gq = pos.grad.cpu().numpy()
    rms = np.sqrt(np.mean(np.sum(ogq * ogq, 1)))
    assert np.max(np.linalg.norm(gq - ogq, axis=1)) / rms < tol
    gp = par.grad.cpu().numpy()
    # checked parameters: charge_O, charge_H, eps_O, sigma_O (eps_H = 0: d/deps_H undefined)
    for k, ref in [(0, ogc[0]), (1, ogc[1]), (2, oge[0]), (4, ogs[0])]:
        assert gp[k] == pytest.approx(ref, rel=10 * tol), k


def test_c4_backward_matches_finite_differences_of_gpu_energy(c1):
    import torch
    import paper_2002_07109_amd as B
    q = jitter_positions(c1.pos, 0.05, seed=2)
    sim = gpu_sim(c1, BOX, fp64=True)
    tp = np.concatenate([FF["charge"], FF["eps"], FF["sigma"]])
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
    rng = np.random.default_rng(9)
    for i in rng.choice(c1.n_atoms, 6, replace=False):
        for c in range(3):
            qp, qm = q.copy(), q.copy()
            qp[i, c] += h
            qm[i, c] -= h
            fd = (energy(qp, tp) - energy(qm, tp)) / (2 * h)
            assert float(pos.grad[i, c]) == pytest.approx(fd, rel=1e-5, abs=1e-5)

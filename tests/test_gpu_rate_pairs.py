"""Per-type-pair rate bounds on the GPU (BOUNCE_RATE_PAIR) against the oracle:
integer bound weights, class-grouped candidate rows exported in canonical
order, jump events bit for bit in FP64, FP64 trajectories (one system and
uneven replicas), and the proposal saving at the same accepted-jump law."""
import numpy as np
import pytest

from helpers import BOX, DROPLET, event_keys, gpu_sim, oracle_params, relaxed_box, relaxed_droplet

pytestmark = pytest.mark.gpu

PDROP = dict(DROPLET, rate_mode=1)
PBOX = dict(BOX, rate_mode=1)


@pytest.fixture(scope="module")
def droplet():
    return relaxed_droplet("c0")


@pytest.fixture(scope="module")
def box():
    return relaxed_box("b8")


def _sys(droplet, box, which):
    return (droplet, PDROP) if which == "drop" else (box, PBOX)


@pytest.mark.parametrize("which", ["drop", "box"])
def test_rate_weights_match_oracle(orc, droplet, box, which):
    sys, cfg = _sys(droplet, box, which)
    sim = gpu_sim(sys, cfg)
    lq, unit = sim.rate_weights()
    olq, ounit = orc.rate_weights(oracle_params(orc, sys, cfg))
    assert np.array_equal(lq, olq)
    np.testing.assert_allclose(unit, ounit, rtol=1e-12)
    assert lq.min() < 2 ** 20 and np.all(lq.max(axis=1) == 2 ** 20)


@pytest.mark.parametrize("which", ["drop", "box"])
def test_candidate_rows_bit_exact(orc, droplet, box, which):
    import paper_2002_07109_amd as B
    sys, cfg = _sys(droplet, box, which)
    sim = gpu_sim(sys, cfg, fp64=True)
    sim.jump_halfstep(0, B.PH_JA)
    p = oracle_params(orc, sys, cfg)
    topo = orc.Topology.from_system(sys)
    order, _ = orc.sort_order(p, sys.pos)
    grp, gcol = sim.get_list(B.LIST_CAND)
    orp, ocol = orc.build_list(p, topo, sys.pos, cfg["r_on"] - cfg["skin"],
                               cfg["r_cut"] + cfg["skin"], order)
    assert np.array_equal(grp, orp)
    assert np.array_equal(gcol, ocol)


@pytest.mark.parametrize("which", ["drop", "box"])
def test_jump_events_bit_exact(orc, droplet, box, which):
    import paper_2002_07109_amd as B
    sys, cfg = _sys(droplet, box, which)
    cfg = dict(cfg, r_on=4.0, r_off=5.0)
    sim = gpu_sim(sys, cfg, fp64=True, log_events=True, event_capacity=4_000_000)
    p = oracle_params(orc, sys, cfg)
    topo = orc.Topology.from_system(sys)
    order, _ = orc.sort_order(p, sys.pos)
    rp, col = orc.build_list(p, topo, sys.pos, cfg["r_on"] - cfg["skin"],
                             cfg["r_cut"] + cfg["skin"], order)
    v = sys.vel.copy()
    all_o = []
    for step, phase in [(0, B.PH_JA), (0, B.PH_JB), (5, B.PH_JA)]:
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
    # both partner classes are proposed
    assert len(np.unique(sys.atom_type[o["partner"]])) == 2


@pytest.mark.parametrize("which,nsteps", [("drop", 120), ("box", 60)])
def test_trajectory_fp64(orc, droplet, box, which, nsteps):
    sys, cfg = _sys(droplet, box, which)
    sim = gpu_sim(sys, cfg, fp64=True, log_events=True, event_capacity=4_000_000)
    sim.step(nsteps)
    sim.sync()
    o = orc.run(oracle_params(orc, sys, cfg), orc.Topology.from_system(sys), sys.pos, sys.vel, 0,
                nsteps, ev_cap=4_000_000)
    assert o["status"] == 0, o["status_name"]
    assert np.abs(sim.pos.cpu().numpy() - o["q"]).max() <= 1e-6
    assert np.abs(sim.vel.cpu().numpy() - o["v"]).max() <= 1e-6
    ev, n = sim.events()
    assert n == o["n_events"]
    assert np.array_equal(event_keys(ev), event_keys(o["events"]))
    c = sim.counters()
    assert c["accepted"] == o["counters"]["accepted"] and c["bound_violations"] == 0


def test_replicas_match_independent_oracle_runs(orc):
    systems = [relaxed_droplet(name) for name in ("r0", "r1", "r2")]
    sim = gpu_sim(systems, PDROP, fp64=True, use_graph=True)
    sim.step(30)
    sim.sync()
    pos = sim.pos.cpu().numpy()
    for r, s in enumerate(systems):
        o = orc.run(oracle_params(orc, s, PDROP, replica=r), orc.Topology.from_system(s),
                    s.pos, s.vel, 0, 30)
        assert o["status"] == 0
        b, e = sim.offsets[r], sim.offsets[r + 1]
        assert np.abs(pos[b:e] - o["q"]).max() <= 1e-6
        assert sim.counters(r)["proposals"] == o["counters"]["proposals"]


def test_fewer_proposals_than_atom_bounds(droplet):
    """Same FP32 run in both modes: per-type-pair bounds propose fewer jumps."""
    res = {}
    for mode in (0, 1):
        sim = gpu_sim(droplet, dict(DROPLET, rate_mode=mode), use_graph=True)
        sim.step(60)
        sim.sync()
        c = sim.counters()
        assert c["bound_violations"] == 0
        res[mode] = c
    assert res[1]["proposals"] < 0.8 * res[0]["proposals"]
    print("proposals per 60 steps: atom bounds %d, pair bounds %d; accepted %d vs %d"
          % (res[0]["proposals"], res[1]["proposals"], res[0]["accepted"], res[1]["accepted"]))

"""Batched replicas at full size: 64 non-periodic water droplets of uneven size
(about 400 to 6,000 atoms, ~190,000 atoms in all), each with its own Philox key
(seed, replica), advanced together and replayed from a hipGraph, either with a
pair-force and an integrator launch per step or with one fused persistent launch
per step (workgroups take (replica, atom tile) items from a queue; a replica's
integrator items wait on a counter of its finished pair items).  Eight sampled
replicas (the smallest, the largest and six others) are checked against
independent oracle runs of the same replica in both launch modes; the two modes
must agree bit for bit, on the droplets and on a periodic box."""
import numpy as np
import pytest

from helpers import BOX, DROPLET, gpu_sim, oracle_params, relaxed_box
from workloads import droplet_batch

pytestmark = pytest.mark.gpu

NSTEPS = 20


@pytest.fixture(scope="module")
def batch():
    return droplet_batch(64)


def _picks(batch):
    sizes = np.array([s.n_atoms for s in batch])
    return sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 3, 11, 17, 29, 40, 55})


@pytest.fixture(scope="module")
def oracle_runs(orc, batch):
    out = {}
    for r in _picks(batch):
        s = batch[r]
        o = orc.run(oracle_params(orc, s, DROPLET, replica=r), orc.Topology.from_system(s),
                    s.pos, s.vel, 0, NSTEPS)
        assert o["status"] == 0, (r, o["status_name"])
        out[r] = o
    return out


@pytest.mark.parametrize("persistent", [0, 1])
def test_batch_fp64_replicas_match_independent_oracle_runs(batch, oracle_runs, persistent):
    assert len(oracle_runs) >= 8
    sim = gpu_sim(batch, dict(DROPLET, persistent=persistent), fp64=True, use_graph=True)
    sim.step(NSTEPS)
    sim.sync()
    pos, vel = sim.pos.cpu().numpy(), sim.vel.cpu().numpy()
    for r, o in oracle_runs.items():
        b, e = sim.offsets[r], sim.offsets[r + 1]
        assert np.abs(pos[b:e] - o["q"]).max() <= 1e-6, r
        assert np.abs(vel[b:e] - o["v"]).max() <= 1e-6, r
        c = sim.counters(r)
        assert c["proposals"] == o["counters"]["proposals"], r
        assert c["accepted"] == o["counters"]["accepted"], r


def _run(systems, cfg, fp64, steps):
    sim = gpu_sim(systems, cfg, fp64=fp64, use_graph=True)
    sim.step(steps)
    sim.sync()
    n = len(systems) if isinstance(systems, (list, tuple)) else 1
    out = (sim.pos.cpu().numpy(), sim.vel.cpu().numpy(),
           [sim.counters(r) for r in range(n)], sim.get_step())
    sim.close()
    return out


@pytest.mark.parametrize("integrator", [0, 1], ids=["bounce", "baoab"])
@pytest.mark.parametrize("fp64", [False, True], ids=["fp32", "fp64"])
def test_fused_launch_is_bit_identical_on_the_batch(batch, fp64, integrator):
    sub = batch[:16]
    cfg = dict(DROPLET, integrator=integrator)
    # 23 steps: two graphs of K = 10 and direct launches around them
    a = _run(sub, dict(cfg, persistent=0), fp64, 23)
    b = _run(sub, dict(cfg, persistent=1), fp64, 23)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2] == b[2] and a[3] == b[3]
    if integrator == 0:
        assert sum(c["proposals"] for c in a[2]) > 0


@pytest.mark.parametrize("integrator", [0, 1], ids=["bounce", "baoab"])
@pytest.mark.parametrize("fp64", [False, True], ids=["fp32", "fp64"])
def test_fused_launch_is_bit_identical_on_one_box(fp64, integrator):
    box = relaxed_box("b8")
    cfg = dict(BOX, integrator=integrator)
    a = _run(box, dict(cfg, persistent=0), fp64, 25)
    b = _run(box, dict(cfg, persistent=1), fp64, 25)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2] == b[2] and a[3] == b[3]


@pytest.mark.parametrize("variant", ["pair_bounds", "split"])
def test_fused_launch_is_bit_identical_with_proposal_classes(batch, variant):
    """The fused launch's integrator with several proposal classes: per-type-pair
    bounds (two classes) on the droplets, separate Coulomb and Lennard-Jones
    mechanisms (four classes) on the box."""
    if variant == "pair_bounds":
        systems, cfg = batch[:8], dict(DROPLET, rate_mode=1)
    else:
        systems, cfg = relaxed_box("b8"), dict(BOX, jump_split=1, r_on_lj=5.0, r_off_lj=6.0)
    for fp64 in (False, True):
        a = _run(systems, dict(cfg, persistent=0), fp64, 23)
        b = _run(systems, dict(cfg, persistent=1), fp64, 23)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), fp64
        assert a[2] == b[2] and a[3] == b[3]
        assert sum(c["proposals"] for c in a[2]) > 0


def test_tuner_times_then_reads_its_cache(batch, tmp_path):
    cache = tmp_path / "tuning.jsonl"
    sim = gpu_sim(batch, DROPLET, fp64=False, use_graph=True)
    sim.step(10)
    sim.sync()
    t = sim.tune(reps=3, cache=cache)
    assert not t["from_cache"]
    assert t["pair_lanes"] in (4, 8, 16, 32) and t["persistent"] in (0, 1)
    assert all(v > 0 for v in t["pair_ms"].values())
    assert t["step_ms"]["two_launches"] > 0 and t["step_ms"]["fused"] > 0
    assert len(cache.read_text().splitlines()) == 1
    sim.step(100)
    sim.sync()
    total = 0
    for r in range(len(batch)):
        c = sim.counters(r)
        assert c["bound_violations"] == 0
        total += c["proposals"]
    assert total > 0
    for e in sim.energies():
        assert np.isfinite(e["pair"]) and 100.0 < e["tkin"] < 1000.0
    sim.close()
    # the same device and configuration: the choice comes from the file
    sim2 = gpu_sim(batch, DROPLET, fp64=False, use_graph=True)
    t2 = sim2.tune(reps=3, cache=cache)
    assert t2["from_cache"]
    assert (t2["pair_lanes"], t2["persistent"]) == (t["pair_lanes"], t["persistent"])
    assert len(cache.read_text().splitlines()) == 1
    sim2.close()


def test_batch_fp32_graph_autotuned_run(batch):
    sim = gpu_sim(batch, DROPLET, fp64=False, use_graph=True)
    sim.step(10)
    sim.sync()
    lanes, times = sim.autotune(reps=3)
    assert lanes in (4, 8, 16, 32)
    sim.step(100)
    sim.sync()
    for e in sim.energies():
        assert np.isfinite(e["pair"]) and 100.0 < e["tkin"] < 1000.0

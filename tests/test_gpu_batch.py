"""Batched replicas at full size: 64 non-periodic water droplets of uneven size
(about 400 to 6,000 atoms, ~190,000 atoms in all), each with its own Philox key
(seed, replica), advanced together by one set of launches per step (every
kernel spans all replicas) and replayed from a hipGraph.  Sampled replicas
(the smallest, the largest and two others) are checked against independent
oracle runs of the same replica."""
import numpy as np
import pytest

from helpers import DROPLET, gpu_sim, oracle_params
from workloads import droplet_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    return droplet_batch(64)


def _picks(batch):
    sizes = np.array([s.n_atoms for s in batch])
    return sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 40})


def test_batch_fp64_replicas_match_independent_oracle_runs(orc, batch):
    nsteps = 20
    sim = gpu_sim(batch, DROPLET, fp64=True, use_graph=True)
    sim.step(nsteps)
    sim.sync()
    pos, vel = sim.pos.cpu().numpy(), sim.vel.cpu().numpy()
    for r in _picks(batch):
        s = batch[r]
        o = orc.run(oracle_params(orc, s, DROPLET, replica=r), orc.Topology.from_system(s),
                    s.pos, s.vel, 0, nsteps)
        assert o["status"] == 0, (r, o["status_name"])
        b, e = sim.offsets[r], sim.offsets[r + 1]
        assert np.abs(pos[b:e] - o["q"]).max() <= 1e-6, r
        assert np.abs(vel[b:e] - o["v"]).max() <= 1e-6, r
        c = sim.counters(r)
        assert c["proposals"] == o["counters"]["proposals"], r
        assert c["accepted"] == o["counters"]["accepted"], r


def test_batch_fp32_graph_autotuned_run(batch):
    sim = gpu_sim(batch, DROPLET, fp64=False, use_graph=True)
    sim.step(10)
    sim.sync()
    lanes, times = sim.autotune(reps=3)
    assert lanes in (4, 8, 16, 32)
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

"""Degenerate and ragged inputs through the whole step, FP64, against the oracle:
replicas of one, two and seven waters beside a 216-water droplet in one context
(ragged tiles, replicas with empty lists), in both launch structures and with
cluster tiles; two waters too far apart to interact (every list empty: the step
is the bonded BAOAB part only); an atom at rest (its Poisson mean is zero)."""
import dataclasses

import numpy as np
import pytest

from helpers import DROPLET, gpu_sim, oracle_params, relaxed_droplet
from workloads import water_droplet
from workloads.water import droplet_grid

pytestmark = pytest.mark.gpu

NSTEPS = 20


def _ragged():
    return [water_droplet(n_waters=1, seed=1), water_droplet(n_waters=2, seed=2),
            water_droplet(n_waters=7, seed=3), relaxed_droplet("c0")]


def _oracle(orc, s, cfg, replica=0, nsteps=NSTEPS):
    o = orc.run(oracle_params(orc, s, cfg, replica=replica), orc.Topology.from_system(s), s.pos, s.vel,
                0, nsteps)
    assert o["status"] == 0, o["status_name"]
    return o


@pytest.mark.parametrize("variant", ["two_launches", "fused", "tiles"])
def test_tiny_and_ragged_replicas_match_the_oracle(orc, variant):
    systems = _ragged()
    cfg = dict(DROPLET, persistent=1 if variant == "fused" else 0)
    fp64 = variant != "tiles"                  # cluster tiles are an FP32 path
    if variant == "tiles":
        cfg["pair_kernel"] = 4
    sim = gpu_sim(systems, cfg, fp64=fp64, use_graph=True)
    sim.step(NSTEPS)
    sim.sync()
    pos, vel = sim.pos.cpu().numpy(), sim.vel.cpu().numpy()
    tol = 1e-6 if fp64 else 1e-3
    for r, s in enumerate(systems):
        o = _oracle(orc, s, cfg, replica=r)
        b, e = sim.offsets[r], sim.offsets[r + 1]
        dq = np.abs(pos[b:e] - o["q"]).max()
        assert dq <= tol, (r, dq)
        if fp64:
            assert np.abs(vel[b:e] - o["v"]).max() <= 1e-6, r
            c = sim.counters(r)
            assert c["proposals"] == o["counters"]["proposals"], r
            assert c["accepted"] == o["counters"]["accepted"], r
    # one water alone has no nonbonded partner: no proposals at all
    assert sim.counters(0)["proposals"] == 0


def test_waters_out_of_range_have_empty_lists(orc):
    import paper_2002_07109_amd as B
    s = water_droplet(n_waters=2, seed=4)
    pos = s.pos.copy()
    pos[3:] += np.array([25.0, 0.0, 0.0]) - (pos[3] - pos[0])     # 25 A apart
    origin, dims = droplet_grid(pos, s.cell_size)
    s = dataclasses.replace(s, pos=pos, grid_origin=origin, grid_dims=dims)
    sim = gpu_sim(s, DROPLET, fp64=True)
    g = sim.gradient(B.G_STEP).cpu().numpy()
    assert np.all(g == 0.0)
    sim.step(NSTEPS)
    sim.sync()
    o = _oracle(orc, s, DROPLET)
    assert np.abs(sim.pos.cpu().numpy() - o["q"]).max() <= 1e-9
    assert sim.counters()["proposals"] == 0 and o["counters"]["proposals"] == 0


def test_an_atom_at_rest(orc):
    s = relaxed_droplet("c0")
    vel = s.vel.copy()
    vel[0] = 0.0
    s = dataclasses.replace(s, vel=vel)
    sim = gpu_sim(s, DROPLET, fp64=True, use_graph=True)
    sim.step(NSTEPS)
    sim.sync()
    o = _oracle(orc, s, DROPLET)
    assert np.abs(sim.pos.cpu().numpy() - o["q"]).max() <= 1e-6
    assert np.abs(sim.vel.cpu().numpy() - o["v"]).max() <= 1e-6
    assert sim.counters()["proposals"] == o["counters"]["proposals"]


@pytest.mark.parametrize("integrator,rate_mode", [(0, 0), (1, 0), (0, 1)],
                         ids=["bounce", "baoab", "bounce_type_pair_bounds"])
def test_list_overflow_is_reported(integrator, rate_mode):
    """A droplet of 1,500 waters squeezed to eight times water's density: its
    rows outgrow the capacities the build sizes from water's density (below the
    droplet's size, which caps them).  The stores past a row's end are dropped
    by the range check of the row's buffer resource (with per-type-pair bounds,
    a class's stores past its own capacity are skipped, so that one class does
    not spill into the next), the counts still take them, and the build
    reports the overflow; the context then still runs a normal droplet."""
    import paper_2002_07109_amd as B
    from paper_2002_07109_amd._abi import E_CAPACITY
    s = water_droplet(n_waters=1500, seed=5)
    c = s.pos.mean(0)
    pos = c + 0.5 * (s.pos - c)
    origin, dims = droplet_grid(pos, s.cell_size)
    s = dataclasses.replace(s, pos=pos, grid_origin=origin, grid_dims=dims)
    sim = gpu_sim(s, dict(DROPLET, integrator=integrator, rate_mode=rate_mode))
    with pytest.raises(B.BounceError) as e:
        sim.profile_kernel(1, 1)
    assert e.value.status == E_CAPACITY
    sim.close()
    # the next context on the device is unaffected
    ok = gpu_sim(water_droplet(n_waters=100, seed=6), dict(DROPLET, integrator=integrator, rate_mode=rate_mode))
    ok.step(20)
    ok.sync()
    assert np.isfinite(ok.pos.cpu().numpy()).all()
    ok.close()

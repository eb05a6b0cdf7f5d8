"""bounce_bind_static: a context bound to the library's static per-device
workspace (no caller allocation) gives the same results as one bound to a
caller-allocated workspace, on two binds in a row (the second with a smaller
system), and systems too large for it are refused."""
import numpy as np
import pytest

from helpers import BOX, DROPLET, FF, gpu_sim, relaxed_box, relaxed_droplet

pytestmark = pytest.mark.gpu


def _static_sim(system, cfg, fp64):
    import paper_2002_07109_amd as B
    p = B.make_params(integrator=cfg["integrator"], coulomb=cfg["coulomb"],
                      periodic=cfg["periodic"], dt=cfg["dt"], gamma=cfg["gamma"],
                      temperature=cfg["temperature"], r_on=cfg["r_on"], r_off=cfg["r_off"],
                      r_cut=cfg["r_cut"], skin=cfg["skin"], ewald_alpha=cfg["ewald_alpha"],
                      rebuild_interval=cfg["rebuild_interval"], seed=cfg["seed"],
                      bound_scale=cfg["bound_scale"], cell_size=system.cell_size,
                      pair_precision=B.PAIR_FP64 if fp64 else B.PAIR_FP32, use_graph=1)
    return B.Simulation(system, p, FF["charge"], FF["eps"], FF["sigma"], static_workspace=True)


def _compare(system, cfg, steps, fp64):
    ref = gpu_sim(system, cfg, fp64=fp64, use_graph=True)
    ref.step(steps)
    ref.sync()
    st = _static_sim(system, cfg, fp64)
    st.step(steps)
    st.sync()
    assert np.array_equal(st.pos.cpu().numpy(), ref.pos.cpu().numpy())
    assert np.array_equal(st.vel.cpu().numpy(), ref.vel.cpu().numpy())
    assert st.counters()["proposals"] == ref.counters()["proposals"]
    e, er = st.energies()[0], ref.energies()[0]
    for k in ("bond", "angle", "coul", "lj", "kin"):
        assert e[k] == er[k], k
    return st


def test_static_workspace_matches_caller_workspace_twice():
    # first bind: the 1,536-atom periodic box; second: a 120-atom droplet
    a = _compare(relaxed_box("b8"), BOX, 30, fp64=False)
    b = _compare(relaxed_droplet("r0"), DROPLET, 40, fp64=True)
    # the first context lost the device's static workspace to the second
    import paper_2002_07109_amd as B
    with pytest.raises(B.BounceError) as e:
        a.step(1)
    assert e.value.status == -8
    b.step(5)
    b.sync()


def test_static_workspace_refuses_large_systems():
    import paper_2002_07109_amd as B
    from workloads import water_box
    big = water_box(n_side=20, box_len=62.0, seed=0)
    with pytest.raises(B.BounceError) as e:
        _static_sim(big, BOX, fp64=False)
    assert e.value.status == -10

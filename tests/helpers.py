"""Shared test set-up: one configuration dict drives both the oracle and the
GPU library, so the two see the same parameters and the same seeded inputs."""
import copy
import os

import numpy as np

from workloads import tip3p_params, water_droplet

FF = tip3p_params()

# bare-Coulomb droplets: with the 5/6 A split the B J A O A J B scheme heats a
# flexible-water droplet quickly at dt = 1 fs (both implementations agree); the
# droplet trajectories run at dt = 0.25 fs, where the scheme is stable
DROPLET = dict(integrator=0, periodic=0, coulomb=0, dt=0.25, gamma=1e-3, temperature=300.0,
               r_on=5.0, r_off=6.0, r_cut=9.0, skin=2.0, ewald_alpha=0.35, rebuild_interval=10,
               seed=0, bound_scale=1.0, rate_mode=0)
# periodic boxes: Ewald real-space erfc with alpha = 0.45/A (the benchmark's model)
BOX = dict(DROPLET, periodic=1, coulomb=1, r_on=6.0, r_off=7.0, dt=1.0, ewald_alpha=0.45)


def oracle_params(orc, sys, cfg, replica=0):
    return orc.make_params(sys, integrator=cfg["integrator"], coulomb=cfg["coulomb"],
                           dt=cfg["dt"], gamma=cfg["gamma"], temperature=cfg["temperature"],
                           r_on=cfg["r_on"], r_off=cfg["r_off"], r_cut=cfg["r_cut"],
                           skin=cfg["skin"], ewald_alpha=cfg["ewald_alpha"],
                           rebuild_interval=cfg["rebuild_interval"], seed=cfg["seed"],
                           replica=replica, bound_scale=cfg["bound_scale"],
                           periodic=bool(cfg["periodic"]), rate_mode=cfg.get("rate_mode", 0),
                           pme_grid=cfg.get("pme_grid"), pme_order=cfg.get("pme_order", 5),
                           respa_m=cfg.get("respa_m", 0), respa_outer=cfg.get("respa_outer", 0),
                           jump_split=cfg.get("jump_split", 0), r_on_lj=cfg.get("r_on_lj"),
                           r_off_lj=cfg.get("r_off_lj"))


def gpu_sim(systems, cfg, fp64=False, log_events=False, event_capacity=0, use_graph=False):
    import paper_2002_07109_amd as B
    cell = (systems[0] if isinstance(systems, (list, tuple)) else systems).cell_size
    p = B.make_params(integrator=cfg["integrator"], coulomb=cfg["coulomb"],
                      periodic=cfg["periodic"], dt=cfg["dt"], gamma=cfg["gamma"],
                      temperature=cfg["temperature"], r_on=cfg["r_on"], r_off=cfg["r_off"],
                      r_cut=cfg["r_cut"], skin=cfg["skin"], ewald_alpha=cfg["ewald_alpha"],
                      rebuild_interval=cfg["rebuild_interval"], seed=cfg["seed"],
                      bound_scale=cfg["bound_scale"], cell_size=cell,
                      pair_precision=B.PAIR_FP64 if fp64 else B.PAIR_FP32,
                      log_events=int(log_events), event_capacity=event_capacity,
                      use_graph=int(use_graph), rate_mode=cfg.get("rate_mode", 0),
                      pme_grid=cfg.get("pme_grid") or (0, 0, 0), pme_order=cfg.get("pme_order", 5),
                      respa_m=cfg.get("respa_m", 0), respa_outer=cfg.get("respa_outer", 0),
                      jump_split=cfg.get("jump_split", 0), r_on_lj=cfg.get("r_on_lj") or 0.0,
                      r_off_lj=cfg.get("r_off_lj") or 0.0, persistent=cfg.get("persistent", 0),
                      pair_kernel=cfg.get("pair_kernel", 0))
    return B.Simulation(systems, p, FF["charge"], FF["eps"], FF["sigma"])


def rel_err(a, b):
    """max_i |a_i - b_i| / RMS_i |b_i| over per-atom 3-vectors."""
    a, b = np.asarray(a), np.asarray(b)
    rms = np.sqrt(np.mean(np.sum(b * b, axis=-1)))
    return float(np.max(np.linalg.norm(a - b, axis=-1)) / rms)


def event_keys(ev, fields=("step", "phase", "atom", "k", "partner", "accepted")):
    keys = np.stack([ev[f].astype(np.int64) for f in fields], 1)
    if keys.size == 0:
        return keys
    return keys[np.lexsort(keys.T[::-1])]


_FIX = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "relaxed_droplets.npz")
_SPEC = {"c0": (216, 0, 5), "r0": (40, 3, 200), "r1": (150, 3, 201), "r2": (90, 3, 202)}
_BOX_SPEC = {"b8": (8, 24.8, 1)}


def relaxed_droplet(name):
    """Seeded droplet with the oracle-relaxed positions and velocities of
    tests/golden/relaxed_droplets.npz (written by tests/golden/make_fixtures.py)."""
    nw, seed, stream = _SPEC[name]
    s = copy.deepcopy(water_droplet(n_waters=nw, seed=seed, stream=stream))
    z = np.load(_FIX)
    s.pos, s.vel = z[name + "_pos"].copy(), z[name + "_vel"].copy()
    return s


def relaxed_box24k():
    """The 24,000-atom benchmark box (20^3 waters, 62 A, seed 0) with the
    oracle-relaxed state of tests/golden/relaxed_box24k.npz."""
    from workloads import water_box
    s = copy.deepcopy(water_box(n_side=20, box_len=62.0, seed=0))
    z = np.load(os.path.join(os.path.dirname(_FIX), "relaxed_box24k.npz"))
    s.pos, s.vel = z["pos"].copy(), z["vel"].copy()
    return s


def relaxed_box(name):
    """Seeded periodic box with the oracle-relaxed state of the fixture file."""
    from workloads import water_box
    n_side, edge, seed = _BOX_SPEC[name]
    s = copy.deepcopy(water_box(n_side=n_side, box_len=edge, seed=seed))
    z = np.load(_FIX)
    s.pos, s.vel = z[name + "_pos"].copy(), z[name + "_vel"].copy()
    return s


def sum_abs_pair_energy(orc, p, topo, q, box=None):
    """Sum over unordered non-excluded pairs within r_cut of |W_sf(r)| (the
    oracle's shifted-force pair energy): the scale against which rounding of
    pair energies of either sign is measured."""
    rp, col = orc.build_list(p, topo, q, 0.0, p.r_cut)
    n = q.shape[0]
    i = np.repeat(np.arange(n), np.diff(rp))
    keep = col > i
    i, j = i[keep], col[keep]
    d = q[i] - q[j]
    if box is not None:
        d -= box * np.rint(d / box)
    r = np.sqrt((d * d).sum(1))
    t = topo.type
    return float(sum(abs(orc.pair_wsf(p, int(a), int(b), float(x))[0])
                     for a, b, x in zip(t[i], t[j], r)))


def first_divergence(gpu_ev, orc_ev):
    """Walk the two event logs half-step by half-step in time order.  Returns
    None if they are identical, else (step, phase, [(atom, k, oracle event or
    None)]) for the first half-step that differs: per atom whose chain differs
    there, its first differing proposal.  Atoms' chains within one half-step
    are independent (positions are fixed during J), so each such atom's first
    difference is a separate accept-test decision."""
    keys = ("step", "phase", "atom", "k", "partner", "accepted")
    a = event_keys(gpu_ev, keys)
    o_sorted = np.sort(orc_ev, order=["step", "phase", "atom", "k"])
    b = event_keys(o_sorted, keys)
    if a.shape == b.shape and np.array_equal(a, b):
        return None
    half = lambda k: k[:, 0] * 4 + k[:, 1]
    ha, hb = half(a), half(b)
    for h in np.union1d(ha, hb):
        ea, eb = a[ha == h], b[hb == h]
        if ea.shape == eb.shape and np.array_equal(ea, eb):
            continue
        ob = o_sorted[hb == h]
        out = []
        for atom in np.union1d(ea[:, 2], eb[:, 2]):
            ra, rb = ea[ea[:, 2] == atom], eb[eb[:, 2] == atom]
            m = min(len(ra), len(rb))
            diff = [k for k in range(m) if not np.array_equal(ra[k], rb[k])]
            if not diff and len(ra) == len(rb):
                continue
            k = diff[0] if diff else m
            orow = ob[ob["atom"] == atom]
            out.append((int(atom), k + 1, orow[k] if k < len(orow) else None))
        return int(h // 4), int(h % 4), out
    return None

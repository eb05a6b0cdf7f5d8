#!/usr/bin/env python
"""Throughput of BOUNCE against BAOAB (both at 1 fs) on one MI355X.

Workload: the periodic 24,000-atom water box (8,000 flexible 3-site waters in a
62 A cube, 1 g/cm^3), real-space Ewald erfc Coulomb (alpha = 0.45/A) + LJ with
a 9 A shifted-force cutoff and a 2 A Verlet skin, FP32 pair arithmetic with FP64
accumulation and FP64 state, BOUNCE split r'/r'' = 6/7 A.  Inputs are synthetic (seeded lattice
waters, Maxwell velocities) and resident in HBM before the timed region; the
state is first relaxed on the GPU (BAOAB with strong friction, untimed).

One JSON line: ns/day of BOUNCE (value) with BAOAB's ns/day, pair evaluations
per second for both, the roofline position of the dominant kernel (the F_0 pair
kernel) and the FP64 CPU oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic FP32 operations per evaluated pair (adds, multiplies, each half of
# an FMA, and each transcendental counted once): r^2 5, rsqrt 1, r 1; Coulomb
# alpha r 1, erfc 1, exp(-(alpha r)^2) 2, g 1, g' 3; Lennard-Jones 10;
# W' = qq g' + LJ' - u'(rc) 3; switch 9; (1 - chi) W'/r 3; accumulation 6
FLOPS_SHORT = 46     # (1 - chi) W'_sf d/r: distance, rsqrt, erfc + exp Coulomb, LJ, switch, accumulate
FLOPS_FULL = 36      # W'_sf d/r without the switch
PEAK_FP32 = 157.3    # TFLOP/s, MI355X vector FP32 (published)
# transcendentals per pair among the counted operations (rsqrt, erfc, exp); the
# op-mix bound issues them at a quarter of the unpacked FP32 rate
TRANSC_PER_PAIR = 3


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pair_short_24k_box_traffic.md")
PAIR_SOURCES = ("kernels_pair.hip", "bounce_pairrow.hpp", "bounce_device.hpp", "bounce_kernels.hpp",
                "bounce_lists.hpp")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pair_source_hash():
    """Hash of the sources the short-range pair kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in PAIR_SOURCES:
        with open(os.path.join(ROOT, "paper_2002_07109_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(lanes):
    """HBM bytes per launch of the short-range pair kernel, from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary; None unless that summary was taken
    on the current kernel source and holds these lanes per atom."""
    try:
        text = open(TRAFFIC_FILE).read()
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_hash") != pair_source_hash():
        return None
    entry = rec.get("by_lanes", {}).get(str(lanes))
    return entry["hbm_bytes_per_launch"] if entry else None


def copy_calibration(mib):
    """A plain device-to-device copy of known size, for scaling the HBM
    counters (FETCH_SIZE, WRITE_SIZE) of a rocprofv3 --pmc run of this script."""
    import torch
    a = torch.ones(mib << 20, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 copies of {mib} MiB")


def pair_count_open(pos, r, n_excl_within):
    """Unordered non-excluded pairs with |d| < r, no periodic images."""
    from scipy.spatial import cKDTree
    t = cKDTree(pos)
    return int(t.count_neighbors(t, r) - pos.shape[0]) // 2 - n_excl_within


def pair_count(pos, box, r, n_excl_within):
    """Unordered non-excluded pairs with |d| < r (minimum image)."""
    from scipy.spatial import cKDTree
    wrapped = np.mod(pos, box)
    wrapped[wrapped >= box] = 0.0
    t = cKDTree(wrapped, boxsize=box)
    return int(t.count_neighbors(t, r) - pos.shape[0]) // 2 - n_excl_within


RATE_MODES = {"atom": 0, "pair": 1}


def pair_ms_over_interval(sim, interval, reps):
    """Mean duration (ms) of the F_0 pair kernel over one list-rebuild interval:
    timed after each of `interval` single steps (the far parts of the force rows
    are walked only on the later steps of an interval), `reps` launches each."""
    t = 0.0
    for _ in range(interval):
        sim.step(1)
        t += sim.profile_kernel(0, reps)
    sim.sync()
    return t / interval


def run_gpu(args, system, ff, integrator, state, rate_mode=0, dt=1.0, rebuild=None, **mesh):
    import torch
    import paper_2002_07109_amd as B
    p = B.make_params(integrator=integrator, pair_precision=B.PAIR_FP32, coulomb=B.COUL_EWALD,
                      periodic=1, dt=dt, gamma=1e-3, temperature=300.0, r_on=args.r_on,
                      r_off=args.r_off, r_cut=9.0, skin=args.skin, ewald_alpha=args.alpha,
                      rebuild_interval=rebuild or args.rebuild, seed=0, cell_size=system.cell_size,
                      use_graph=0 if args.no_graph else 1, rate_mode=rate_mode,
                      pair_kernel=args.pair_kernel, **mesh)
    sim = B.Simulation(system, p, ff["charge"], ff["eps"], ff["sigma"])
    sim.set_state(pos=state[0], vel=state[1], step=0)
    sim.step(args.warmup)
    sim.sync()
    tuned = sim.tune(reps=20)      # lanes per atom and the launch structure
    lanes, tune = tuned["pair_lanes"], tuned["pair_ms"]
    # the autotuner drops the K-step graph: run to the next list interval and
    # replay one whole interval, so that the graph is captured and instantiated
    # before the timed region, which then starts at a list rebuild
    K = rebuild or args.rebuild
    sim.step((-sim.get_step()) % K + K)
    sim.sync()
    c0 = sim.counters()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(sim.stream)
    sim.step(args.steps)
    ev1.record(sim.stream)
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    c1 = sim.counters()
    pair_ms = pair_ms_over_interval(sim, rebuild or args.rebuild, 10)
    build_ms = sim.profile_kernel(1, 10)
    mesh_ms = sim.profile_kernel(4, 20) if mesh.get("pme_grid") else None
    e = sim.energies()[0]
    t_e = time.perf_counter()
    sim.energies()                             # the energy pass, timed on its own
    energy_ms = 1e3 * (time.perf_counter() - t_e)
    step_ms = sim.profile_kernel(3, 50)        # advances the state: taken last
    out = dict(wall_s=wall, gpu_ms=gpu_ms, ms_per_step=1e3 * wall / args.steps,
               proposals_per_step=(c1["proposals"] - c0["proposals"]) / args.steps,
               accepted_per_step=(c1["accepted"] - c0["accepted"]) / args.steps,
               pair_kernel_ms=pair_ms, build_ms=build_ms, step_kernel_ms=step_ms, t_kin=e["tkin"],
               lanes=lanes, tune_ms={k: round(v, 5) for k, v in tune.items()},
               launch="fused" if tuned["persistent"] else "two launches",
               dry_step_ms={k: round(v, 5) for k, v in tuned["step_ms"].items()},
               e_pot=e["pair"] + e["bond"] + e["angle"], mesh_ms=mesh_ms,
               pos=sim.pos.cpu().numpy(), list_slots=sim.list_size(B.LIST_FORCE), energy_ms=energy_ms)
    sim.close()
    return out


def equilibrate(args, system, ff):
    import paper_2002_07109_amd as B
    p = B.make_params(integrator=B.BAOAB, pair_precision=B.PAIR_FP32, periodic=1, dt=1.0,
                      gamma=0.05, temperature=300.0, r_cut=9.0, skin=2.0, rebuild_interval=10,
                      ewald_alpha=args.alpha,
                      seed=12345, cell_size=system.cell_size, use_graph=1)
    sim = B.Simulation(system, p, ff["charge"], ff["eps"], ff["sigma"])
    done = 0
    while done < args.equil:
        k = min(500, args.equil - done)
        sim.step(k)
        sim.sync()
        done += k
        log(f"equilibration {done}/{args.equil} steps: T_kin = {sim.energies()[0]['tkin']:.1f} K")
    state = (sim.pos.cpu().numpy(), sim.vel.cpu().numpy())
    sim.close()
    return state


def run_batch(args, ff):
    """64 uneven non-periodic droplets in one context (every kernel spans all
    replicas; the K-step schedule is one hipGraph)."""
    import torch
    import paper_2002_07109_amd as B
    from workloads import droplet_batch
    systems = droplet_batch(64)
    mk = lambda integ, gamma, seed, mode=0: B.make_params(
        integrator=integ, pair_precision=B.PAIR_FP32, coulomb=B.COUL_BARE, periodic=0,
        dt=args.batch_dt, gamma=gamma, temperature=300.0, r_on=7.0, r_off=8.0, r_cut=9.0,
        skin=2.0, rebuild_interval=args.batch_rebuild, seed=seed, cell_size=systems[0].cell_size, use_graph=1,
        rate_mode=mode)
    # relax the lattice starts (BAOAB with strong friction, untimed)
    sim = B.Simulation(systems, mk(B.BAOAB, 0.05, 99), ff["charge"], ff["eps"], ff["sigma"])
    sim.step(800)
    sim.sync()
    pos, vel = sim.pos.cpu().numpy(), sim.vel.cpu().numpy()
    sim.close()
    sizes = [s.n_atoms for s in systems]
    out = {"workload": "64 non-periodic flexible-water droplets, %d-%d atoms (%d in all), bare "
                       "Coulomb + LJ, rc 9 A, BOUNCE r'/r'' = 7/8 A, dt %g fs, FP32 pair arithmetic"
                       % (min(sizes), max(sizes), sum(sizes), args.batch_dt),
           "rebuild_interval": args.batch_rebuild,
           "steps": args.batch_steps}
    # BOUNCE with one bound per atom type and per type pair, and BAOAB at the
    # same time step for comparison
    for mode_name, integ, mode in (("atom_bounds", B.BJAOAJB, 0), ("pair_bounds", B.BJAOAJB, 1),
                                   ("baoab", B.BAOAB, 0)):
        sim = B.Simulation(systems, mk(integ, 1e-3, 0, mode), ff["charge"], ff["eps"],
                           ff["sigma"])
        sim.set_state(pos=pos, vel=vel, step=0)
        sim.step(50)
        sim.sync()
        tuned = sim.tune(reps=10)
        lanes = tuned["pair_lanes"]
        sim.step(10)
        sim.sync()
        c0 = [sim.counters(r) for r in range(len(systems))]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(args.batch_steps)
        sim.sync()
        wall = time.perf_counter() - t0
        c1 = [sim.counters(r) for r in range(len(systems))]
        n = sim.n
        # the pair kernel's roofline over all droplets: pairs within r'' (BOUNCE)
        # or rc (BAOAB) counted per droplet (no periodic images, exclusions removed)
        rlim, fl = (8.0, FLOPS_SHORT) if integ == B.BJAOAJB else (9.0, FLOPS_FULL)
        pair_ms = pair_ms_over_interval(sim, args.batch_rebuild, 4)
        q = sim.pos.cpu().numpy()
        pairs = 0
        for r, s in enumerate(systems):
            b, e = sim.offsets[r], sim.offsets[r + 1]
            pairs += pair_count_open(q[b:e], rlim, s.excl.shape[0])
        sim.close()
        tflops = pairs * fl / (pair_ms * 1e-3) / 1e12
        ms = 1e3 * wall / args.batch_steps
        diff = lambda k: (sum(c[k] for c in c1) - sum(c[k] for c in c0)) / args.batch_steps
        out[mode_name] = {"ms_per_step": round(ms, 5), "atom_steps_per_s": n * 1e3 / ms,
                          "proposals_per_step": diff("proposals"),
                          "accepted_per_step": diff("accepted"), "pair_lanes": lanes,
                          "pair_kernel_us": round(pair_ms * 1e3, 3), "pairs_in_range": pairs,
                          "pair_kernel_tflops": round(tflops, 4),
                          "pair_kernel_frac": round(tflops / PEAK_FP32, 5),
                          "launch": "fused" if tuned["persistent"] else "two launches",
                          "dry_step_ms": {k: round(v, 5) for k, v in tuned["step_ms"].items()}}
        log(f"batch {mode_name}: {out[mode_name]}")
    out["speedup_vs_baoab"] = round(out["baoab"]["ms_per_step"] / out["atom_bounds"]["ms_per_step"], 4)
    return out


RDF_RMAX, RDF_BINS = 8.0, 160


def structure_summary(counts, n_samples, n_o, volume):
    """O-O radial distribution from accumulated pair counts: first peak position
    and height, first minimum, and the coordination number up to that minimum."""
    dr = RDF_RMAX / RDF_BINS
    edges = np.arange(RDF_BINS + 1) * dr
    shell = 4.0 / 3.0 * np.pi * np.diff(edges ** 3)
    rho = n_o / volume
    g = counts[0, 0] / (n_samples * n_o * rho * shell)
    mid = 0.5 * (edges[1:] + edges[:-1])
    k1 = int(np.argmax(g))
    kmin = k1 + int(np.argmin(g[k1:k1 + int(2.0 / dr)]))
    coord = float(counts[0, 0, :kmin + 1].sum() / (n_samples * n_o))
    return {"oo_peak_r": round(float(mid[k1]), 3), "oo_peak_g": round(float(g[k1]), 3),
            "oo_min_r": round(float(mid[kmin]), 3), "oo_coordination": round(coord, 3)}


def accuracy_run(args, system, ff, state, integ, dt, m=0, r_on=None, r_off=None):
    """One run for the accuracy comparison: 2 ps to decorrelate from the start,
    then args.accuracy ps sampled every 100 fs.  Returns <T_kin> and <E_pot>
    per water with block standard errors (10 blocks), the O-O radial
    distribution summary accumulated over the samples and the O self-diffusion
    coefficient from the slope of the unwrapped mean squared displacement over
    the second half of the run."""
    import paper_2002_07109_amd as B
    n_o = int((system.atom_type == 0).sum())
    volume = float(np.prod(system.box))
    p = B.make_params(integrator=integ, pair_precision=B.PAIR_FP32, coulomb=B.COUL_EWALD,
                      periodic=1, dt=dt, gamma=1e-3, temperature=300.0,
                      r_on=args.r_on if r_on is None else r_on,
                      r_off=args.r_off if r_off is None else r_off, r_cut=9.0, skin=args.skin,
                      ewald_alpha=args.alpha,
                      rebuild_interval=args.rebuild if dt == 1.0 else 4 * args.rebuild,
                      seed=args.accuracy_seed, cell_size=system.cell_size, use_graph=1, respa_m=m,
                      respa_outer=B.OUTER_NONBONDED if m else B.OUTER_RECIP)
    sim = B.Simulation(system, p, ff["charge"], ff["eps"], ff["sigma"])
    sim.set_state(pos=state[0], vel=state[1], step=0)
    per = int(round(100.0 / dt))
    n_samples = int(round(args.accuracy * 1000.0 / 100.0))
    sim.step(int(round(2000.0 / dt)))        # 2 ps to decorrelate from the start
    ref = sim.pos.clone()
    T, E, msd = [], [], []
    counts = np.zeros((2, 2, RDF_BINS))
    for _ in range(n_samples):
        sim.step(per)
        e = sim.energies()[0]
        T.append(e["tkin"])
        E.append((e["pair"] + e["bond"] + e["angle"]) / (system.n_atoms / 3))
        counts += sim.rdf_counts(RDF_RMAX, RDF_BINS)
        msd.append(sim.msd(ref)[0, 0])
    sim.close()
    res = {}
    for key, x in (("t_kin_K", np.array(T)), ("e_pot_per_water", np.array(E))):
        blocks = x[: len(x) // 10 * 10].reshape(10, -1).mean(1)
        res[key] = [round(float(x.mean()), 4), round(float(blocks.std(ddof=1) / np.sqrt(10)), 4)]
    res.update(structure_summary(counts, n_samples, n_o, volume))
    t_fs = 100.0 * np.arange(1, n_samples + 1)
    half = n_samples // 2
    slope = np.polyfit(t_fs[half:], np.array(msd)[half:], 1)[0]    # A^2 / fs
    res["d_o_1e-5_cm2_s"] = round(float(slope / 6.0 * 1e4), 3)
    return res


def matched(res, ref, ba):
    """|X - X_ref| <= |X_BAOAB - X_ref| + 2 sigma (sigma of X), per quantity."""
    return {key: bool(abs(res[key][0] - ref[key][0]) <= abs(ba[key][0] - ref[key][0]) +
                      2.0 * res[key][1])
            for key in ("t_kin_K", "e_pot_per_water")}


def run_accuracy(args, system, ff, state):
    """<T_kin> and <E_pot> per water of BOUNCE and BAOAB at 1 fs and of BOUNCE-RESPA
    (1 fs inner, short-range pair force on a 2 fs outer step) against BAOAB at
    0.25 fs (the reference), each over args.accuracy ps from the same state
    (accuracy_run).  With --accuracy-splits, BOUNCE at 1 fs is also run and
    timed at each switching window r'/r'' given, against the same reference."""
    import paper_2002_07109_amd as B
    out = {}
    # (name, integrator, inner dt, RESPA outer step in inner steps: the
    # short-range pair force on it; 0 = none)
    for name, integ, dt, m in (("bounce_1fs", B.BJAOAJB, 1.0, 0), ("baoab_1fs", B.BAOAB, 1.0, 0),
                               ("bounce_respa_1_2fs", B.BJAOAJB, 1.0, 2),
                               ("baoab_0.25fs", B.BAOAB, 0.25, 0)):
        out[name] = accuracy_run(args, system, ff, state, integ, dt, m)
        log(f"accuracy {name}: {out[name]}")
    ref, ba = out["baoab_0.25fs"], out["baoab_1fs"]
    for name in ("bounce_1fs", "bounce_respa_1_2fs"):
        out[name]["matched"] = matched(out[name], ref, ba)
    if args.accuracy_splits:
        sweep = {}
        base = run_gpu(args, system, ff, B.BAOAB, state)
        for r_on, r_off in args.accuracy_splits:
            key = f"{r_on:g}/{r_off:g}"
            res = accuracy_run(args, system, ff, state, B.BJAOAJB, 1.0, 0, r_on, r_off)
            res["matched"] = matched(res, ref, ba)
            sub = argparse.Namespace(**vars(args))
            sub.r_on, sub.r_off = r_on, r_off
            tm = run_gpu(sub, system, ff, B.BJAOAJB, state)
            res["ms_per_step"] = round(tm["ms_per_step"], 5)
            res["speedup_vs_baoab"] = round(base["ms_per_step"] / tm["ms_per_step"], 4)
            res["proposals_per_step"] = tm["proposals_per_step"]
            sweep[key] = res
            log(f"accuracy sweep {key}: {res}")
        out["split_sweep"] = dict(sweep, baoab_ms_per_step=round(base["ms_per_step"], 5))
    return out


def run_big(args, ff):
    """The same model on a 4x larger periodic box (32,000 waters in a 98 A
    cube, 96,000 atoms: a 32^3 lattice with 768 sites removed): BOUNCE and
    BAOAB ms/step after the same relaxation, showing how the latency-bound
    kernels fill the GPU."""
    from workloads import water_box
    system = water_box(n_side=32, box_len=98.0, seed=3, remove=768)
    sub_args = argparse.Namespace(**vars(args))
    sub_args.equil = 600
    sub_args.steps = args.big_steps
    sub_args.warmup = 50
    state = equilibrate(sub_args, system, ff)
    import paper_2002_07109_amd as B
    out = {"workload": "periodic 96,000-atom flexible water box (32,000 waters, 98 A cube), same "
                       "model and settings as the 24,000-atom box", "steps": args.big_steps}
    for name, integ in (("baoab", B.BAOAB), ("bounce", B.BJAOAJB)):
        r = run_gpu(sub_args, system, ff, integ, state)
        # the pair kernel's roofline at this size (pairs within r'' for BOUNCE's
        # short-range kernel, within rc for BAOAB's)
        rlim, fl = (args.r_off, FLOPS_SHORT) if integ == B.BJAOAJB else (9.0, FLOPS_FULL)
        pairs = pair_count(r["pos"], system.box, rlim, system.excl.shape[0])
        tflops = pairs * fl / (r["pair_kernel_ms"] * 1e-3) / 1e12
        out[name] = {"ms_per_step": round(r["ms_per_step"], 5),
                     "ns_per_day": round(1e-6 / (r["ms_per_step"] * 1e-3) * 86400.0, 3),
                     "pair_kernel_us": round(r["pair_kernel_ms"] * 1e3, 3),
                     "pair_kernel_tflops": round(tflops, 4),
                     "pair_kernel_frac": round(tflops / PEAK_FP32, 5),
                     "list_build_us": round(r["build_ms"] * 1e3, 3), "pair_lanes": r["lanes"]}
        log(f"96k box {name}: {out[name]}")
    out["speedup_vs_baoab"] = round(out["baoab"]["ms_per_step"] / out["bounce"]["ms_per_step"], 4)
    return out


def run_mesh(args, ff):
    """The 96,000-atom box with the reciprocal Ewald part by smooth PME (64^3
    mesh, order-5 B-splines, alpha = 0.35/A, real-space cutoff 9 A): BAOAB 1 fs
    with the mesh force every step, BOUNCE with it in F_0 every step, and
    BOUNCE-RESPA with it on an outer step of m = 2 and 5 inner steps (m divides
    the list interval), and BOUNCE-RESPA with the short-range pair force on the
    outer step too (bonded terms inner): 1/2 fs and 0.5/2 fs.  ns/day counts
    simulated time, so runs with a 0.5 fs inner step take twice the steps."""
    from workloads import water_box
    system = water_box(n_side=32, box_len=98.0, seed=3, remove=768)
    sub_args = argparse.Namespace(**vars(args))
    sub_args.equil = 600
    sub_args.steps = args.mesh_steps
    sub_args.warmup = 50
    sub_args.alpha = 0.35
    sub_args.r_on, sub_args.r_off = args.mesh_split
    state = equilibrate(sub_args, system, ff)
    import paper_2002_07109_amd as B
    grid = (64, 64, 64)
    out = {"workload": "periodic 96,000-atom flexible water box (32,000 waters, 98 A cube), real-space erfc "
                       "Coulomb + LJ (9 A cutoff) plus smooth-PME reciprocal sum (64^3 mesh, "
                       "order 5, alpha 0.35/A)", "steps": args.mesh_steps,
           "split": list(args.mesh_split)}
    # (name, integrator, m, outer force, inner dt, list interval in steps)
    runs = (("baoab", B.BAOAB, 0, B.OUTER_RECIP, 1.0, 10),
            ("bounce", B.BJAOAJB, 0, B.OUTER_RECIP, 1.0, 10),
            ("bounce_respa2", B.BJAOAJB, 2, B.OUTER_RECIP, 1.0, 10),
            ("bounce_respa5", B.BJAOAJB, 5, B.OUTER_RECIP, 1.0, 10),
            ("bounce_respa_nb_1_2", B.BJAOAJB, 2, B.OUTER_NONBONDED, 1.0, 10),
            ("bounce_respa_nb_05_2", B.BJAOAJB, 4, B.OUTER_NONBONDED, 0.5, 20))
    for name, integ, m, outer, dt, rebuild in runs:
        steps = int(round(args.mesh_steps / dt))       # the same simulated time
        sub_args.steps = steps
        try:
            r = run_gpu(sub_args, system, ff, integ, state, dt=dt, rebuild=rebuild, pme_grid=grid,
                        pme_order=5, respa_m=m, respa_outer=outer)
        except B.BounceError as e:
            out[name] = {"failed": str(e), "respa_m": m}
            log(f"96k box with mesh, {name}: {e}")
            continue
        out[name] = {"ms_per_step": round(r["ms_per_step"], 5), "dt_fs": dt, "steps": steps,
                     "ns_per_day": round(dt * 1e-6 / (r["ms_per_step"] * 1e-3) * 86400.0, 3),
                     "respa_m": m, "outer": "nonbonded+recip" if outer else "recip",
                     "mesh_us": round(r["mesh_ms"] * 1e3, 3),
                     "pair_kernel_us": round(r["pair_kernel_ms"] * 1e3, 3),
                     "t_kin": round(r["t_kin"], 2)}
        log(f"96k box with mesh, {name}: {out[name]}")
    for name, *_ in runs[1:]:
        if "ns_per_day" in out[name] and "ns_per_day" in out["baoab"]:
            out[name]["speedup_vs_baoab"] = round(out[name]["ns_per_day"] / out["baoab"]["ns_per_day"], 4)
    return out


def run_split(args, system, ff, state):
    """The separate Coulomb and Lennard-Jones jump mechanisms (jump_split)
    against the combined one on the same box and state, at the benchmark's
    alpha and at 0.35/A: ms per step, jump proposals per atom and step (all,
    and the Lennard-Jones share from a logged run), and the kinetic temperature
    over the second of 2 ps (BAOAB at 1 fs alongside).  A run stopped by a
    device condition (e.g. the skin guard after heating) is reported as such."""
    import paper_2002_07109_amd as B
    out = {"workload": "24,000-atom box, Coulomb window r'/r'' = %g/%g A; split: Lennard-Jones "
                       "window %g/%g A" % (args.r_on, args.r_off, *args.split_lj)}
    n = system.n_atoms
    for alpha in sorted({args.alpha, 0.35}, reverse=True):
        res = {}
        for name, integ, split in (("baoab", B.BAOAB, 0), ("combined", B.BJAOAJB, 0),
                                   ("split", B.BJAOAJB, 1)):
            mk = lambda log: B.make_params(
                integrator=integ, pair_precision=B.PAIR_FP32, coulomb=B.COUL_EWALD, periodic=1,
                dt=1.0, gamma=1e-3, temperature=300.0, r_on=args.r_on, r_off=args.r_off, r_cut=9.0,
                skin=args.skin, ewald_alpha=alpha, rebuild_interval=args.rebuild, seed=5,
                cell_size=system.cell_size, use_graph=1, jump_split=split,
                r_on_lj=args.split_lj[0] if split else 0.0,
                r_off_lj=args.split_lj[1] if split else 0.0,
                log_events=log, event_capacity=400000 if log else 0)
            sim = B.Simulation(system, mk(0), ff["charge"], ff["eps"], ff["sigma"])
            sim.set_state(pos=state[0], vel=state[1], step=0)
            r = {}
            try:
                sim.step(1000)
                sim.sync()
                T = []
                c0 = sim.counters()
                t0 = time.perf_counter()
                for _ in range(10):
                    sim.step(100)
                    T.append(sim.energies()[0]["tkin"])
                c1 = sim.counters()
                r["t_kin_K"] = round(float(np.mean(T)), 2)
                r["proposals_per_atom_step"] = (c1["proposals"] - c0["proposals"]) / (1000 * n)
                r["accepted_per_atom_step"] = (c1["accepted"] - c0["accepted"]) / (1000 * n)
                sim.step((-sim.get_step()) % args.rebuild + args.rebuild)
                sim.sync()
                t0 = time.perf_counter()
                sim.step(500)
                sim.sync()
                r["ms_per_step"] = round(1e3 * (time.perf_counter() - t0) / 500, 5)
            except B.BounceError as e:
                r["stopped"] = str(e)
            sim.close()
            if integ == B.BJAOAJB and "stopped" not in r:
                lg = B.Simulation(system, mk(1), ff["charge"], ff["eps"], ff["sigma"])
                lg.set_state(pos=state[0], vel=state[1], step=0)
                lg.step(50)
                lg.sync()
                ev, ne = lg.events()
                lg.close()
                r["lj_share_of_proposals"] = round(float((ev["mech"] == 1).mean()), 4) if len(ev) else 0.0
                r["lj_proposals_per_atom_step"] = float((ev["mech"] == 1).sum()) / (50 * n)
            res[name] = r
            log(f"split mechanisms, alpha {alpha}: {name}: {r}")
        out["alpha_%g" % alpha] = res
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(args):
    """One oracle leg, run in a child process whose OMP_NUM_THREADS fixes the
    thread count: `steps` steps of the seeded 24,000-atom box (the list search
    runs at step 0 and every `rebuild` steps; the oracle times it apart)."""
    import ctypes
    from oracle import oracle as orc
    from workloads import water_box
    integ = {"bounce": orc.BOUNCE, "baoab": orc.BAOAB}[args.cpu_leg]
    system = water_box(n_side=20, box_len=62.0, seed=0)
    p = orc.make_params(system, integrator=integ, r_on=args.r_on, r_off=args.r_off,
                        r_cut=9.0, skin=args.skin, rebuild_interval=args.rebuild,
                        ewald_alpha=args.alpha)
    topo = orc.Topology.from_system(system)
    t0 = time.perf_counter()
    o = orc.run(p, topo, system.pos, system.vel, 0, args.cpu_steps)
    wall = time.perf_counter() - t0
    try:
        threads = ctypes.CDLL("libgomp.so.1").omp_get_max_threads()
    except OSError:
        threads = int(os.environ.get("OMP_NUM_THREADS", "1"))
    print(json.dumps(dict(integrator=args.cpu_leg, steps=args.cpu_steps, wall_s=wall,
                          threads=threads, rebuilds=int(o["counters"]["rebuilds"]),
                          list_search_s=o["list_seconds"], status=o["status_name"])), flush=True)


def cpu_baseline(args, system):
    """The FP64 oracle on bounded samples of the same workload (its seeded input
    state): BOUNCE and BAOAB, on one thread and on all host threads, each in a
    child process.  `value` is BOUNCE on all threads.  The oracle's list search
    is a plain O(N^2) loop; each leg states its share of the wall time and the
    rate with it taken out."""
    import subprocess
    all_threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    legs = {}
    for integ in ("bounce", "baoab"):
        for threads, steps in ((all_threads, args.cpu_steps), (1, args.cpu_steps_single)):
            env = dict(os.environ, OMP_NUM_THREADS=str(threads))
            cmd = [sys.executable, os.path.abspath(__file__), "--cpu-leg", integ,
                   "--cpu-steps", str(steps), "--r-on", str(args.r_on), "--r-off", str(args.r_off),
                   "--skin", str(args.skin), "--rebuild", str(args.rebuild), "--alpha", str(args.alpha)]
            log(f"oracle leg: {integ}, {threads} thread(s), {steps} steps")
            try:
                out = subprocess.run(cmd, env=env, capture_output=True, text=True, check=True,
                                     timeout=600)
                r = json.loads(out.stdout.strip().splitlines()[-1])
            except (subprocess.SubprocessError, ValueError, IndexError) as e:
                log(f"oracle leg {integ}/{threads} failed: {e}")
                legs[f"{integ}_{threads}t"] = {"error": str(e)[:200]}
                continue
            list_s = r["list_search_s"]
            rest = r["wall_s"] - list_s
            legs[f"{integ}_{r['threads']}t"] = {
                "ns_per_day": round(steps * 1e-6 / r["wall_s"] * 86400.0, 5),
                "ns_per_day_without_list_search": round(steps * 1e-6 / rest * 86400.0, 5),
                "threads": r["threads"], "steps": steps, "wall_s": round(r["wall_s"], 2),
                "list_searches": r["rebuilds"], "list_search_share": round(min(list_s / r["wall_s"], 1.0), 3),
                "status": r["status"]}
    main_leg = legs.get(f"bounce_{all_threads}t", {})
    if "ns_per_day" not in main_leg:
        return dict(value=None, unit="ns/day", cores=all_threads, kind="oracle",
                    sample="the oracle leg did not complete", legs=legs)
    return dict(value=main_leg["ns_per_day"], unit="ns/day", cores=main_leg["threads"], kind="oracle",
                sample=f"{main_leg['steps']} BOUNCE steps of the 24,000-atom box from its seeded input "
                       f"(list search at step 0 and every {args.rebuild} steps), "
                       f"{main_leg['wall_s']:.1f} s wall on {main_leg['threads']} threads",
                cpu_model=cpu_model(), host_threads=len(os.sched_getaffinity(0)), legs=legs)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--equil", type=int, default=1000)
    ap.add_argument("--skin", type=float, default=2.0)
    ap.add_argument("--r-on", type=float, default=6.0)
    ap.add_argument("--r-off", type=float, default=7.0)
    ap.add_argument("--rebuild", type=int, default=10)
    ap.add_argument("--alpha", type=float, default=0.45)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--rate-mode", choices=sorted(RATE_MODES), default="atom",
                    help="jump rate bounds of the headline BOUNCE run: one per atom type "
                         "(atom) or per type pair, superposed (pair); the other is also timed")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--cpu-steps-single", type=int, default=2,
                    help="steps of the one-thread oracle legs")
    ap.add_argument("--pair-kernel", type=int, choices=(0, 4, 8), default=0,
                    help="F_0 pair force: 0 per-atom rows, 4 or 8 cluster-pair tiles")
    ap.add_argument("--skip-box", action="store_true",
                    help="run only the --batch / --big / --mesh legs (no headline line)")
    ap.add_argument("--cpu-leg", choices=("bounce", "baoab"), default=None,
                    help=argparse.SUPPRESS)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--batch", action="store_true",
                    help="also time 64 uneven droplets in one context")
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--batch-dt", type=float, default=0.25)
    ap.add_argument("--batch-rebuild", type=int, default=40,
                    help="list rebuild interval K of the batch (steps; 40 x 0.25 fs = the 10 fs "
                         "list lifetime of the 1 fs box)")
    ap.add_argument("--big", action="store_true",
                    help="also time the 96,000-atom box with the same model")
    ap.add_argument("--big-steps", type=int, default=500)
    ap.add_argument("--mesh", action="store_true",
                    help="also time the 96,000-atom box with smooth PME (BAOAB, BOUNCE, BOUNCE-RESPA)")
    ap.add_argument("--mesh-steps", type=int, default=500)
    ap.add_argument("--mesh-split", type=lambda t: tuple(float(v) for v in t.split(",")),
                    default=(7.0, 8.0), metavar="R_ON,R_OFF",
                    help="switching window r', r'' of the mesh workload (A); at its alpha = "
                         "0.35/A the 6/7 A split runs away within 1,000 steps")
    ap.add_argument("--split", action="store_true",
                    help="also compare separate Coulomb and Lennard-Jones jump mechanisms with "
                         "the combined one (at the benchmark's alpha and at 0.35/A)")
    ap.add_argument("--split-lj", type=lambda t: tuple(float(v) for v in t.split(",")),
                    default=(5.0, 6.0), metavar="R_ON,R_OFF",
                    help="Lennard-Jones switching window of the separate mechanisms (A)")
    ap.add_argument("--accuracy", type=float, default=0.0, metavar="PS",
                    help="also compare <T_kin>, <E_pot> of BOUNCE and BAOAB at 1 fs with "
                         "BAOAB at 0.25 fs over PS picoseconds each")
    ap.add_argument("--accuracy-seed", type=int, default=7,
                    help="Philox seed of the accuracy runs (one replicate per seed)")
    ap.add_argument("--accuracy-splits", default="",
                    type=lambda t: [tuple(float(v) for v in p.split(",")) for p in t.split(";") if p],
                    metavar="R_ON,R_OFF;...",
                    help="with --accuracy: also run and time BOUNCE at these switching windows")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB device to device (counter calibration)")
    args = ap.parse_args()
    if args.cpu_leg:
        cpu_leg(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); no multi-GPU "
              "decomposition is built.", file=sys.stderr)
        sys.exit(2)

    from workloads import tip3p_params, water_box
    ff = tip3p_params()
    if args.skip_box:
        # only the extra legs asked for (for profiling them alone): no headline
        extra = {}
        if args.batch:
            log("timing 64 uneven droplets")
            extra["batch"] = run_batch(args, ff)
        if args.big:
            log("timing the 96,000-atom box")
            extra["big_box"] = run_big(args, ff)
        if args.mesh:
            log("timing the 96,000-atom box with the PME mesh")
            extra["mesh_box"] = run_mesh(args, ff)
        print(json.dumps(extra), flush=True)
        return
    log("building the 24,000-atom water box")
    system = water_box(n_side=20, box_len=62.0, seed=0)
    n_excl = system.excl.shape[0]
    state = equilibrate(args, system, ff)

    import paper_2002_07109_amd as B
    res = {}
    mode = RATE_MODES[args.rate_mode]
    other = "pair" if args.rate_mode == "atom" else "atom"
    for name, integ, rm in (("baoab", B.BAOAB, 0), ("bounce", B.BJAOAJB, mode),
                            ("bounce_" + other, B.BJAOAJB, RATE_MODES[other])):
        log(f"timing {name}: {args.warmup} warmup + {args.steps} steps")
        res[name] = run_gpu(args, system, ff, integ, state, rate_mode=rm)
        log(f"{name}: {res[name]['ms_per_step']:.4f} ms/step, step kernel "
            f"{res[name]['step_kernel_ms']*1e3:.1f} us, T_kin {res[name]['t_kin']:.1f} K")
    # BOUNCE-RESPA (Sec. V) on the same box: bonded terms and jumps on the inner
    # step, the short-range pair force on an outer step of 2 fs; the same
    # simulated time as the runs above
    respa = {}
    for name, dt, m in (("1/2 fs", 1.0, 2), ("0.5/2 fs", 0.5, 4)):
        sub = argparse.Namespace(**vars(args))
        sub.steps, sub.warmup = int(round(args.steps / dt)), int(round(args.warmup / dt))
        log(f"timing BOUNCE-RESPA {name}: {sub.warmup} warmup + {sub.steps} steps")
        r = run_gpu(sub, system, ff, B.BJAOAJB, state, rate_mode=mode, dt=dt,
                    rebuild=int(round(args.rebuild / dt)), respa_m=m, respa_outer=B.OUTER_NONBONDED)
        respa[name] = {"ms_per_step": round(r["ms_per_step"], 5), "dt_fs": dt, "respa_m": m,
                       "ns_per_day": round(dt * 1e-6 / (r["ms_per_step"] * 1e-3) * 86400.0, 3),
                       "t_kin_K": round(r["t_kin"], 2)}
        log(f"BOUNCE-RESPA {name}: {respa[name]}")

    box = system.box
    bo, ba = res["bounce"], res["baoab"]
    short_pairs = pair_count(bo["pos"], box, args.r_off, n_excl)
    full_pairs_bo = pair_count(bo["pos"], box, 9.0, n_excl)
    full_pairs_ba = pair_count(ba["pos"], box, 9.0, n_excl)
    ns_day = lambda ms: 1.0 * 1e-6 / (ms * 1e-3) * 86400.0
    steps_s_bo = 1e3 / bo["ms_per_step"]
    steps_s_ba = 1e3 / ba["ms_per_step"]
    # the dominant kernel of a step is the F_0 pair kernel
    achieved = short_pairs * FLOPS_SHORT / (bo["pair_kernel_ms"] * 1e-3) / 1e12
    achieved_ba = full_pairs_ba * FLOPS_FULL / (ba["pair_kernel_ms"] * 1e-3) / 1e12
    # the committed counter record is the row kernel's
    traffic = measured_traffic(bo["lanes"]) if not args.pair_kernel else None
    # unpacked FP32 with the transcendentals at a quarter rate
    peak_opmix = (PEAK_FP32 / 2) * FLOPS_SHORT / ((FLOPS_SHORT - TRANSC_PER_PAIR) + 4 * TRANSC_PER_PAIR)
    line = {
        "metric": "ns/day & pair-evals/s, BOUNCE vs BAOAB 1fs on same GPU, 24k-atom box",
        "value": round(ns_day(bo["ms_per_step"]), 3),
        "unit": "ns/day",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(bo["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic, f64 accumulation and state",
        "data": "synthetic",
        "config": {"workload": "periodic 24,000-atom flexible water box, 62 A cube, Ewald erfc "
                               "(alpha %g/A) + LJ, rc 9 A, skin 2 A, BOUNCE r'/r'' = %g/%g A, "
                               "dt 1 fs" % (args.alpha, args.r_on, args.r_off),
                   "n_atoms": system.n_atoms, "rebuild_interval": args.rebuild,
                   "skin": args.skin, "hip_graph": not args.no_graph,
                   "pair_kernel": "rows" if not args.pair_kernel else "clusters of %d" % args.pair_kernel},
        "bounce": {"ns_per_day": round(ns_day(bo["ms_per_step"]), 3),
                   "ms_per_step": round(bo["ms_per_step"], 5),
                   "pair_evals_per_s": (short_pairs + bo["proposals_per_step"]) * steps_s_bo,
                   "pair_slots_per_s": bo["list_slots"] * steps_s_bo,
                   "energy_pass_ms": round(bo["energy_ms"], 4),
                   "baoab_equivalent_pair_evals_per_s": full_pairs_bo * steps_s_bo,
                   "short_pairs_per_step": short_pairs,
                   "proposals_per_step": bo["proposals_per_step"],
                   "accepted_per_step": bo["accepted_per_step"],
                   "step_kernel_us": round(bo["step_kernel_ms"] * 1e3, 3),
                   "pair_kernel_us": round(bo["pair_kernel_ms"] * 1e3, 3),
                   "list_build_us": round(bo["build_ms"] * 1e3, 3),
                   "pair_lanes": bo["lanes"], "autotune_ms": bo["tune_ms"],
                   "launch": bo["launch"], "tuner_dry_step_ms": bo["dry_step_ms"],
                   "rate_bounds": args.rate_mode,
                   "t_kin_K": round(bo["t_kin"], 2), "e_pot": round(bo["e_pot"], 2)},
        "bounce_%s_bounds" % other: {
            "ms_per_step": round(res["bounce_" + other]["ms_per_step"], 5),
            "ns_per_day": round(ns_day(res["bounce_" + other]["ms_per_step"]), 3),
            "proposals_per_step": res["bounce_" + other]["proposals_per_step"],
            "accepted_per_step": res["bounce_" + other]["accepted_per_step"],
            "step_kernel_us": round(res["bounce_" + other]["step_kernel_ms"] * 1e3, 3),
            "list_build_us": round(res["bounce_" + other]["build_ms"] * 1e3, 3)},
        "baoab": {"ns_per_day": round(ns_day(ba["ms_per_step"]), 3),
                  "ms_per_step": round(ba["ms_per_step"], 5),
                  "pair_evals_per_s": full_pairs_ba * steps_s_ba,
                  "pair_slots_per_s": ba["list_slots"] * steps_s_ba,
                  "pairs_per_step": full_pairs_ba,
                  "step_kernel_us": round(ba["step_kernel_ms"] * 1e3, 3),
                  "pair_kernel_us": round(ba["pair_kernel_ms"] * 1e3, 3),
                  "pair_kernel_tflops": round(achieved_ba, 3),
                  "list_build_us": round(ba["build_ms"] * 1e3, 3),
                  "pair_lanes": ba["lanes"], "autotune_ms": ba["tune_ms"],
                  "launch": ba["launch"], "tuner_dry_step_ms": ba["dry_step_ms"],
                  "t_kin_K": round(ba["t_kin"], 2), "e_pot": round(ba["e_pot"], 2)},
        "speedup_vs_baoab": round(ba["ms_per_step"] / bo["ms_per_step"], 4),
        "bounce_respa_nonbonded": {k: dict(v, speedup_vs_baoab=round(v["ns_per_day"] / ns_day(ba["ms_per_step"]), 4))
                                   for k, v in respa.items()},
        "roofline": {"kernel": "F_0 pair kernel (BOUNCE short range)", "bound": "alu",
                     "achieved": round(achieved, 4), "peak": PEAK_FP32, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32, 5),
                     "traffic": traffic,
                     "flops_per_pair": FLOPS_SHORT, "pairs_per_launch": short_pairs,
                     "peak_unpacked": PEAK_FP32 / 2,
                     "frac_unpacked": round(achieved / (PEAK_FP32 / 2), 5),
                     "peak_opmix": round(peak_opmix, 3),
                     "frac_opmix": round(achieved / peak_opmix, 5),
                     "pair_slots_per_launch": bo["list_slots"],
                     "useful_pairs_per_slot": round(short_pairs / bo["list_slots"], 4),
                     "hbm_frac": (round(traffic / (bo["pair_kernel_ms"] * 1e-3) / 8e12, 4)
                                  if traffic else None)},
    }
    if args.batch:
        log("timing 64 uneven droplets")
        line["batch"] = run_batch(args, ff)
    if args.big:
        log("timing the 96,000-atom box")
        line["big_box"] = run_big(args, ff)
    if args.mesh:
        log("timing the 96,000-atom box with the PME mesh")
        line["mesh_box"] = run_mesh(args, ff)
    if args.split:
        log("comparing separate and combined jump mechanisms")
        line["split_mechanisms"] = run_split(args, system, ff, state)
    if args.accuracy > 0:
        line["accuracy"] = run_accuracy(args, system, ff, state)
    if not args.skip_cpu:
        log("timing the CPU oracle")
        line["cpu_baseline"] = cpu_baseline(args, system)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

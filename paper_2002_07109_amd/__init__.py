"""MI355X (gfx950) BOUNCE direct-space library: Python binding.

The C-ABI functions of include/bounce.h are available under the same names
(``bounce_step``, ``bounce_sync`` ...) through :func:`lib`.  :class:`Simulation`
marshals torch tensors (device memory, current HIP stream) into those calls and
:class:`DirectEnergy` wraps the differentiable direct-space energy as a
``torch.autograd.Function``.  No computation happens in Python.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import _abi
from ._abi import (BAOAB, BJAOAJB, COUL_BARE, COUL_EWALD, G_BONDED, G_FULL, G_LONG, G_RECIP, G_STEP,
                   G_SHORT,
                   LIST_CAND, LIST_FORCE, OUTER_NONBONDED, OUTER_RECIP, PAIR_FP32, PAIR_FP64, PH_JA, PH_JB, PH_O, RATE_ATOM,
                   RATE_PAIR, BounceError,
                   bounce_counters, bounce_event, bounce_params, bounce_system, check)

__all__ = ["lib", "Simulation", "DirectEnergy", "make_params", "BounceError", "BJAOAJB", "BAOAB",
           "PAIR_FP32", "PAIR_FP64", "COUL_BARE", "COUL_EWALD", "PH_JA", "PH_O", "PH_JB",
           "G_BONDED", "G_SHORT", "G_LONG", "G_FULL", "G_RECIP", "G_STEP", "LIST_FORCE", "LIST_CAND", "RATE_ATOM",
           "RATE_PAIR", "OUTER_RECIP", "OUTER_NONBONDED"]


def lib():
    """The loaded libbounce.so with typed C-ABI functions."""
    return _abi.load()


def make_params(**kw) -> bounce_params:
    """bounce_params with defaults: BOUNCE, FP32 pair math, dt = 1 fs, gamma = 1/ps,
    300 K, r'/r'' = 6/7, rc = 9, skin 2, alpha 0.35, K = 10, one rate bound per
    atom type (RATE_ATOM), no reciprocal-space mesh (pme_grid = (0, 0, 0); when
    set: B-spline order 5, mesh force in F_0 unless respa_m >= 1); with
    respa_m >= 1 and respa_outer = OUTER_NONBONDED the short-range pair force
    moves to the outer step too; jump_split = 1 gives the Coulomb and the
    Lennard-Jones long-range parts separate jump mechanisms (the LJ window
    r_on_lj, r_off_lj defaults to the Coulomb one); persistent = 1 makes each step one
    persistent launch over all replicas; pair_kernel = 4 or 8 evaluates F_0's pair
    force over cluster pairs of that many atoms instead of per-atom rows."""
    d = dict(integrator=BJAOAJB, pair_precision=PAIR_FP32, coulomb=COUL_EWALD, periodic=1,
             rebuild_interval=10, max_proposals=100000, log_events=0, use_graph=0, dt=1.0,
             gamma=1e-3, temperature=300.0, r_on=6.0, r_off=7.0, r_cut=9.0, skin=2.0,
             ewald_alpha=0.35, bound_scale=1.0, cell_size=4.4, seed=0, event_capacity=0,
             pair_lanes=0, rate_mode=RATE_ATOM, pme_grid=(0, 0, 0), pme_order=5, respa_m=0,
             respa_outer=OUTER_RECIP, jump_split=0, r_on_lj=0.0, r_off_lj=0.0, persistent=0,
             pair_kernel=0)
    d.update(kw)
    p = bounce_params()
    for k, v in d.items():
        if k == "pme_grid":
            for c in range(3):
                p.pme_grid[c] = int(v[c])
        else:
            setattr(p, k, v)
    return p


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _tptr(t):
    return C.c_void_p(t.data_ptr())


class Simulation:
    """One context over one or more replicas (systems with the attributes of
    ``workloads.WaterSystem``); positions and velocities live in torch tensors
    of shape (N, 3), float64, on ``device``."""

    def __init__(self, systems, params: bounce_params, charge, eps, sigma, device="cuda:0",
                 stream=None, static_workspace=False):
        import torch
        if not isinstance(systems, (list, tuple)):
            systems = [systems]
        self.torch = torch
        self.device = torch.device(device)
        self.L = lib()
        self.params = params
        self.systems = systems
        self.n_replicas = len(systems)
        sizes = [s.n_atoms for s in systems]
        self.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.n = int(self.offsets[-1])
        off = self.offsets
        cat = lambda f, dt: np.ascontiguousarray(np.concatenate([f(s) for s in systems]), dt)
        self._keep = dict(off=off, type=cat(lambda s: s.atom_type, np.int32),
                          mass=cat(lambda s: s.mass, np.float64))
        shift = lambda arr, r: arr + int(off[r])
        self._keep["bonds"] = np.ascontiguousarray(np.concatenate(
            [shift(s.bonds, r) for r, s in enumerate(systems)]), np.int32)
        self._keep["angles"] = np.ascontiguousarray(np.concatenate(
            [shift(s.angles, r) for r, s in enumerate(systems)]), np.int32)
        self._keep["excl"] = np.ascontiguousarray(np.concatenate(
            [shift(s.excl, r) for r, s in enumerate(systems)]), np.int32)
        for name in ("bond_k", "bond_r0", "angle_k", "angle_t0"):
            self._keep[name] = cat(lambda s, nm=name: getattr(s, nm), np.float64)
        self._keep["box"] = np.ascontiguousarray(np.stack([s.box for s in systems]), np.float64)
        self._keep["origin"] = np.ascontiguousarray(np.stack([s.grid_origin for s in systems]),
                                                    np.float64)
        self._keep["dims"] = np.ascontiguousarray(np.stack([s.grid_dims for s in systems]),
                                                  np.int32)
        self._keep["charge"] = np.ascontiguousarray(charge, np.float64)
        self._keep["eps"] = np.ascontiguousarray(eps, np.float64)
        self._keep["sigma"] = np.ascontiguousarray(sigma, np.float64)
        k = self._keep
        sysc = bounce_system()
        sysc.n_replicas = self.n_replicas
        sysc.n_atoms = self.n
        sysc.replica_offset = k["off"].ctypes.data
        sysc.box = k["box"].ctypes.data
        sysc.grid_origin = k["origin"].ctypes.data
        sysc.grid_dims = k["dims"].ctypes.data
        sysc.type = k["type"].ctypes.data
        sysc.mass = k["mass"].ctypes.data
        sysc.n_types = len(charge)
        sysc.charge, sysc.eps, sysc.sigma = (k["charge"].ctypes.data, k["eps"].ctypes.data,
                                             k["sigma"].ctypes.data)
        sysc.n_bonds = k["bonds"].shape[0]
        sysc.bonds, sysc.bond_k, sysc.bond_r0 = (k["bonds"].ctypes.data, k["bond_k"].ctypes.data,
                                                 k["bond_r0"].ctypes.data)
        sysc.n_angles = k["angles"].shape[0]
        sysc.angles, sysc.angle_k, sysc.angle_t0 = (k["angles"].ctypes.data,
                                                    k["angle_k"].ctypes.data,
                                                    k["angle_t0"].ctypes.data)
        sysc.n_excl = k["excl"].shape[0]
        sysc.excl = k["excl"].ctypes.data
        self.n_types = len(charge)
        ctx = C.c_void_p()
        check(self.L.bounce_create(C.byref(params), C.byref(ctx)), None, "bounce_create")
        self.ctx = ctx
        check(self.L.bounce_set_system(ctx, C.byref(sysc)), ctx, "bounce_set_system")
        nbytes = C.c_uint64()
        check(self.L.bounce_workspace_size(ctx, C.byref(nbytes)), ctx, "bounce_workspace_size")
        pos = np.concatenate([s.pos for s in systems])
        vel = np.concatenate([s.vel for s in systems])
        self.pos = torch.tensor(pos, dtype=torch.float64, device=self.device).contiguous()
        self.vel = torch.tensor(vel, dtype=torch.float64, device=self.device).contiguous()
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if static_workspace:
            # the library's static per-device workspace (bounce_bind_static)
            self.workspace = None
            with torch.cuda.device(self.device):
                check(self.L.bounce_bind_static(ctx, _tptr(self.pos), _tptr(self.vel),
                                                C.c_void_p(self.stream.cuda_stream)), ctx,
                      "bounce_bind_static")
        else:
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            check(self.L.bounce_bind(ctx, _tptr(self.workspace), nbytes.value, _tptr(self.pos),
                                     _tptr(self.vel), C.c_void_p(self.stream.cuda_stream)), ctx,
                  "bounce_bind")

    # -- stepping ----------------------------------------------------------
    def step(self, n):
        check(self.L.bounce_step(self.ctx, int(n)), self.ctx, "bounce_step")

    def sync(self):
        check(self.L.bounce_sync(self.ctx), self.ctx, "bounce_sync")

    def set_step(self, n):
        check(self.L.bounce_set_step(self.ctx, int(n)), self.ctx, "bounce_set_step")

    def get_step(self):
        v = C.c_int64()
        check(self.L.bounce_get_step(self.ctx, C.byref(v)), self.ctx, "bounce_get_step")
        return v.value

    def set_state(self, pos=None, vel=None, step=None):
        self.stream.synchronize()
        if pos is not None:
            self.pos.copy_(self.torch.as_tensor(pos, dtype=self.torch.float64))
        if vel is not None:
            self.vel.copy_(self.torch.as_tensor(vel, dtype=self.torch.float64))
        self.torch.cuda.synchronize(self.device)
        self.set_step(self.get_step() if step is None else step)

    def update_params(self, **kw):
        for k, v in kw.items():
            setattr(self.params, k, v)
        check(self.L.bounce_update_params(self.ctx, C.byref(self.params)), self.ctx,
              "bounce_update_params")

    # -- diagnostics -------------------------------------------------------
    def gradient(self, which):
        g = self.torch.zeros_like(self.pos)
        check(self.L.bounce_compute_gradient(self.ctx, int(which), _tptr(g)), self.ctx,
              "bounce_compute_gradient")
        return g

    def energies(self):
        out = np.zeros((self.n_replicas, 7))
        check(self.L.bounce_compute_energies(self.ctx, _ptr(out)), self.ctx,
              "bounce_compute_energies")
        keys = ["bond", "angle", "coul", "lj", "pair", "kin", "tkin"]
        return [dict(zip(keys, row.tolist())) for row in out]

    def counters(self, replica=0):
        c = bounce_counters()
        check(self.L.bounce_get_counters(self.ctx, int(replica), C.byref(c)), self.ctx,
              "bounce_get_counters")
        return {k: int(getattr(c, k)) for k, _ in c._fields_}

    def events(self):
        n = C.c_int64()
        check(self.L.bounce_get_events(self.ctx, None, 0, C.byref(n)), self.ctx, "bounce_get_events")
        cap = min(n.value, self.params.event_capacity)
        buf = (bounce_event * max(cap, 1))()
        check(self.L.bounce_get_events(self.ctx, C.cast(buf, C.c_void_p), cap, C.byref(n)),
              self.ctx, "bounce_get_events")
        dt = np.dtype([("step", np.int64), ("phase", np.int32), ("atom", np.int32),
                       ("k", np.int32), ("partner", np.int32), ("accepted", np.int32),
                       ("replica", np.int32), ("mech", np.int32), ("pad", np.int32)])
        arr = np.frombuffer(bytes(buf), dtype=dt, count=max(cap, 1))[:cap].copy()
        return arr, n.value

    def get_list(self, which):
        rp = np.zeros(self.n + 1, np.int64)
        cap = 1
        col = np.zeros(cap, np.int32)
        st = self.L.bounce_get_list(self.ctx, int(which), _ptr(rp), _ptr(col), cap)
        if st != 0:
            cap = int(rp[-1])
            col = np.zeros(max(cap, 1), np.int32)
            check(self.L.bounce_get_list(self.ctx, int(which), _ptr(rp), _ptr(col), cap),
                  self.ctx, "bounce_get_list")
        return rp, col[:int(rp[-1])]

    def list_size(self, which):
        """Entries of a list set's rows (LIST_FORCE: the pair kernel's slots per launch)."""
        rp = np.zeros(self.n + 1, np.int64)
        col = np.zeros(1, np.int32)
        self.L.bounce_get_list(self.ctx, int(which), _ptr(rp), _ptr(col), 1)   # sizes only
        return int(rp[-1])

    def rate_bounds(self):
        """(L_ab [a, b] or, with separate mechanisms, [m, a, b]; L_a [a])."""
        nt, nm = self.n_types, 2 if self.params.jump_split else 1
        lab, la = np.zeros(nm * nt * nt), np.zeros(nt)
        check(self.L.bounce_rate_bounds(self.ctx, _ptr(lab), _ptr(la)), self.ctx,
              "bounce_rate_bounds")
        return (lab.reshape(nt, nt) if nm == 1 else lab.reshape(nm, nt, nt)), la

    def rate_weights(self):
        """Integer bound weights Lq[a][m n_types + b] and units unit[a] of the
        jump step: the bound of a partner of type b of an atom of type a under
        mechanism m is Lq[a][m n_types + b] * unit[a]."""
        nt, nm = self.n_types, 2 if self.params.jump_split else 1
        lq, unit = np.zeros(nt * nm * nt, np.uint32), np.zeros(nt)
        check(self.L.bounce_rate_weights(self.ctx, _ptr(lq), _ptr(unit)), self.ctx,
              "bounce_rate_weights")
        return lq.reshape(nt, nm * nt), unit

    def rdf_counts(self, r_max, n_bins):
        """Ordered non-excluded pair counts [n_types, n_types, n_bins] with r < r_max
        at the current positions (all replicas)."""
        nt = self.n_types
        out = np.zeros(nt * nt * int(n_bins), np.uint64)
        check(self.L.bounce_rdf_counts(self.ctx, float(r_max), int(n_bins), _ptr(out)), self.ctx,
              "bounce_rdf_counts")
        return out.reshape(nt, nt, int(n_bins))

    def msd(self, ref):
        """Mean squared displacement from ref (a float64 (N, 3) tensor on the device)
        per replica and atom type: array [n_replicas, n_types]."""
        ref = ref.contiguous()
        if ref.dtype != self.torch.float64 or ref.device != self.pos.device or \
                tuple(ref.shape) != tuple(self.pos.shape):
            raise ValueError("ref must be a float64 (N, 3) tensor on the simulation's device")
        out = np.zeros((len(self.offsets) - 1) * self.n_types, np.float64)
        check(self.L.bounce_msd(self.ctx, _tptr(ref), _ptr(out)), self.ctx, "bounce_msd")
        return out.reshape(-1, self.n_types)

    def pme_energy(self):
        """Mesh Ewald parts at the current positions: (E_recip, E_self, E_excl) in
        kcal/mol, the last the excluded pairs' erf(alpha r)/r correction."""
        out = np.zeros(3)
        check(self.L.bounce_pme_energy(self.ctx, _ptr(out)), self.ctx, "bounce_pme_energy")
        return out

    def jump_halfstep(self, step, phase):
        check(self.L.bounce_jump_halfstep(self.ctx, int(step), int(phase)), self.ctx,
              "bounce_jump_halfstep")

    def profile_kernel(self, which, reps):
        """Mean duration (ms) per launch, timed with HIP events on the bound stream:
        0 the F_0 pair kernel, 2 the integrator kernel with kicks, jumps and
        drifts off (both leave the trajectory unchanged), 1 the list build at
        the current positions (later steps use these lists), 3 the integrator
        kernel of `reps` real steps (advances the trajectory by reps + 1 steps),
        4 the reciprocal-space mesh sum (needs pme_grid; trajectory unchanged)."""
        ms = C.c_double()
        check(self.L.bounce_profile_kernel(self.ctx, int(which), int(reps), C.byref(ms)), self.ctx,
              "bounce_profile_kernel")
        return ms.value

    def autotune(self, reps=20):
        """Pick the pair kernel's lanes per atom by timing; returns (lanes, {lanes: ms})."""
        lanes = C.c_int32()
        ms = np.zeros(4)
        check(self.L.bounce_autotune(self.ctx, int(reps), C.byref(lanes), _ptr(ms)), self.ctx,
              "bounce_autotune")
        return lanes.value, dict(zip((4, 8, 16, 32), ms.tolist()))

    def tune(self, reps=20, cache=None):
        """Pick the pair kernel's lanes per atom and the launch structure (two
        launches or one fused launch per step) by timing, or read them from the
        JSON-lines cache file `cache` when it holds this device and
        configuration; returns the choice and the times as a dict."""
        t = _abi.bounce_tuning()
        path = None if cache is None else os.fsencode(os.fspath(cache))
        check(self.L.bounce_autotune_cached(self.ctx, int(reps), path, C.byref(t)), self.ctx,
              "bounce_autotune_cached")
        return {"pair_lanes": t.pair_lanes, "persistent": t.persistent,
                "pair_ms": dict(zip((4, 8, 16, 32), list(t.pair_ms))),
                "step_ms": {"two_launches": t.step_ms[0], "fused": t.step_ms[1]},
                "from_cache": bool(t.from_cache)}

    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            self.L.bounce_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _direct_energy_fwd(sim, pos, tparams):
    torch = sim.torch
    e = torch.zeros(1, dtype=torch.float64, device=pos.device)
    check(sim.L.bounce_direct_energy(sim.ctx, _tptr(pos), _tptr(tparams), _tptr(e)), sim.ctx,
          "bounce_direct_energy")
    return e[0]


try:
    import torch as _torch

    class DirectEnergy(_torch.autograd.Function):
        """E(q; charge, eps, sigma) = sum over non-excluded pairs within rc of the
        shifted-force Coulomb + LJ energy; backward returns dE/dq and dE/d(type params)
        from the hand-written backward kernel.  ``tparams`` = cat(charge, eps, sigma)."""

        @staticmethod
        def forward(ctx, pos, tparams, sim):
            pos = pos.detach().contiguous()
            tparams = tparams.detach().contiguous()
            ctx.save_for_backward(pos, tparams)
            ctx.sim = sim
            return _direct_energy_fwd(sim, pos, tparams)

        @staticmethod
        def backward(ctx, grad_out):
            pos, tparams = ctx.saved_tensors
            sim = ctx.sim
            go = grad_out.detach().reshape(1).to(_torch.float64).contiguous()
            gpos = _torch.empty_like(pos)
            gpar = _torch.empty_like(tparams)
            check(sim.L.bounce_direct_energy_bwd(sim.ctx, _tptr(pos), _tptr(tparams), _tptr(go),
                                                 _tptr(gpos), _tptr(gpar)), sim.ctx,
                  "bounce_direct_energy_bwd")
            return gpos, gpar, None
except ImportError:  # pragma: no cover
    DirectEnergy = None

"""ctypes marshalling of the C ABI declared in include/bounce.h.

Argument marshalling only: every computation runs in libbounce.so.  Loading
fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbounce.so")
MAX_TYPES = 8

OK, E_ARG, E_HIP, E_CAPACITY, E_SKIN, E_BOUND, E_POISSON_CAP, E_NONFINITE, E_STATE, E_GRID, \
    E_WORKSPACE = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10
BJAOAJB, BAOAB = 0, 1
PAIR_FP32, PAIR_FP64 = 0, 1
COUL_BARE, COUL_EWALD = 0, 1
PH_JA, PH_O, PH_JB = 0, 1, 2
G_BONDED, G_SHORT, G_LONG, G_FULL, G_RECIP, G_STEP = 1, 2, 4, 8, 16, 32
OUTER_RECIP, OUTER_NONBONDED = 0, 1
LIST_FORCE, LIST_CAND = 0, 1
RATE_ATOM, RATE_PAIR = 0, 1


class bounce_params(C.Structure):
    _fields_ = [("integrator", C.c_int32), ("pair_precision", C.c_int32), ("coulomb", C.c_int32),
                ("periodic", C.c_int32), ("rebuild_interval", C.c_int32),
                ("max_proposals", C.c_int32), ("log_events", C.c_int32), ("use_graph", C.c_int32),
                ("dt", C.c_double), ("gamma", C.c_double), ("temperature", C.c_double),
                ("r_on", C.c_double), ("r_off", C.c_double), ("r_cut", C.c_double),
                ("skin", C.c_double), ("ewald_alpha", C.c_double), ("bound_scale", C.c_double),
                ("cell_size", C.c_double), ("seed", C.c_uint64), ("event_capacity", C.c_int64),
                ("pair_lanes", C.c_int32), ("rate_mode", C.c_int32),
                ("pme_grid", C.c_int32 * 3), ("pme_order", C.c_int32), ("respa_m", C.c_int32),
                ("respa_outer", C.c_int32), ("jump_split", C.c_int32), ("r_on_lj", C.c_double),
                ("r_off_lj", C.c_double), ("persistent", C.c_int32), ("pair_kernel", C.c_int32)]


class bounce_system(C.Structure):
    _fields_ = [("n_replicas", C.c_int32), ("n_atoms", C.c_int32),
                ("replica_offset", C.c_void_p), ("box", C.c_void_p), ("grid_origin", C.c_void_p),
                ("grid_dims", C.c_void_p), ("type", C.c_void_p), ("mass", C.c_void_p),
                ("n_types", C.c_int32), ("charge", C.c_void_p), ("eps", C.c_void_p),
                ("sigma", C.c_void_p), ("n_bonds", C.c_int32), ("bonds", C.c_void_p),
                ("bond_k", C.c_void_p), ("bond_r0", C.c_void_p), ("n_angles", C.c_int32),
                ("angles", C.c_void_p), ("angle_k", C.c_void_p), ("angle_t0", C.c_void_p),
                ("n_excl", C.c_int32), ("excl", C.c_void_p)]


class bounce_counters(C.Structure):
    _fields_ = [("proposals", C.c_int64), ("accepted", C.c_int64),
                ("bound_violations", C.c_int64), ("rebuilds", C.c_int64), ("steps", C.c_int64)]


class bounce_event(C.Structure):
    _fields_ = [("step", C.c_int64), ("phase", C.c_int32), ("atom", C.c_int32), ("k", C.c_int32),
                ("partner", C.c_int32), ("accepted", C.c_int32), ("replica", C.c_int32),
                ("mech", C.c_int32), ("pad", C.c_int32)]


_P = C.POINTER
vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
ctx_p = C.c_void_p

# name -> (restype, argtypes); one entry per function of include/bounce.h
class bounce_tuning(C.Structure):
    _fields_ = [("pair_lanes", C.c_int32), ("persistent", C.c_int32), ("pair_ms", C.c_double * 4),
                ("step_ms", C.c_double * 2), ("from_cache", C.c_int32), ("pad", C.c_int32)]


SIGNATURES = {
    "bounce_create": (i32, [_P(bounce_params), _P(ctx_p)]),
    "bounce_destroy": (None, [ctx_p]),
    "bounce_update_params": (i32, [ctx_p, _P(bounce_params)]),
    "bounce_set_system": (i32, [ctx_p, _P(bounce_system)]),
    "bounce_workspace_size": (i32, [ctx_p, _P(u64)]),
    "bounce_bind": (i32, [ctx_p, vp, u64, vp, vp, vp]),
    "bounce_bind_static": (i32, [ctx_p, vp, vp, vp]),
    "bounce_set_step": (i32, [ctx_p, i64]),
    "bounce_get_step": (i32, [ctx_p, _P(i64)]),
    "bounce_step": (i32, [ctx_p, i32]),
    "bounce_sync": (i32, [ctx_p]),
    "bounce_compute_gradient": (i32, [ctx_p, i32, vp]),
    "bounce_compute_energies": (i32, [ctx_p, vp]),
    "bounce_get_counters": (i32, [ctx_p, i32, _P(bounce_counters)]),
    "bounce_get_events": (i32, [ctx_p, vp, i64, _P(i64)]),
    "bounce_get_list": (i32, [ctx_p, i32, vp, vp, i64]),
    "bounce_rate_bounds": (i32, [ctx_p, vp, vp]),
    "bounce_rate_weights": (i32, [ctx_p, vp, vp]),
    "bounce_rdf_counts": (i32, [ctx_p, C.c_double, i32, vp]),
    "bounce_msd": (i32, [ctx_p, vp, vp]),
    "bounce_pme_energy": (i32, [ctx_p, vp]),
    "bounce_jump_halfstep": (i32, [ctx_p, i64, i32]),
    "bounce_direct_energy": (i32, [ctx_p, vp, vp, vp]),
    "bounce_direct_energy_bwd": (i32, [ctx_p, vp, vp, vp, vp, vp]),
    "bounce_profile_kernel": (i32, [ctx_p, i32, i32, _P(C.c_double)]),
    "bounce_autotune": (i32, [ctx_p, i32, _P(i32), vp]),
    "bounce_autotune_cached": (i32, [ctx_p, i32, C.c_char_p, _P(bounce_tuning)]),
    "bounce_status_string": (C.c_char_p, [i32]),
    "bounce_last_error": (C.c_char_p, [ctx_p]),
}

_lib = None


def load(path: str | None = None):
    """Load libbounce.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"libbounce.so not built ({p}); run paper_2002_07109_amd/build.py or "
                          "__graft_entry__.build()")
    L = C.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = L
    return L


class BounceError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def check(status, ctx=None, what=""):
    if status != OK:
        L = load()
        detail = L.bounce_last_error(ctx).decode() if ctx else L.bounce_status_string(status).decode()
        raise BounceError(status, f"{what}: {detail}")
    return status

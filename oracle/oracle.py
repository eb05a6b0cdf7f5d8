"""ctypes front-end of the FP64 CPU oracle (test infrastructure only).

Only the test-suite, the entry module's smoke check and the benchmark's CPU
baseline import this module.  It compiles ``bounce_oracle.c`` with gcc on
first use (or when :func:`build` is called) into ``oracle/liborc.so``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bounce_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

MAXT = 8
BOUNCE, BAOAB = 0, 1
COUL_BARE, COUL_EWALD = 0, 1
PH_JA, PH_O, PH_JB = 0, 1, 2
RATE_ATOM, RATE_PAIR = 0, 1
WEIGHT_BITS = 20
G_BONDED, G_SHORT, G_LONG, G_FULL, G_RECIP = 1, 2, 4, 8, 16
OUTER_RECIP, OUTER_NONBONDED = 0, 1
STATUS = {0: "OK", -1: "ARG", -4: "SKIN", -5: "BOUND", -6: "POISSON_CAP", -7: "NONFINITE",
          -9: "GRID"}
KE, KB, ACC = 332.0637, 0.0019872041, 4.184e-4


def build(force=True):
    """Compile the oracle (plain C, -O2, no fast-math, no FMA contraction)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [("integrator", C.c_int32), ("coulomb", C.c_int32), ("periodic", C.c_int32),
                ("n_types", C.c_int32), ("rebuild_interval", C.c_int32),
                ("max_proposals", C.c_int32),
                ("dt", C.c_double), ("gamma", C.c_double), ("temperature", C.c_double),
                ("r_on", C.c_double), ("r_off", C.c_double), ("r_cut", C.c_double),
                ("skin", C.c_double), ("ewald_alpha", C.c_double), ("bound_scale", C.c_double),
                ("box", C.c_double * 3), ("cell_size", C.c_double),
                ("grid_origin", C.c_double * 3), ("grid_dims", C.c_int32 * 3),
                ("rate_mode", C.c_int32), ("seed", C.c_uint64), ("replica", C.c_uint64),
                ("charge", C.c_double * MAXT), ("eps", C.c_double * MAXT),
                ("sigma", C.c_double * MAXT), ("pme_grid", C.c_int32 * 3), ("pme_order", C.c_int32),
                ("respa_m", C.c_int32), ("respa_outer", C.c_int32), ("jump_split", C.c_int32),
                ("r_on_lj", C.c_double), ("r_off_lj", C.c_double)]


class Topo(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("n_bonds", C.c_int32), ("n_angles", C.c_int32),
                ("n_excl", C.c_int32), ("type", C.c_void_p), ("mass", C.c_void_p),
                ("bonds", C.c_void_p), ("bond_k", C.c_void_p), ("bond_r0", C.c_void_p),
                ("angles", C.c_void_p), ("angle_k", C.c_void_p), ("angle_t0", C.c_void_p),
                ("excl", C.c_void_p)]


class Counters(C.Structure):
    _fields_ = [("proposals", C.c_int64), ("accepted", C.c_int64),
                ("bound_violations", C.c_int64), ("rebuilds", C.c_int64),
                ("pair_evals", C.c_int64), ("steps", C.c_int64), ("list_seconds", C.c_double)]

    def as_dict(self):
        """The event and step counts (the list-build wall time is returned apart)."""
        return {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "list_seconds"}


EVENT_DTYPE = np.dtype([("step", np.int64), ("phase", np.int32), ("atom", np.int32),
                        ("k", np.int32), ("partner", np.int32), ("accepted", np.int32),
                        ("mech", np.int32), ("margin", np.float64), ("scale", np.float64)])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P, T = C.POINTER(Params), C.POINTER(Topo)
        vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
        L.orc_philox4x64_10.argtypes = [vp, vp, vp]
        L.orc_u01.argtypes = [u64]; L.orc_u01.restype = C.c_double
        L.orc_umulh.argtypes = [u64, u64]; L.orc_umulh.restype = u64
        L.orc_pair_u.argtypes = [P, C.c_int, C.c_int, C.c_double, vp, vp]
        L.orc_pair_wsf.argtypes = [P, C.c_int, C.c_int, C.c_double, vp, vp]
        L.orc_chi.argtypes = [P, C.c_double]; L.orc_chi.restype = C.c_double
        L.orc_rate_bounds.argtypes = [P, vp, vp]
        L.orc_rate_weights.argtypes = [P, vp, vp]
        L.orc_reflect.argtypes = [vp, vp, vp]
        L.orc_sort_order.argtypes = [P, i32, vp, vp, vp]; L.orc_sort_order.restype = C.c_int
        L.orc_build_list.argtypes = [P, T, vp, C.c_double, C.c_double, vp, vp, vp, i64]
        L.orc_build_list.restype = i64
        L.orc_list_row.argtypes = [P, T, vp, C.c_double, C.c_double, vp, i32, vp, i32]
        L.orc_list_row.restype = i32
        L.orc_gradient.argtypes = [P, T, vp, C.c_int, vp]
        L.orc_gradient_atom.argtypes = [P, T, vp, C.c_int, i32, vp]
        L.orc_energies.argtypes = [P, T, vp, vp, vp]
        L.orc_jump_halfstep.argtypes = [P, T, vp, vp, vp, vp, i64, i32, vp, i64, vp,
                                        C.POINTER(Counters)]
        L.orc_jump_halfstep.restype = C.c_int
        L.orc_run.argtypes = [P, T, vp, vp, i64, i32, vp, i64, vp, C.POINTER(Counters)]
        L.orc_run.restype = C.c_int
        L.orc_rdf_counts.argtypes = [P, T, vp, C.c_double, i32, vp]
        L.orc_pme.argtypes = [P, T, vp, vp, vp]
        L.orc_ewald_recip.argtypes = [P, T, vp, i32, vp]
        L.orc_ewald_recip.restype = C.c_double
        L.orc_direct_energy.argtypes = [P, T, vp, vp, vp, vp, vp]
        L.orc_direct_energy.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def make_params(sys=None, *, integrator=BOUNCE, coulomb=None, dt=1.0, gamma=1e-3,
                temperature=300.0, r_on=5.0, r_off=6.0, r_cut=9.0, skin=2.0, ewald_alpha=0.35,
                rebuild_interval=10, seed=0, replica=0, bound_scale=1.0, max_proposals=100000,
                charge=None, eps=None, sigma=None, periodic=None, box=None, cell_size=None,
                grid_origin=None, grid_dims=None, rate_mode=RATE_ATOM, pme_grid=None, pme_order=5,
                respa_m=0, respa_outer=0, jump_split=0, r_on_lj=None, r_off_lj=None):
    """Parameters for the oracle; geometry defaults are taken from a WaterSystem."""
    p = Params()
    p.integrator = integrator
    if periodic is None:
        periodic = bool(sys.periodic) if sys is not None else False
    p.periodic = int(periodic)
    if coulomb is None:
        coulomb = COUL_EWALD if periodic else COUL_BARE
    p.coulomb = coulomb
    p.dt, p.gamma, p.temperature = dt, gamma, temperature
    p.r_on, p.r_off, p.r_cut, p.skin = r_on, r_off, r_cut, skin
    p.ewald_alpha, p.bound_scale = ewald_alpha, bound_scale
    p.rebuild_interval, p.max_proposals = rebuild_interval, max_proposals
    p.seed, p.replica = seed, replica
    p.rate_mode = rate_mode
    for k in range(3):
        p.pme_grid[k] = int(pme_grid[k]) if pme_grid is not None else 0
    p.pme_order, p.respa_m, p.respa_outer = int(pme_order), int(respa_m), int(respa_outer)
    # separate Coulomb and Lennard-Jones jump mechanisms; the LJ switch window
    # defaults to the Coulomb one
    p.jump_split = int(jump_split)
    p.r_on_lj = r_on if r_on_lj is None else r_on_lj
    p.r_off_lj = r_off if r_off_lj is None else r_off_lj
    if sys is not None:
        from workloads import tip3p_params
        ff = tip3p_params()
        charge = ff["charge"] if charge is None else charge
        eps = ff["eps"] if eps is None else eps
        sigma = ff["sigma"] if sigma is None else sigma
        box = sys.box if box is None else box
        cell_size = sys.cell_size if cell_size is None else cell_size
        grid_origin = sys.grid_origin if grid_origin is None else grid_origin
        grid_dims = sys.grid_dims if grid_dims is None else grid_dims
    nt = len(charge)
    p.n_types = nt
    for a in range(nt):
        p.charge[a], p.eps[a], p.sigma[a] = charge[a], eps[a], sigma[a]
    for k in range(3):
        p.box[k] = float(box[k]) if box is not None else 0.0
        p.grid_origin[k] = float(grid_origin[k]) if grid_origin is not None else 0.0
        p.grid_dims[k] = int(grid_dims[k]) if grid_dims is not None else 0
    p.cell_size = float(cell_size) if cell_size is not None else 4.4
    return p


class Topology:
    """Keeps the numpy arrays alive behind the ctypes struct."""

    def __init__(self, atom_type, mass, bonds=None, bond_k=None, bond_r0=None, angles=None,
                 angle_k=None, angle_t0=None, excl=None):
        z2 = np.zeros((0, 2), np.int32)
        self.type = np.ascontiguousarray(atom_type, np.int32)
        self.mass = np.ascontiguousarray(mass, np.float64)
        self.bonds = np.ascontiguousarray(bonds if bonds is not None else z2, np.int32)
        self.bond_k = np.ascontiguousarray(bond_k if bond_k is not None else [], np.float64)
        self.bond_r0 = np.ascontiguousarray(bond_r0 if bond_r0 is not None else [], np.float64)
        self.angles = np.ascontiguousarray(angles if angles is not None else np.zeros((0, 3)),
                                           np.int32)
        self.angle_k = np.ascontiguousarray(angle_k if angle_k is not None else [], np.float64)
        self.angle_t0 = np.ascontiguousarray(angle_t0 if angle_t0 is not None else [], np.float64)
        self.excl = np.ascontiguousarray(excl if excl is not None else z2, np.int32)
        t = Topo()
        t.n_atoms = self.type.shape[0]
        t.n_bonds, t.n_angles, t.n_excl = self.bonds.shape[0], self.angles.shape[0], self.excl.shape[0]
        for name in ("type", "mass", "bonds", "bond_k", "bond_r0", "angles", "angle_k",
                     "angle_t0", "excl"):
            setattr(t, name, getattr(self, name).ctypes.data)
        self.c = t

    @classmethod
    def from_system(cls, s):
        return cls(s.atom_type, s.mass, s.bonds, s.bond_k, s.bond_r0, s.angles, s.angle_k,
                   s.angle_t0, s.excl)

    @property
    def n(self):
        return int(self.type.shape[0])


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint64)
    k = np.ascontiguousarray(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def u01(w):
    return lib().orc_u01(int(w))


def umulh(a, b):
    return int(lib().orc_umulh(int(a), int(b)))


def pair_u(p, a, b, r):
    u, du = C.c_double(), C.c_double()
    lib().orc_pair_u(C.byref(p), a, b, r, C.byref(u), C.byref(du))
    return u.value, du.value


def pair_wsf(p, a, b, r):
    w, dw = C.c_double(), C.c_double()
    lib().orc_pair_wsf(C.byref(p), a, b, r, C.byref(w), C.byref(dw))
    return w.value, dw.value


def chi(p, r):
    return lib().orc_chi(C.byref(p), r)


def rate_bounds(p):
    """(L_ab, L_a): L_ab[a, b] ([m, a, b] with separate mechanisms) and L_a."""
    nt, nm = p.n_types, 2 if p.jump_split else 1
    L_ab = np.zeros(nm * nt * nt)
    L_a = np.zeros(nt)
    lib().orc_rate_bounds(C.byref(p), _ptr(L_ab), _ptr(L_a))
    return (L_ab.reshape(nt, nt) if nm == 1 else L_ab.reshape(nm, nt, nt)), L_a


def rate_weights(p):
    """(Lq, unit): Lq[a, m n_types + b], unit[a]."""
    nt, nm = p.n_types, 2 if p.jump_split else 1
    Lq = np.zeros(nt * nm * nt, np.uint32)
    unit = np.zeros(nt)
    lib().orc_rate_weights(C.byref(p), _ptr(Lq), _ptr(unit))
    return Lq.reshape(nt, nm * nt), unit


def reflect(v, F):
    v = np.ascontiguousarray(v, np.float64)
    F = np.ascontiguousarray(F, np.float64)
    out = np.zeros(3)
    lib().orc_reflect(_ptr(v), _ptr(F), _ptr(out))
    return out


def sort_order(p, q):
    q = np.ascontiguousarray(q, np.float64)
    n = q.shape[0]
    order = np.zeros(n, np.int32)
    cell = np.zeros(n, np.int64)
    st = lib().orc_sort_order(C.byref(p), n, _ptr(q), _ptr(order), _ptr(cell))
    if st != 0:
        raise RuntimeError("oracle sort_order: " + STATUS.get(st, str(st)))
    return order, cell


def build_list(p, topo, q, rmin, rmax, order=None):
    q = np.ascontiguousarray(q, np.float64)
    if order is None:
        order, _ = sort_order(p, q)
    n = topo.n
    row_ptr = np.zeros(n + 1, np.int64)
    total = lib().orc_build_list(C.byref(p), C.byref(topo.c), _ptr(q), rmin, rmax, _ptr(order),
                                 _ptr(row_ptr), None, 0)
    total = int(row_ptr[-1])
    col = np.zeros(max(total, 1), np.int32)
    lib().orc_build_list(C.byref(p), C.byref(topo.c), _ptr(q), rmin, rmax, _ptr(order),
                         _ptr(row_ptr), _ptr(col), total)
    return row_ptr, col[:total]


def list_row(p, topo, q, rmin, rmax, order, i, cap=4096):
    q = np.ascontiguousarray(q, np.float64)
    col = np.zeros(cap, np.int32)
    m = lib().orc_list_row(C.byref(p), C.byref(topo.c), _ptr(q), rmin, rmax, _ptr(order),
                           int(i), _ptr(col), cap)
    if m > cap:
        return list_row(p, topo, q, rmin, rmax, order, i, cap=m)
    return col[:m].copy()


def gradient(p, topo, q, which):
    q = np.ascontiguousarray(q, np.float64)
    g = np.zeros_like(q)
    lib().orc_gradient(C.byref(p), C.byref(topo.c), _ptr(q), which, _ptr(g))
    return g


def gradient_atom(p, topo, q, which, i):
    q = np.ascontiguousarray(q, np.float64)
    g = np.zeros(3)
    lib().orc_gradient_atom(C.byref(p), C.byref(topo.c), _ptr(q), which, int(i), _ptr(g))
    return g


def energies(p, topo, q, v):
    q = np.ascontiguousarray(q, np.float64)
    v = np.ascontiguousarray(v, np.float64)
    out = np.zeros(7)
    lib().orc_energies(C.byref(p), C.byref(topo.c), _ptr(q), _ptr(v), _ptr(out))
    return dict(zip(["bond", "angle", "coul", "lj", "pair", "kin", "tkin"], out.tolist()))


def jump_halfstep(p, topo, q, v, row_ptr, col, step, phase, ev_cap=0):
    q = np.ascontiguousarray(q, np.float64)
    v = np.array(v, np.float64, copy=True, order="C")
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col = np.ascontiguousarray(col if len(col) else np.zeros(1, np.int32), np.int32)
    ev = np.zeros(max(ev_cap, 1), EVENT_DTYPE)
    nev = C.c_int64(0)
    cnt = Counters()
    st = lib().orc_jump_halfstep(C.byref(p), C.byref(topo.c), _ptr(q), _ptr(v), _ptr(row_ptr),
                                 _ptr(col), int(step), int(phase),
                                 _ptr(ev) if ev_cap else None, ev_cap, C.byref(nev),
                                 C.byref(cnt))
    return dict(v=v, status=st, counters=cnt.as_dict(),
                events=ev[:min(nev.value, ev_cap)] if ev_cap else None)


def run(p, topo, q, v, step0, nsteps, ev_cap=0):
    q = np.array(q, np.float64, copy=True, order="C")
    v = np.array(v, np.float64, copy=True, order="C")
    ev = np.zeros(max(ev_cap, 1), EVENT_DTYPE)
    nev = C.c_int64(0)
    cnt = Counters()
    st = lib().orc_run(C.byref(p), C.byref(topo.c), _ptr(q), _ptr(v), int(step0), int(nsteps),
                       _ptr(ev) if ev_cap else None, ev_cap, C.byref(nev), C.byref(cnt))
    return dict(q=q, v=v, status=st, status_name=STATUS.get(st, str(st)),
                counters=cnt.as_dict(), list_seconds=float(cnt.list_seconds), n_events=nev.value,
                events=ev[:min(nev.value, ev_cap)] if ev_cap else None)


def rdf_counts(p, topo, q, r_max, nbins):
    """Ordered non-excluded pair counts [n_types, n_types, nbins] with r < r_max."""
    q = np.ascontiguousarray(q, np.float64)
    nt = p.n_types
    counts = np.zeros(nt * nt * nbins, np.int64)
    lib().orc_rdf_counts(C.byref(p), C.byref(topo.c), _ptr(q), float(r_max), int(nbins),
                         _ptr(counts))
    return counts.reshape(nt, nt, nbins)


def pme(p, topo, q, grad=True):
    """Smooth-PME reciprocal part: ((E_rec, E_self, E_excl), gradient of E_rec + E_excl)."""
    q = np.ascontiguousarray(q, np.float64)
    g = np.zeros_like(q) if grad else None
    e = np.zeros(3)
    lib().orc_pme(C.byref(p), C.byref(topo.c), _ptr(q), _ptr(g), _ptr(e))
    return tuple(e.tolist()), g


def ewald_recip(p, topo, q, kmax, grad=True):
    """Plain reciprocal Ewald sum over |k_a| <= kmax: (E_rec, gradient)."""
    q = np.ascontiguousarray(q, np.float64)
    g = np.zeros_like(q) if grad else None
    E = lib().orc_ewald_recip(C.byref(p), C.byref(topo.c), _ptr(q), int(kmax), _ptr(g))
    return E, g


def direct_energy(p, topo, q, grads=True):
    q = np.ascontiguousarray(q, np.float64)
    nt = p.n_types
    gq = np.zeros_like(q) if grads else None
    gc, ge, gs = (np.zeros(nt), np.zeros(nt), np.zeros(nt)) if grads else (None, None, None)
    E = lib().orc_direct_energy(C.byref(p), C.byref(topo.c), _ptr(q), _ptr(gq), _ptr(gc),
                                _ptr(ge), _ptr(gs))
    return (E, gq, gc, ge, gs) if grads else E

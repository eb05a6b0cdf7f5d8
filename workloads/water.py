"""Synthetic flexible 3-site water systems.

The paper's own systems (TIP3P/SPC water boxes and droplets, solvated proteins)
are not available, so every workload is generated here from a seed: waters sit
on a simple-cubic lattice whose spacing gives 1 g/cm^3, each with a uniformly
random orientation (re-drawn until no intermolecular contact is closer than a
clash threshold), and velocities are Maxwell-Boltzmann at the target
temperature.  Droplets keep the waters nearest to the lattice centre.

Units: Angstrom, fs, amu, kcal/mol, elementary charge.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

KB_KCAL = 0.0019872041          # Boltzmann constant, kcal/(mol K)
ACC_CONV = 4.184e-4             # (kcal/mol/Angstrom)/amu -> Angstrom/fs^2

# Flexible TIP3P-like water: O type 0, H type 1.
O_MASS, H_MASS = 15.999, 1.008
OH_BOND, HOH_ANGLE_DEG = 0.9572, 104.52
BOND_K, ANGLE_K = 450.0, 55.0   # k in E = k (x - x0)^2
WATER_SPACING = 3.1             # lattice spacing giving ~1 g/cm^3


def tip3p_params():
    """Per-type nonbonded parameters: charge (e), epsilon (kcal/mol), sigma (A)."""
    return dict(charge=np.array([-0.834, 0.417]),
                eps=np.array([0.152, 0.0]),
                sigma=np.array([3.15, 0.0]),
                mass=np.array([O_MASS, H_MASS]))


@dataclasses.dataclass
class WaterSystem:
    pos: np.ndarray            # (N,3) float64
    vel: np.ndarray            # (N,3) float64
    atom_type: np.ndarray      # (N,) int32
    mass: np.ndarray           # (N,) float64
    bonds: np.ndarray          # (nb,2) int32
    bond_k: np.ndarray
    bond_r0: np.ndarray
    angles: np.ndarray         # (na,3) int32, vertex in the middle
    angle_k: np.ndarray
    angle_t0: np.ndarray
    excl: np.ndarray           # (ne,2) int32 excluded nonbonded pairs
    periodic: bool
    box: np.ndarray            # (3,) float64 (periodic) else zeros
    grid_origin: np.ndarray    # droplet cell-grid origin (3,)
    grid_dims: np.ndarray      # droplet cell-grid dims (3,) int32
    cell_size: float
    n_types: int = 2

    @property
    def n_atoms(self):
        return int(self.pos.shape[0])


def _rng(seed, stream):
    return np.random.Generator(np.random.Philox(key=[int(seed) & (2**64 - 1), int(stream)]))


def _random_rotations(rng, n):
    qv = rng.standard_normal((n, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - z * w); R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w); R[:, 2, 1] = 2 * (y * z + x * w); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _water_frame():
    half = math.radians(HOH_ANGLE_DEG) / 2
    return np.array([[0.0, 0.0, 0.0],
                     [OH_BOND * math.sin(half), OH_BOND * math.cos(half), 0.0],
                     [-OH_BOND * math.sin(half), OH_BOND * math.cos(half), 0.0]])


def _place_waters(sites, rng, box=None, clash=1.7, max_tries=200):
    """Put one water on each site with a random orientation avoiding H clashes
    with the waters already placed on neighbouring sites."""
    n = sites.shape[0]
    frame = _water_frame()
    out = np.empty((n, 3, 3))
    reach = 2.5 * WATER_SPACING
    # coarse bins of the sites to find neighbouring sites quickly
    key = np.floor(sites / reach).astype(np.int64)
    bins = {}
    for m in range(n):
        bins.setdefault(tuple(key[m]), []).append(m)
    nbin = None
    if box is not None:
        nbin = np.maximum(1, np.floor(box / reach).astype(np.int64))
        key = np.floor((sites % box) / (box / nbin)).astype(np.int64) % nbin
        bins = {}
        for m in range(n):
            bins.setdefault(tuple(key[m]), []).append(m)
    offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    c2 = clash * clash
    for m in range(n):
        kk = key[m]
        near = set()
        for o in offs:
            t = kk + np.array(o)
            if nbin is not None:
                t = t % nbin
            near.update(bins.get(tuple(t), ()))
        prev = np.array(sorted(x for x in near if x < m), dtype=np.int64)
        for _ in range(max_tries):
            R = _random_rotations(rng, 1)[0]
            xyz = sites[m] + frame @ R.T
            if prev.size == 0:
                break
            others = out[prev]                                  # (p,3,3)
            d = xyz[1:, None, :] - others.reshape(-1, 3)[None]  # our H vs all their atoms
            d_o = xyz[0][None, :] - others[:, 1:, :].reshape(-1, 3)  # our O vs their H
            if box is not None:
                d -= box * np.rint(d / box)
                d_o -= box * np.rint(d_o / box)
            if (np.einsum("ijk,ijk->ij", d, d).min() > c2
                    and np.einsum("ij,ij->i", d_o, d_o).min() > c2):
                break
        out[m] = xyz
    return out.reshape(-1, 3)


def _topology(n_waters):
    base = 3 * np.arange(n_waters, dtype=np.int32)
    atom_type = np.tile(np.array([0, 1, 1], dtype=np.int32), n_waters)
    mass = np.tile(np.array([O_MASS, H_MASS, H_MASS]), n_waters)
    bonds = np.concatenate([np.stack([base, base + 1], 1), np.stack([base, base + 2], 1)])
    bonds = bonds[np.argsort(bonds[:, 0], kind="stable")]
    angles = np.stack([base + 1, base, base + 2], 1).astype(np.int32)
    excl = np.concatenate([np.stack([base, base + 1], 1), np.stack([base, base + 2], 1),
                           np.stack([base + 1, base + 2], 1)])
    excl = excl[np.lexsort((excl[:, 1], excl[:, 0]))].astype(np.int32)
    nb, na = bonds.shape[0], angles.shape[0]
    return dict(atom_type=atom_type, mass=mass, bonds=bonds.astype(np.int32),
                bond_k=np.full(nb, BOND_K), bond_r0=np.full(nb, OH_BOND),
                angles=angles, angle_k=np.full(na, ANGLE_K),
                angle_t0=np.full(na, math.radians(HOH_ANGLE_DEG)), excl=excl)


def maxwell_velocities(mass, temperature, seed, stream=3):
    rng = _rng(seed, stream)
    sd = np.sqrt(KB_KCAL * temperature / mass * ACC_CONV)
    return rng.standard_normal((mass.shape[0], 3)) * sd[:, None]


def water_box(n_side=20, box_len=62.0, temperature=300.0, seed=0, cell_size=3.8, remove=0):
    """Periodic cube of n_side^3 waters on a lattice (the 24,000-atom box is n_side=20);
    remove > 0 drops that many lattice sites, chosen by a Philox stream of their
    own (the 96,000-atom box is n_side=32, 98 A, remove=768)."""
    rng = _rng(seed, 4)
    spacing = box_len / n_side
    g = (np.arange(n_side) + 0.5) * spacing
    sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    if remove > 0:
        drop = _rng(seed, 7).permutation(sites.shape[0])[:int(remove)]
        sites = np.delete(sites, drop, axis=0)
    box = np.full(3, float(box_len))
    pos = _place_waters(sites, rng, box=box)
    topo = _topology(sites.shape[0])
    vel = maxwell_velocities(topo["mass"], temperature, seed)
    return WaterSystem(pos=pos, vel=vel, periodic=True, box=box,
                       grid_origin=np.zeros(3), grid_dims=np.zeros(3, np.int32),
                       cell_size=cell_size, **topo)


def _droplet_sites(n_waters, spacing=WATER_SPACING, lattice=20):
    g = (np.arange(lattice) - (lattice - 1) / 2.0) * spacing
    sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    r2 = np.einsum("ij,ij->i", sites, sites)
    order = np.lexsort((np.arange(sites.shape[0]), r2))
    return sites[order[:n_waters]]


def droplet_grid(pos, cell_size, margin=12.0):
    lo = pos.min(0) - margin
    hi = pos.max(0) + margin
    dims = np.ceil((hi - lo) / cell_size).astype(np.int32)
    return lo, dims


def water_droplet(n_waters=216, temperature=300.0, seed=0, cell_size=3.8, stream=5):
    """Non-periodic droplet of the n_waters lattice waters nearest the centre
    (216 waters = the 648-atom droplet)."""
    rng = _rng(seed, stream)
    sites = _droplet_sites(n_waters)
    pos = _place_waters(sites, rng, box=None)
    topo = _topology(n_waters)
    vel = maxwell_velocities(topo["mass"], temperature, seed, stream=3 + 16 * stream)
    origin, dims = droplet_grid(pos, cell_size)
    return WaterSystem(pos=pos, vel=vel, periodic=False, box=np.zeros(3),
                       grid_origin=origin, grid_dims=dims, cell_size=cell_size, **topo)


def droplet_batch(n_replicas=64, min_atoms=300, max_atoms=6000, temperature=300.0, seed=0,
                  cell_size=3.8):
    """Uneven droplets: atom counts uniform in [min_atoms, max_atoms], rounded to whole waters."""
    rng = _rng(seed, 0xC2)
    n_atoms = rng.integers(min_atoms, max_atoms + 1, size=n_replicas)
    n_waters = np.maximum(1, np.rint(n_atoms / 3).astype(int))
    return [water_droplet(int(nw), temperature, seed, cell_size, stream=100 + r)
            for r, nw in enumerate(n_waters)]


def jitter_positions(pos, sigma, seed):
    rng = _rng(seed, 7)
    return pos + sigma * rng.standard_normal(pos.shape)

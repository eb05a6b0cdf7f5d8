"""Write tests/golden/relaxed_droplets.npz: seeded droplets and a small periodic
box relaxed by the FP64 oracle (BAOAB, dt 0.5 fs, gamma 0.05/fs) so that short parity runs
start near 300 K instead of from the hot random-orientation lattice; and
tests/golden/relaxed_box24k.npz, the 24,000-atom benchmark box (20^3 waters,
62 A, seed 0) relaxed the same way (`python make_fixtures.py box24k`).  Calls
only oracle/ and workloads/."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from workloads import water_box, water_droplet  # noqa: E402

# (name, n_waters, seed, stream) of every relaxed droplet
DROPLETS = [("c0", 216, 0, 5), ("r0", 40, 3, 200), ("r1", 150, 3, 201), ("r2", 90, 3, 202)]
# (name, waters per edge, box edge, seed) of every relaxed periodic box
BOXES = [("b8", 8, 24.8, 1)]


def relax(sys_, steps=3000):
    coul = orc.COUL_EWALD if sys_.periodic else orc.COUL_BARE
    p = orc.make_params(sys_, integrator=orc.BAOAB, coulomb=coul, dt=0.5, gamma=0.05,
                        r_cut=9.0, skin=2.0, rebuild_interval=10, seed=777, ewald_alpha=0.45)
    o = orc.run(p, orc.Topology.from_system(sys_), sys_.pos, sys_.vel, 0, steps)
    assert o["status"] == 0, o["status_name"]
    return o["q"], o["v"]


def main_box24k():
    s = water_box(n_side=20, box_len=62.0, seed=0)
    q, v = relax(s, steps=1500)
    np.savez_compressed(os.path.join(HERE, "relaxed_box24k.npz"), pos=q, vel=v)
    print("24,000-atom box relaxed")


def main():
    out = {}
    for name, nw, seed, stream in DROPLETS:
        s = water_droplet(n_waters=nw, seed=seed, stream=stream, cell_size=4.4)
        q, v = relax(s)
        out[name + "_pos"], out[name + "_vel"] = q, v
        print(name, nw, "waters relaxed")
    for name, n_side, edge, seed in BOXES:
        s = water_box(n_side=n_side, box_len=edge, seed=seed, cell_size=4.4)
        q, v = relax(s, steps=2000)
        out[name + "_pos"], out[name + "_vel"] = q, v
        print(name, n_side ** 3, "waters relaxed")
    np.savez_compressed(os.path.join(HERE, "relaxed_droplets.npz"), **out)


if __name__ == "__main__":
    if sys.argv[1:] == ["box24k"]:
        main_box24k()
    else:
        main()

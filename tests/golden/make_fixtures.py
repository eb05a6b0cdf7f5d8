"""Write tests/golden/relaxed_droplets.npz: seeded droplets relaxed by the FP64
oracle (BAOAB, dt 0.5 fs, gamma 0.05/fs, 3000 steps) so that short parity runs
start near 300 K instead of from the hot random-orientation lattice.  Calls only
oracle/ and workloads/."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from workloads import water_droplet  # noqa: E402

# (name, n_waters, seed, stream) of every relaxed droplet
DROPLETS = [("c0", 216, 0, 5), ("r0", 40, 3, 200), ("r1", 150, 3, 201), ("r2", 90, 3, 202)]


def relax(sys_, steps=3000):
    p = orc.make_params(sys_, integrator=orc.BAOAB, coulomb=orc.COUL_BARE, dt=0.5, gamma=0.05,
                        r_cut=9.0, skin=2.0, rebuild_interval=10, seed=777)
    o = orc.run(p, orc.Topology.from_system(sys_), sys_.pos, sys_.vel, 0, steps)
    assert o["status"] == 0, o["status_name"]
    return o["q"], o["v"]


def main():
    out = {}
    for name, nw, seed, stream in DROPLETS:
        s = water_droplet(n_waters=nw, seed=seed, stream=stream)
        q, v = relax(s)
        out[name + "_pos"], out[name + "_vel"] = q, v
        print(name, nw, "waters relaxed")
    np.savez_compressed(os.path.join(HERE, "relaxed_droplets.npz"), **out)


if __name__ == "__main__":
    main()

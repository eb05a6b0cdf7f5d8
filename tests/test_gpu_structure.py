"""Structure and diffusion diagnostics through the C ABI against the oracle:
pair-distance histograms bit for bit (periodic box, droplet, uneven replicas)
and mean squared displacements against their definition."""
import numpy as np
import pytest

from helpers import BOX, DROPLET, gpu_sim, oracle_params, relaxed_box, relaxed_droplet

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which", ["drop", "box"])
def test_rdf_counts_bit_exact(orc, which):
    sys, cfg = (relaxed_droplet("c0"), DROPLET) if which == "drop" else (relaxed_box("b8"), BOX)
    sim = gpu_sim(sys, cfg)
    sim.step(20)
    sim.sync()
    pos = sim.pos.cpu().numpy()
    p = oracle_params(orc, sys, cfg)
    for r_max, nbins in ((8.0, 160), (9.0, 7), (3.5, 1000)):
        g = sim.rdf_counts(r_max, nbins)
        o = orc.rdf_counts(p, orc.Topology.from_system(sys), pos, r_max, nbins)
        assert np.array_equal(g.astype(np.int64), o), (r_max, nbins)
    assert g.sum() > 0


def test_rdf_counts_replicas(orc):
    systems = [relaxed_droplet(name) for name in ("r0", "r1", "r2")]
    sim = gpu_sim(systems, DROPLET)
    g = sim.rdf_counts(8.0, 64).astype(np.int64)
    o = sum(orc.rdf_counts(oracle_params(orc, s, DROPLET, replica=r), orc.Topology.from_system(s),
                           s.pos, 8.0, 64) for r, s in enumerate(systems))
    assert np.array_equal(g, o)


def test_rdf_rejects_bad_ranges():
    import paper_2002_07109_amd as B
    sim = gpu_sim(relaxed_droplet("c0"), DROPLET)
    for r_max, nbins in ((0.0, 10), (9.5, 10), (8.0, 3000)):
        with pytest.raises(B.BounceError):
            sim.rdf_counts(r_max, nbins)


def test_msd_matches_definition():
    systems = [relaxed_droplet(name) for name in ("r0", "r1")]
    sim = gpu_sim(systems, DROPLET)
    ref = sim.pos.clone()
    sim.step(40)
    sim.sync()
    m = sim.msd(ref)
    d2 = ((sim.pos - ref) ** 2).sum(1).cpu().numpy()
    types = np.concatenate([s.atom_type for s in systems])
    for r in range(2):
        b, e = sim.offsets[r], sim.offsets[r + 1]
        for a in range(2):
            sel = types[b:e] == a
            assert m[r, a] == pytest.approx(d2[b:e][sel].mean(), rel=1e-12)
    assert np.all(m > 0)

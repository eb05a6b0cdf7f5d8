"""Pins of the oracle's pair-structure histogram (the radial-distribution
diagnostic): exact shell counts of a simple cubic lattice, a single pair and
an excluded pair, the ideal-gas law of pair distances, and symmetry between
type pairs."""
import math

import numpy as np
import pytest
from scipy import stats


def _params(orc, periodic, box, nt=1):
    return orc.make_params(None, charge=[0.0] * nt, eps=[0.0] * nt, sigma=[0.0] * nt,
                           periodic=periodic, box=[box] * 3 if box else None, coulomb=0)


def test_simple_cubic_shells(orc):
    n, a = 6, 3.1
    g = np.arange(n) * a
    q = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    topo = orc.Topology(np.zeros(len(q), np.int32), np.ones(len(q)))
    p = _params(orc, True, n * a)
    r_max, nbins = 2.1 * a, 200
    c = orc.rdf_counts(p, topo, q, r_max, nbins)[0, 0]
    dr = r_max / nbins
    expect = np.zeros(nbins, np.int64)
    for shell, m in ((1.0, 6), (math.sqrt(2), 12), (math.sqrt(3), 8), (2.0, 6)):
        expect[int(shell * a / dr)] += m * len(q)
    assert np.array_equal(c, expect)


def test_single_and_excluded_pair(orc):
    q = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])          # r = 3
    topo = orc.Topology(np.array([0, 1], np.int32), np.ones(2))
    p = _params(orc, False, None, nt=2)
    c = orc.rdf_counts(p, topo, q, 4.0, 8)
    expect = np.zeros((2, 2, 8), np.int64)
    expect[0, 1, 6] = expect[1, 0, 6] = 1                     # 3.0 / 0.5 = bin 6
    assert np.array_equal(c, expect)
    topo_x = orc.Topology(np.array([0, 1], np.int32), np.ones(2), excl=np.array([[0, 1]]))
    assert orc.rdf_counts(p, topo_x, q, 4.0, 8).sum() == 0
    assert orc.rdf_counts(p, topo, q, 3.0, 8).sum() == 0      # r < r_max is strict


def test_ideal_gas_pair_law(orc):
    rng = np.random.default_rng(5)
    L, n = 30.0, 1500
    q = rng.uniform(0.0, L, (n, 3))
    topo = orc.Topology(np.zeros(n, np.int32), np.ones(n))
    p = _params(orc, True, L)
    r_max, nbins = 10.0, 20
    c = orc.rdf_counts(p, topo, q, r_max, nbins)[0, 0]
    edges = np.arange(nbins + 1) * (r_max / nbins)
    shell = 4.0 / 3.0 * math.pi * np.diff(edges ** 3)
    expect = n * (n - 1) / L ** 3 * shell
    # ordered pairs come in twos: test the unordered counts against Poisson scatter
    chi2 = (((c / 2 - expect / 2) ** 2) / (expect / 2)).sum()
    assert stats.chi2.sf(chi2, nbins) > 1e-4
    assert np.all(c % 2 == 0)


def test_type_pair_symmetry(orc):
    from workloads import water_droplet
    s = water_droplet(n_waters=40, seed=2)
    p = orc.make_params(s)
    c = orc.rdf_counts(p, orc.Topology.from_system(s), s.pos, 8.0, 64)
    assert np.array_equal(c[0, 1], c[1, 0])
    # intramolecular pairs are excluded: no O-H pair below 1.2 A
    assert c[0, 1, : int(1.2 / (8.0 / 64))].sum() == 0

"""Pins of the oracle's Philox4x64-10 stream and its uniform / index maps.

numpy's Philox bit generator is an independent implementation of the same
published generator (Salmon et al., SC'11); its first output block at counter c
is the Philox block of counter c + 1.
"""
import numpy as np
import pytest


def _numpy_block(ctr, key):
    # numpy advances the counter before output: start it one below, with the
    # borrow propagated the borrow of the -1 through the 256-bit counter
    words = [int(x) for x in ctr]
    val = sum(w << (64 * k) for k, w in enumerate(words)) - 1
    val %= 1 << 256
    pre = np.array([(val >> (64 * k)) & ((1 << 64) - 1) for k in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=pre)
    return bg.random_raw(4)


def test_philox_matches_numpy(orc):
    rng = np.random.default_rng(1234)
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        ctr[0] += 1  # keep away from the all-zero borrow case in half the draws
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        assert np.array_equal(orc.philox(ctr, key), _numpy_block(ctr, key))


def test_philox_counter_layout_used_by_the_process(orc):
    # counter = (step, phase << 32 | atom, k, 0), key = (seed, replica)
    step, phase, atom, k = 17, 2, 12345, 3
    ctr = [step, (phase << 32) | atom, k, 0]
    assert np.array_equal(orc.philox(ctr, [9, 4]), _numpy_block(ctr, [9, 4]))


def test_u01_open_interval_and_exact(orc):
    assert orc.u01(0) == 0.5 * 2.0**-52
    assert orc.u01(2**64 - 1) == 1.0 - 2.0**-53
    assert 0.0 < orc.u01(0) < orc.u01(2**64 - 1) < 1.0
    rng = np.random.default_rng(5)
    for w in rng.integers(0, 2**63, size=100, dtype=np.int64):
        w = int(w) * 2 + 1
        assert orc.u01(w) == ((w >> 12) + 0.5) / 2.0**52


def test_umulh_against_python_bigint(orc):
    rng = np.random.default_rng(6)
    for _ in range(500):
        a = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        c = int(rng.integers(1, 100000))
        assert orc.umulh(a, c) == (a * c) >> 64
        assert 0 <= orc.umulh(a, c) < c


def test_index_draw_is_uniform(orc):
    # J = umulh(w, n) over Philox words is uniform on {0..n-1} (chi-square)
    from scipy import stats
    n = 7
    counts = np.zeros(n)
    for s in range(7000):
        w = int(orc.philox([s, 1, 2, 0], [3, 0])[0])
        counts[orc.umulh(w, n)] += 1
    chi2 = ((counts - 1000.0) ** 2 / 1000.0).sum()
    assert stats.chi2.sf(chi2, n - 1) > 1e-4


def test_proposal_words_follow_the_layout(orc):
    """The partner of every logged proposal k comes from word 0 of the Philox
    block (step, phase, i, k), computed here by numpy's independent Philox
    (word 0 of block k = 0 is the count's uniform); the member index is
    umulh64(word, |C_i|).  Five candidates per atom and a mean of two
    proposals, so that k = 1, 2 and >= 3 all occur, in both half-steps."""
    KB = 0.0019872041
    n_groups, nc = 300, 5
    n = (nc + 1) * n_groups
    p = orc.make_params(None, charge=[-0.834], eps=[0.0], sigma=[0.0], periodic=False,
                        coulomb=0, r_on=5.0, r_off=6.0, r_cut=9.0, bound_scale=40.0, dt=1.0,
                        seed=11, replica=3)
    dirs = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [0, -1, 0]], float)
    q = np.zeros((n, 3))
    v = np.zeros((n, 3))
    row_ptr = np.zeros(n + 1, np.int64)
    col = []
    _, L_a = orc.rate_bounds(p)
    beta = 1.0 / (KB * 300.0)
    speed = 2.0 / (nc * beta * L_a[0] * 40.0 * 0.5)     # a mean of two proposals
    for g in range(n_groups):
        c = (nc + 1) * g
        q[c] = [200.0 * g, 0.0, 0.0]
        for m in range(nc):
            q[c + 1 + m] = q[c] + (6.5 + 0.4 * m) * dirs[m]
        v[c] = speed * np.array([0.6, -0.64, 0.48])
        col.extend(range(c + 1, c + 1 + nc))
    for a in range(n):
        row_ptr[a + 1] = row_ptr[a] + (nc if a % (nc + 1) == 0 else 0)
    col = np.array(col, np.int32)
    topo = orc.Topology(np.zeros(n, np.int32), np.full(n, 15.999))
    for step, phase in ((4, orc.PH_JA), (4, orc.PH_JB)):
        out = orc.jump_halfstep(p, topo, q, v, row_ptr, col, step=step, phase=phase, ev_cap=10**5)
        ev = out["events"]
        assert (ev["k"] == 1).any() and (ev["k"] == 2).any() and (ev["k"] >= 3).any()
        for e in ev:
            i, k = int(e["atom"]), int(e["k"])
            w = _numpy_block([step, (phase << 32) | i, k, 0], [11, 3])[0]
            J = (int(w) * nc) >> 64
            assert int(e["partner"]) == int(col[row_ptr[i] + J]), (step, phase, i, k)

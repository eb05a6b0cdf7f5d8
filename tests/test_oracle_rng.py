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

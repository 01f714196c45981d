"""Pins of the oracle's counter-based generator (Philox4x32-10, Salmon et al.
SC'11) and of its conversion of two 32-bit words into a uniform in (0, 1)."""
import os

import numpy as np

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append([int(x, 16) for x in line.split()])
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for row in rows:
        out = O.philox(row[0:4], row[4:6])
        assert [int(x) for x in out] == row[6:10]


def test_philox_counter_sensitivity():
    # flipping any single counter bit changes about half of the 128 output bits
    base = O.philox([5, 6, 7, 8], [9, 10])
    flips = []
    for w in range(4):
        for b in (0, 13, 31):
            ctr = [5, 6, 7, 8]
            ctr[w] ^= 1 << b
            out = O.philox(ctr, [9, 10])
            flips.append(sum(bin(int(a) ^ int(c)).count("1") for a, c in zip(base, out)))
    assert 40 < np.mean(flips) < 88


def test_u01_range_and_exactness():
    assert O.u01(0, 0) == 2.0 ** -53
    assert O.u01(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    # the low 12 bits of the 64-bit word are dropped; steps are 2^-52
    assert O.u01(0xFFF, 0) == 2.0 ** -53
    assert O.u01(0x1000, 0) == 2.0 ** -53 + 2.0 ** -52
    assert O.u01(0, 0x80000000) == 0.5 + 2.0 ** -53


def test_u01_uniformity_chi2():
    from scipy import stats
    n = 40000
    u = np.empty(n)
    for k in range(n // 2):
        x = O.philox([k, 3, 0, 0], [1234, 0])
        u[2 * k] = O.u01(int(x[0]), int(x[1]))
        u[2 * k + 1] = O.u01(int(x[2]), int(x[3]))
    assert u.min() > 0.0 and u.max() < 1.0
    counts, _ = np.histogram(u, bins=40, range=(0.0, 1.0))
    p = stats.chisquare(counts).pvalue
    assert p > 1e-3

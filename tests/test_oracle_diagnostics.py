"""Pins of the oracle's sigma_d(m, r) diagnostic (paper, Benchmark: dust
surface density as a function of particle mass and distance from the star):
hand-computed bins, the half-open edge rule, exclusion of inactive and
out-of-range particles, mass conservation, and agreement of the bin counts
with numpy's independent two-dimensional histogram."""
import numpy as np

import oracle as O
from paper_2507_21239_amd import workloads as W

AU = W.AU


def _part(r, m, M, active=None):
    n = len(r)
    return dict(r=np.asarray(r, float), m=np.asarray(m, float), M=np.asarray(M, float),
                active=np.ones(n, np.uint8) if active is None else np.asarray(active, np.uint8))


def test_single_particles_hand_computed():
    re = np.array([1.0, 2.0, 4.0]) * AU
    me = np.array([1e-12, 1e-9, 1e-6, 1e-3])
    # bin (1, 2): r in [2, 4) AU, m in [1e-6, 1e-3)
    part = _part([3.0 * AU], [5e-5], [7.0e20])
    sigma, count, n = O.sigma_hist(part, re, me)
    assert n == 1 and count.sum() == 1 and count[1, 2] == 1
    area = np.pi * ((4.0 * AU) ** 2 - (2.0 * AU) ** 2)
    assert sigma[1, 2] == 7.0e20 / area
    assert np.count_nonzero(sigma) == 1


def test_edges_are_half_open_and_out_of_range_is_dropped():
    re = np.array([1.0, 2.0, 4.0]) * AU
    me = np.array([1.0, 10.0, 100.0])
    r = [1.0 * AU, 2.0 * AU, 4.0 * AU, 0.5 * AU, 3.0 * AU, 3.0 * AU]
    m = [1.0, 10.0, 5.0, 5.0, 100.0, 0.5]
    sigma, count, n = O.sigma_hist(_part(r, m, np.ones(6)), re, me)
    # the first edge is inside its bin, the last edge outside: r = 4 AU,
    # r = 0.5 AU, m = 100 and m = 0.5 fall out
    assert n == 2
    assert count[0, 0] == 1 and count[1, 1] == 1 and count.sum() == 2


def test_inactive_particles_are_excluded_and_column_mode_has_unit_area():
    re = np.array([0.5, 1.5]) * AU
    me = np.array([1.0, 2.0])
    part = _part([AU, AU, AU], [1.5, 1.5, 1.5], [2.0, 3.0, 5.0], active=[1, 0, 1])
    sigma, count, n = O.sigma_hist(part, re, me, column=True)
    assert n == 2 and count[0, 0] == 2 and sigma[0, 0] == 7.0


def test_mass_conservation_and_counts_match_histogram2d():
    rng = np.random.default_rng(5)
    N = 20000
    r = AU * 10.0 ** rng.uniform(-0.1, 2.1, N)
    m = 10.0 ** rng.uniform(-12.5, 2.5, N)
    M = rng.uniform(0.5, 2.0, N) * 1e22
    act = (rng.random(N) > 0.05).astype(np.uint8)
    re = AU * np.geomspace(1.0, 100.0, 31)
    me = np.geomspace(1e-12, 1e2, 57)
    sigma, count, n = O.sigma_hist(_part(r, m, M, act), re, me)
    inside = (act == 1) & (r >= re[0]) & (r < re[-1]) & (m >= me[0]) & (m < me[-1])
    assert n == inside.sum() == count.sum()
    h, _, _ = np.histogram2d(r[inside], m[inside], bins=[re, me])
    assert np.array_equal(h.astype(np.uint32), count)
    area = np.pi * (re[1:] ** 2 - re[:-1] ** 2)
    total = (sigma * area[:, None]).sum()
    assert abs(total - M[inside].sum()) <= 1e-12 * M[inside].sum()
    # every bin's mass is the sum of its members' swarm masses
    hm, _, _ = np.histogram2d(r[inside], m[inside], bins=[re, me], weights=M[inside])
    assert np.allclose(sigma * area[:, None], hm, rtol=1e-12, atol=0.0)

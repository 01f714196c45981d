"""Pins of the oracle's event sampling (Zsom & Dullemond 2008): on tiny cells
the frequencies of the chosen pairs (i, j) must follow the brute-force
probabilities r_ij / R, and waiting times must be exponential with rate R."""
import numpy as np
import pytest
from scipy import stats

import oracle as O
from paper_2507_21239_amd import workloads as W

AU = W.AU


def _tiny_cell(n=4, seed=3):
    rng = np.random.default_rng(seed)
    m = 10.0 ** rng.uniform(-11, -4, n)
    M = 10.0 ** rng.uniform(20, 21, n)
    gas = [1e36, 3e-11, 120.0, 1e-3, 5 * AU, 0.4]
    return m, M, gas


@pytest.mark.parametrize("kernel", ["physical", "constant"])
def test_pair_frequencies_match_rates(kernel):
    m, M, gas = _tiny_cell()
    n = len(m)
    p = W.benchmark_params(kernel=kernel, dm_max=0.0, k0=1.0)
    R, rs = O.cell_rates(p, gas, np.arange(n), m, M)
    prob = R / R.sum()
    draws = 20000
    counts = np.zeros((n, n))
    taus = np.empty(draws)
    cells = dict(cell_start=np.array([0, n], dtype=np.int32), order=np.arange(n, dtype=np.int32),
                 gas=np.array([gas]))
    for s in range(draws):
        part = dict(m=m.copy(), M=M)
        out = O.collide_all(p, cells, s, part, 0.0, 1, log_per_cell=1)
        ev = out["log"][0][0]
        counts[ev["i"], ev["j"]] += 1
        taus[s] = out["stats"]["t_end"][0]
    exp = prob * draws
    mask = exp > 5
    chi2 = ((counts[mask] - exp[mask]) ** 2 / exp[mask]).sum()
    assert stats.chi2.sf(chi2, mask.sum() - 1) > 1e-4, (counts, exp)
    assert counts[~mask].sum() <= max(20.0, 3 * exp[~mask].sum())
    # exponential waiting times with the total rate
    assert stats.kstest(taus, "expon", args=(0, 1.0 / R.sum())).pvalue > 1e-4


def test_time_limited_stop_is_memoryless():
    # with a time limit dt the first event happens inside dt with probability
    # 1 - exp(-R dt) (constant kernel: every r_ij = n_j K = 1, R = n^2)
    n = 3
    p = W.benchmark_params(kernel="constant", dm_max=0.0, k0=1.0)
    gas = [1.0, 1.0, 1.0, 1.0, AU, 0.0]
    cells = dict(cell_start=np.array([0, n], dtype=np.int32), order=np.arange(n, dtype=np.int32),
                 gas=np.array([gas]))
    R0 = n * n * 1.0
    dt = 0.05
    hits = 0
    trials = 20000
    for s in range(trials):
        part = dict(m=np.ones(n), M=np.ones(n))
        out = O.collide_all(p, cells, s, part, dt, 1)
        hits += int(out["stats"]["events"][0])
    pexp = 1.0 - np.exp(-R0 * dt)
    se = np.sqrt(pexp * (1 - pexp) / trials)
    assert abs(hits / trials - pexp) < 4 * se


def test_incremental_rates_match_fresh_rates():
    # after many events the incrementally updated row sums agree with a fresh
    # evaluation up to accumulated rounding
    rng = np.random.default_rng(5)
    n = 40
    m = 10.0 ** rng.uniform(-11, -6, n)
    M = np.full(n, 1e22)
    gas = [1e36, 1e-10, 150.0, 1e-3, 3 * AU, 0.2]
    p = W.benchmark_params(dm_max=0.0)
    R0, rs0 = O.cell_rates(p, gas, np.arange(n), m, M)
    cells = dict(cell_start=np.array([0, n], dtype=np.int32), order=np.arange(n, dtype=np.int32),
                 gas=np.array([gas]))
    part = dict(m=m.copy(), M=M)
    out = O.collide_all(p, cells, 0, part, 0.0, 300)
    assert out["stats"]["events"][0] == 300
    assert not np.array_equal(part["m"], m)
    assert np.array_equal(part["M"], M)
    assert out["stats"]["drift"][0] < 1e-11

"""Pins of the oracle's collision Monte Carlo against the analytic solutions
of the Smoluchowski equation (the coagulation equation the paper names as
the usual model, Statement of Need) for the constant and linear kernels,
plus exact swarm-mass conservation.

Representative particles sample the mass-weighted distribution (Zsom &
Dullemond 2008), so the mean representative mass is M2/M1 and the mean of
1/m is M0/M1.  Monomers, n0 = 1, total mass density 1:
  constant K = 1:  n_k = (1+T/2)^-2 (T/(2+T))^(k-1);  M0 = 1/(1+T/2);  M2 = 1 + T
  linear K = m_i + m_j:  n_k = e^-T (k g)^(k-1) e^(-k g) / k!, g = 1 - e^-T;
                         M0 = e^-T;  M2 = e^(2T)
"""
import numpy as np
import pytest
from scipy import special, stats

import oracle as O
from paper_2507_21239_amd import workloads as W

N_SEEDS = 64


def _ensemble(make, seeds):
    ms, evs = [], []
    for s in seeds:
        w = make(s)
        M0 = w["particles"]["M"].copy()
        out = O.collide_all(w["params"], w["cells"], 0, w["particles"], w["dt"], w["max_events"])
        assert np.array_equal(w["particles"]["M"], M0)          # swarm masses never written
        ms.append(w["particles"]["m"].copy())
        evs.append(int(out["stats"]["events"][0]))
    return np.array(ms), np.array(evs)


def _mean_se(per_seed):
    return per_seed.mean(), per_seed.std(ddof=1) / np.sqrt(len(per_seed))


@pytest.fixture(scope="module")
def constant_runs():
    return _ensemble(lambda s: W.c1_single_cell(seed=s), range(N_SEEDS))


def test_constant_kernel_moments(constant_runs):
    ms, _ = constant_runs
    T = 1998.0
    mean_m, se_m = _mean_se(ms.mean(axis=1))
    assert abs(mean_m - (1.0 + T)) < 3.5 * se_m, (mean_m, se_m)
    mean_inv, se_inv = _mean_se((1.0 / ms).mean(axis=1))
    assert abs(mean_inv - 1.0 / (1.0 + T / 2.0)) < 3.5 * se_inv, (mean_inv, se_inv)


def test_constant_kernel_masses_are_integers(constant_runs):
    ms, _ = constant_runs
    assert np.all(ms == np.rint(ms))
    assert ms.min() >= 1.0


def test_constant_kernel_mass_histogram(constant_runs):
    ms, _ = constant_runs
    T = 1998.0
    rho = T / (2.0 + T)
    k = np.arange(1, 40000)
    f = k * (1.0 + T / 2.0) ** -2 * rho ** (k - 1)          # mass fraction in size k
    assert abs(f.sum() - 1.0) < 1e-6
    cdf = np.cumsum(f)
    edges_k = [int(np.searchsorted(cdf, q)) + 1 for q in np.linspace(0.1, 0.9, 9)]
    bins = np.concatenate([[0.5], np.array(edges_k) + 0.5, [k[-1] + 0.5]])
    expected = np.diff(np.concatenate([[0.0], cdf[np.array(edges_k) - 1], [cdf[-1]]])) * ms.size
    observed, _ = np.histogram(ms.ravel(), bins=bins)
    chi2 = ((observed - expected) ** 2 / expected).sum()
    # particles of one run are weakly correlated; allow a generous bound
    assert chi2 < stats.chi2.ppf(0.9999, len(expected) - 1) * 2.0, (observed, expected)


def test_constant_kernel_event_count(constant_runs):
    _, evs = constant_runs
    # events per representative particle = int_0^t K n_tot dt = 2 ln(1 + T/2)
    expect = 200 * 2.0 * np.log(1.0 + 1998.0 / 2.0)
    mean, se = _mean_se(evs.astype(float))
    assert abs(mean - expect) / expect < 0.02 and abs(mean - expect) < 6 * se, (mean, se, expect)


def test_linear_kernel_moments():
    T = 2.0
    ms, _ = _ensemble(lambda s: W.linear_single_cell(seed=s, t_end=T), range(N_SEEDS))
    mean_m, se_m = _mean_se(ms.mean(axis=1))
    assert abs(mean_m - np.exp(2 * T)) < 3.5 * se_m, (mean_m, se_m)
    mean_inv, se_inv = _mean_se((1.0 / ms).mean(axis=1))
    assert abs(mean_inv - np.exp(-T)) < 3.5 * se_inv, (mean_inv, se_inv)
    # histogram against the analytic mass fraction k n_k
    g = 1.0 - np.exp(-T)
    k = np.arange(1, 3000).astype(float)
    logn = -T + (k - 1) * np.log(k * g) - k * g - special.gammaln(k + 1)
    f = k * np.exp(logn)
    assert abs(f.sum() - 1.0) < 1e-6 and abs((k * f).sum() - np.exp(2 * T)) / np.exp(2 * T) < 1e-6
    bins = np.array([0.5, 1.5, 3.5, 8.5, 20.5, 50.5, 120.5, 3000.0])
    cdf = np.concatenate([[0.0], np.cumsum(f)])
    expected = np.diff(np.interp(bins - 0.5, np.arange(len(cdf)), cdf)) * ms.size
    observed, _ = np.histogram(ms.ravel(), bins=bins)
    rel = np.abs(observed - expected) / expected
    assert np.all(rel < 0.15), (observed, expected)


def test_event_log_replays_masses():
    # replaying the logged (i, j) sticking events on the initial masses gives
    # the final masses bit for bit
    w = W.c1_single_cell(seed=7)
    m_init = w["particles"]["m"].copy()
    out = O.collide_all(w["params"], w["cells"], 0, w["particles"], w["dt"], 0, log_per_cell=6000)
    ne = int(out["stats"]["events"][0])
    assert 0 < ne < 6000
    log = out["log"][0][:ne]
    m = m_init.copy()
    for e in log:
        assert e["outcome"] == 0
        m[e["i"]] = m[e["i"]] + m[e["j"]]
    assert np.array_equal(m, w["particles"]["m"])

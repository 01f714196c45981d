"""GPU sigma_d(m, r) against the oracle on seeded synthetic particles:
counts bit-exact, masses within the reordering bound of FP64 sums (the GPU
adds with atomics in arbitrary order: relative 2 * count * 2^-53 per bin)."""
import numpy as np
import pytest

import oracle as O
from paper_2507_21239_amd import workloads as W

from gpu_common import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
AU = W.AU


def _particles(seed, N, column=False):
    rng = np.random.default_rng(seed)
    part = W._particles(N)
    part["r"][:] = AU if column else AU * 10.0 ** rng.uniform(-0.2, 2.2, N)
    part["z"][:] = np.abs(rng.standard_normal(N)) * 0.05 * AU
    part["m"][:] = 10.0 ** rng.uniform(-12.5, 3.0, N)
    part["M"][:] = rng.uniform(0.1, 3.0, N) * 1e21
    part["active"][:] = (rng.random(N) > 0.07).astype(np.uint8)
    return part


def _compare(part, params, re, me, column=False):
    from paper_2507_21239_amd import api
    sim = api.Simulation(params, api.to_device(part), precision="mixed")
    sig, cnt = sim.sigma_hist(re, me)
    sig = sig.cpu().numpy()
    cnt = cnt.cpu().numpy().view(np.uint32)
    sim.close()
    osig, ocnt, n = O.sigma_hist(part, re, me, column=column)
    assert np.array_equal(cnt, ocnt)
    bound = 2.0 * np.maximum(ocnt, 1) * 2.0 ** -53 * np.abs(osig)
    assert np.all(np.abs(sig - osig) <= bound + 1e-300), np.max(np.abs(sig - osig) / (bound + 1e-300))
    return n


@pytest.mark.parametrize("N,n_rb,n_mb,seed", [(50_000, 30, 60, 0),      # LDS bins
                                             (50_000, 100, 64, 1),     # 6400 bins: global atomics
                                             (2_000_000, 60, 64, 2),   # the large disk's size
                                             (777, 1, 1, 3)])
def test_sigma_hist_matches_oracle(N, n_rb, n_mb, seed):
    say("sigma_hist", N, n_rb, n_mb)
    part = _particles(seed, N)
    re = AU * np.geomspace(1.0, 100.0, n_rb + 1)
    me = np.geomspace(1e-12, 1e2, n_mb + 1)
    # particles exactly on edges: the first and interior edges belong to the
    # bin they open, the last edge to none
    k = min(N, 5)
    part["r"][:k] = re[np.linspace(0, n_rb, k).astype(int)]
    part["m"][:k] = me[np.linspace(0, n_mb, k).astype(int)]
    n = _compare(part, W.benchmark_params(), re, me)
    assert n > 0


def test_sigma_hist_column_mode_and_empty():
    part = _particles(4, 3000, column=True)
    params = W.benchmark_params(n_r=1, n_z=5, column=1)
    re = np.array([0.5, 1.5]) * AU
    me = np.geomspace(1e-12, 1e2, 41)
    _compare(part, params, re, me, column=True)
    part["active"][:] = 0
    assert _compare(part, params, re, me, column=True) == 0


def test_sigma_hist_rejects_bad_edges():
    from paper_2507_21239_amd import api
    part = _particles(5, 100)
    sim = api.Simulation(W.benchmark_params(), api.to_device(part), precision="mixed")
    good = np.geomspace(1.0, 2.0, 5)
    for re, me in ((good[::-1], good), (good, np.array([1.0, 1.0, 2.0])),
                   (np.array([1.0, np.nan]), good), (np.array([-1.0, 1.0]), good),
                   (np.array([1.0]), good)):
        with pytest.raises(api.MCDError):
            sim.sigma_hist(re, me)
    sim.close()


def test_benchmark_shaped_run_conserves_swarm_mass():
    from paper_2507_21239_amd import disk_run
    say("disk_run short")
    out = disk_run.run(N=20_000, n_r=20, n_z=5, years=20.0, dt_yr=1.0, precision="mixed",
                       r_bins=40, m_bins=50, history_every=4, n_comp=8, verbose=False)
    # histories: one row per 4 steps, masses never below the monomer mass,
    # composition fractions summing to one (one-hot start, mass-weighted mixing)
    h = out["history"]
    assert h.shape == (5, 16, 3 + 8)
    assert np.all(h[:, :, 2] > 0.0)
    assert np.allclose(h[:, :, 3:].sum(axis=2), 1.0, atol=1e-5)
    area = np.pi * (out["r_edges"][1:] ** 2 - out["r_edges"][:-1] ** 2)
    binned = float((out["sigma"] * area[:, None]).sum())
    # every active particle lies inside the edges, which span the initial disk
    # and the whole mass range; swarm masses never change
    assert out["count"].sum() == out["n_active"]
    assert abs(binned - out["active_swarm_mass"]) <= 1e-11 * out["active_swarm_mass"]
    assert out["steps"] == 20 and out["events"] > 0

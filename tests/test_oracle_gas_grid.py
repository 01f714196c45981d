"""Pins of the oracle's gridded gas (post-processing a hydrodynamic state,
the paper's Statement of Need) against closed forms: exact node values, exact
interpolation of power laws (log-linear in ln r), the pressure slope and the
radial-diffusion correction of the power-law disk, a vertical slab whose
surface density is exact, and clamping outside the grid."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2507_21239_amd import workloads as W

AU = W.AU


def _powerlaw_grid(P, r_nodes, z_nodes):
    rho = np.zeros((len(r_nodes), len(z_nodes)))
    T = np.zeros_like(rho)
    for k, r in enumerate(r_nodes):
        for l, z in enumerate(z_nodes):
            d = O.disk_local(P, r, z)
            rho[k, l], T[k, l] = d["rho_g"], d["T"]
    return dict(r_nodes=r_nodes, z_nodes=z_nodes, rho=rho, T=T, alpha=np.full_like(rho, P["alpha"]))


def test_nodes_and_midplane_power_laws_are_reproduced():
    P = W.benchmark_params()
    rn = AU * np.geomspace(1.0, 100.0, 25)
    zn = np.linspace(0.0, 0.3 * AU, 40)   # up to ~9 scale heights at 1 AU: no underflow
    G = dict(P, gas_grid=_powerlaw_grid(P, rn, zn))
    for r in rn[::6]:
        for z in zn[::13]:
            a, b = O.local_gas(G, r, z), O.disk_local(P, r, z)
            assert a["rho_g"] == pytest.approx(b["rho_g"], rel=1e-13)
            assert a["T"] == pytest.approx(b["T"], rel=1e-13)
    for r in AU * np.geomspace(1.1, 90.0, 17):   # between nodes, midplane
        a, b, pl = O.local_gas(G, r, 0.0), O.disk_local(P, r, 0.0), O.local_gas(P, r, 0.0)
        assert a["rho_g"] == pytest.approx(b["rho_g"], rel=1e-12)
        assert a["T"] == pytest.approx(b["T"], rel=1e-12)
        assert a["alpha"] == pytest.approx(P["alpha"], rel=1e-14)
        # -d ln P / d ln r of the power-law disk at the midplane
        assert a["slopeP"] == pytest.approx(P["p"] + (P["q"] + 3.0) / 2.0, rel=1e-10)
        assert pl["slopeP"] == P["p"] + (P["q"] + 3.0) / 2.0
        assert pl["corr"] == 2.5 - P["q"] - P["p"]


def test_vertical_slab_diffusion_correction_is_exact():
    # rho_g = 1e-9 (r/AU)^-2 up to z = 0.2 AU, T = 300 (r/AU)^-0.6, alpha =
    # 1e-3 (r/AU)^0.5: Sigma_g = 2 z_max rho_g exactly, so the correction
    # factor d ln(r Sigma_g alpha c_s H) / d ln r is -2 + 0.5 - 0.6 + 5/2
    P = W.benchmark_params()
    rn = AU * np.geomspace(1.0, 50.0, 12)
    zn = np.linspace(0.0, 0.2 * AU, 5)
    x = rn / AU
    ones = np.ones(len(zn))
    grid = dict(r_nodes=rn, z_nodes=zn, rho=np.outer(1e-9 * x ** -2.0, ones),
                T=np.outer(300.0 * x ** -0.6, ones), alpha=np.outer(1e-3 * x ** 0.5, ones))
    G = dict(P, gas_grid=grid)
    for r in AU * np.geomspace(1.3, 45.0, 9):
        for z in (0.0, 0.05 * AU, 0.2 * AU, 1.0 * AU):
            a = O.local_gas(G, r, z)
            assert a["corr"] == pytest.approx(-2.0 + 0.5 - 0.6 + 2.5, abs=1e-12)
            assert a["slopeP"] == pytest.approx(2.0 + 0.6, abs=1e-12)
            assert a["rho_g"] == pytest.approx(1e-9 * (r / AU) ** -2.0, rel=1e-12)
            assert a["alpha"] == pytest.approx(1e-3 * (r / AU) ** 0.5, rel=1e-12)
            cs = math.sqrt(1.380649e-16 * a["T"] / (P["mu"] * 1.6735575e-24))
            assert a["cs"] == pytest.approx(cs, rel=1e-12)


def test_outside_the_grid_values_are_clamped():
    P = W.benchmark_params()
    rn = AU * np.array([2.0, 4.0, 8.0])
    zn = np.array([0.0, 0.1 * AU])
    rho = np.array([[3.0, 1.0], [2.0, 0.5], [1.0, 0.25]]) * 1e-10
    T = np.array([[200.0, 210.0], [150.0, 160.0], [100.0, 110.0]])
    grid = dict(r_nodes=rn, z_nodes=zn, rho=rho, T=T, alpha=np.full_like(rho, 1e-3))
    G = dict(P, gas_grid=grid)
    a = O.local_gas(G, 1.0 * AU, 1.0 * AU)       # inside of r_0, above z_max
    assert a["rho_g"] == pytest.approx(1e-10, rel=1e-14) and a["T"] == pytest.approx(210.0, rel=1e-14)
    b = O.local_gas(G, 20.0 * AU, 0.0)
    assert b["rho_g"] == pytest.approx(1e-10, rel=1e-14) and b["T"] == pytest.approx(100.0, rel=1e-14)
    # bilinear in (ln r, z) of the logarithms at an interior point
    c = O.local_gas(G, math.sqrt(2.0 * 4.0) * AU, 0.05 * AU)
    want = math.exp(0.25 * sum(math.log(v) for v in (3.0e-10, 1.0e-10, 2.0e-10, 0.5e-10)))
    assert c["rho_g"] == pytest.approx(want, rel=1e-13)

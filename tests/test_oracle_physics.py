"""Pins of the oracle's gas state, particle properties, pair kernel, rates
and collision outcomes against closed forms and special values that follow
from the physics by a different route than the oracle's own formulas.

Reference values at 1 AU for the paper's benchmark disk (Benchmark table:
Sigma_g = 1000 g/cm^2, T = 280 K, alpha = 1e-3; mu = 2.34, 1 Msun) worked by
hand:  c_s = sqrt(k T / (mu m_H)) = 993.6 m/s;  Omega = 1.991e-7 /s;
H = c_s/Omega = 0.0334 AU;  rho_mid = Sigma/(sqrt(2 pi) H) = 7.99e-10 g/cm^3;
lambda = mu m_H / (rho sigma_H2) = 2.45 cm;  eta v_K = 45.6 m/s;
Re = alpha c_s H / (v_th lambda / 2) = 2.56e8.
"""
import numpy as np
import pytest
from scipy import integrate

import oracle as O
from paper_2507_21239_amd import workloads as W

AU = W.AU
KB = 1.380649e-16


def rel(a, b):
    return abs(a - b) / abs(b)


def P(**kw):
    return W.benchmark_params(**kw)


def midplane_gas(params, r):
    d = O.disk_local(params, r, 0.0)
    return d, O.gas_derive(params, [1e30, d["rho_g"], d["T"], params["alpha"], r, 0.0])


def mass_for_epstein_St(params, Sigma_g, St):
    # midplane Epstein identity St = pi a rho_s / (2 Sigma_g), solved for a
    a = 2.0 * Sigma_g * St / (np.pi * params["rho_s"])
    return 4.0 / 3.0 * np.pi * params["rho_s"] * a ** 3


def test_benchmark_table_matches_paper():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "benchmark_table.txt")
    p = P()
    with open(path) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                name, val = line.split()[:2]
                assert p[name] == float(val), name


def test_gas_sanity_1au():
    p = P()
    d, g = midplane_gas(p, AU)
    assert rel(d["cs"], 99360.0) < 1e-3
    assert rel(d["Omega"], 1.991e-7) < 1e-3
    assert rel(d["H"] / AU, 0.0334) < 2e-3
    assert rel(d["rho_g"], 7.99e-10) < 2e-3
    assert rel(g.lambda_, 2.45) < 3e-3
    assert rel(g.eta_vK, 4560.0) < 2e-3
    assert rel(g.Re, 2.56e8) < 1e-2
    assert rel(g.St_eta, 2.56e8 ** -0.5) < 1e-2
    assert g.z_c == 0.0


def test_power_laws():
    p = P()
    d1 = O.disk_local(p, AU, 0.0)
    d4 = O.disk_local(p, 4 * AU, 0.0)
    assert rel(d4["Sigma_g"], d1["Sigma_g"] / 4.0) < 1e-14          # p = 1
    assert rel(d4["T"], d1["T"] / 2.0) < 1e-14                      # q = 0.5
    # vertically isothermal Gaussian: rho(z = H) / rho(0) = e^-1/2
    dz = O.disk_local(p, AU, d1["H"])
    assert rel(dz["rho_g"] / d1["rho_g"], np.exp(-0.5)) < 1e-14
    assert dz["T"] == d1["T"]


def test_midplane_epstein_identity():
    p = P()
    d, g = midplane_gas(p, AU)
    for a in (1e-5, 1e-4, 1e-2, 1.0):
        m = 4.0 / 3.0 * np.pi * p["rho_s"] * a ** 3
        q = O.particle(p, g, m, 1.0)
        assert rel(q.a, a) < 1e-14
        assert rel(q.St, np.pi * a * p["rho_s"] / (2.0 * d["Sigma_g"])) < 1e-13


def test_drag_law_continuous_at_switch():
    p = P()
    _, g = midplane_gas(p, AU)
    a_sw = 2.25 * g.lambda_
    ts = []
    for f in (1.0 - 1e-12, 1.0 + 1e-12):
        m = 4.0 / 3.0 * np.pi * p["rho_s"] * (a_sw * f) ** 3
        ts.append(O.particle(p, g, m, 1.0).t_s)
    assert rel(ts[0], ts[1]) < 1e-10
    # Stokes regime: t_s ~ a^2 beyond the switch
    m1 = 4.0 / 3.0 * np.pi * p["rho_s"] * (4 * a_sw) ** 3
    m2 = 4.0 / 3.0 * np.pi * p["rho_s"] * (8 * a_sw) ** 3
    assert rel(O.particle(p, g, m2, 1.0).t_s / O.particle(p, g, m1, 1.0).t_s, 4.0) < 1e-12


@pytest.fixture(scope="module")
def outer_disk():
    # at 100 AU the Epstein regime extends beyond St = 1
    p = P()
    r = 100 * AU
    d = O.disk_local(p, r, 0.0)
    def gas(zeta=0.0):
        return O.gas_derive(p, [1e30, d["rho_g"], d["T"], p["alpha"], r, zeta])
    def part(params, g, St):
        return O.particle(params, g, mass_for_epstein_St(params, d["Sigma_g"], St), 1.0)
    return d, gas, part


def test_radial_drift_closed_forms(outer_disk):
    d, gas, part = outer_disk
    p = P(flags=["radial"])
    g = gas()
    p1, p0 = part(p, g, 1.0), part(p, g, 1e-9)
    assert rel(p1.St, 1.0) < 1e-12
    # maximum drift speed, eta v_K, is reached at St = 1
    assert rel(p1.v_r, -g.eta_vK) < 1e-12
    assert rel(O.rel_velocity(p, g, p1, p0), g.eta_vK) < 1e-8
    # v_r(St) = v_r(1/St)
    assert O.rel_velocity(p, g, part(p, g, 2.0), part(p, g, 0.5)) < 1e-9 * g.eta_vK


def test_azimuthal_and_settling_closed_forms(outer_disk):
    d, gas, part = outer_disk
    pa = P(flags=["azimuthal"])
    g = gas()
    assert rel(O.rel_velocity(pa, g, part(pa, g, 1.0), part(pa, g, 1e-12)), g.eta_vK / 2.0) < 1e-10
    assert rel(part(pa, g, 1e-12).v_phi, -g.eta_vK) < 1e-10
    ps = P(flags=["settling"])
    g1 = gas(zeta=1.0)                         # z_c = H, so z_c Omega = c_s
    assert rel(g1.z_c, g1.H) < 1e-15
    dv = O.rel_velocity(ps, g1, part(ps, g1, 1.0), part(ps, g1, 1e-12))
    assert rel(dv, d["cs"] / 2.0) < 1e-10


def test_brownian_reduced_mass_form():
    # mean relative thermal speed of two Maxwellian particles, sqrt(8kT/(pi mu))
    p = P(flags=["brownian"])
    _, g = midplane_gas(p, AU)
    for mi, mj in ((1e-12, 1e-12), (1e-12, 3e-9), (2.5e-6, 1e-11)):
        qi, qj = O.particle(p, g, mi, 1.0), O.particle(p, g, mj, 1.0)
        mu_red = mi * mj / (mi + mj)
        dv = np.sqrt(8.0 * KB * g.T / (np.pi * mu_red))
        ai = (3 * mi / (4 * np.pi * p["rho_s"])) ** (1 / 3)
        aj = (3 * mj / (4 * np.pi * p["rho_s"])) ** (1 / 3)
        assert rel(O.pair_kernel(p, g, qi, qj), np.pi * (ai + aj) ** 2 * dv) < 1e-12


def test_turbulence_special_values():
    p = P()
    _, g = midplane_gas(p, AU)
    Vg2, Se = g.Vg2, g.St_eta
    # intermediate regime, equal particles: bracket = 2 y_a - 2 + 2/(1 + y_a) = 1.96923...
    for s in (1e-3, 0.1, 0.9):
        assert rel(O.dv2_turb(g, s, s), Vg2 * s * 1.9692307692307692) < 1e-13
    # intermediate regime, epsilon -> 0: bracket -> 2 y_a - 1 + 2/(1 + y_a) = 2.96923...
    assert rel(O.dv2_turb(g, 0.1, 1e-14), Vg2 * 0.1 * 2.9692307692307692) < 1e-12
    # heavy regime: equal particles 2 Vg^2/(1 + St)
    for s in (1.0, 3.0, 1e4):
        assert rel(O.dv2_turb(g, s, s), 2.0 * Vg2 / (1.0 + s)) < 1e-14
    # tightly coupled: identical particles move together; a tracer partner
    # leaves Vg^2 St1^2 / (St1 + St_eta)
    s = Se / 10
    assert O.dv2_turb(g, s, s) == 0.0
    assert rel(O.dv2_turb(g, s, s * 1e-12), Vg2 * s * s / (s + Se)) < 1e-10
    # symmetric in the pair
    assert O.dv2_turb(g, 0.3, 0.01) == O.dv2_turb(g, 0.01, 0.3)


def test_velocity_sources_add_in_quadrature():
    base = P()
    d, _ = midplane_gas(base, 5 * AU)
    prim = [1e30, d["rho_g"] * 0.3, d["T"], base["alpha"], 5 * AU, 0.7]
    for mi, mj in ((1e-11, 1e-3), (1e-6, 1e-6 * 1.0001), (3.0, 1e-8)):
        parts = []
        for f in W.VELOCITY_SOURCES:
            pf = P(flags=[f])
            g = O.gas_derive(pf, prim)
            parts.append(O.rel_velocity(pf, g, O.particle(pf, g, mi, 1.0), O.particle(pf, g, mj, 1.0)))
            assert parts[-1] >= 0.0
        g = O.gas_derive(base, prim)
        allv = O.rel_velocity(base, g, O.particle(base, g, mi, 1.0), O.particle(base, g, mj, 1.0))
        assert rel(allv, np.sqrt(np.sum(np.square(parts)))) < 1e-13
        assert min(parts) >= 0.0 and allv > max(parts)


def test_rate_definition_and_grouping():
    # constant kernel: r_ij = n_j K = M_j/(m_j V) K
    p = P(kernel="constant", k0=2.5, dm_max=0.0)
    g = O.gas_derive(p, [7.0, 1.0, 1.0, 1.0, AU, 0.0])
    qi, qj = O.particle(p, g, 3.0, 11.0), O.particle(p, g, 2.0, 5.0)
    assert rel(O.rate(p, g, qi, qj), 5.0 / (2.0 * 7.0) * 2.5) < 1e-15
    # grouping keeps the mean mass-gain rate: rate * (mass gained) = n_j K m_j
    pg = P(kernel="constant", k0=2.5, dm_max=1e-3)
    for mi, mj in ((1e6, 1.0), (5.0, 1.0), (1e3, 0.5)):
        qi, qj = O.particle(pg, g, mi, 11.0), O.particle(pg, g, mj, 5.0)
        rate = O.rate(pg, g, qi, qj)
        kind, mnew = O.outcome(pg, 0.0, mi, mj, 0.5)
        assert kind == "stick"
        assert rel(rate * (mnew - mi), 5.0 / (mj * 7.0) * 2.5 * mj) < 1e-12
    # the rate matrix of a cell agrees with the single-pair rates
    m = np.array([1.0, 2.0, 7.0]); M = np.array([1.0, 3.0, 5.0])
    R, rs = O.cell_rates(pg, [7.0, 1.0, 1.0, 1.0, AU, 0.0], [0, 1, 2], m, M)
    qs = [O.particle(pg, g, m[k], M[k]) for k in range(3)]
    for i in range(3):
        for j in range(3):
            assert R[i, j] == O.rate(pg, g, qs[i], qs[j])
        assert rs[i] == R[i, 0] + R[i, 1] + R[i, 2]


def test_outcome_thresholds():
    p = P()
    m0 = 4.0 / 3.0 * np.pi * p["a_mono"] ** 3 * p["rho_s"]
    vf = p["v_frag"]
    assert O.outcome(p, np.nextafter(vf, 0.0), 2.0, 1.0, 0.5) == ("stick", 3.0)
    kind, mn = O.outcome(p, vf, 2.0, 1.0, 0.5)
    assert kind == "frag" and m0 <= mn <= 2.0
    assert O.outcome(p, 2 * vf, 10.0, 1.0, 0.5) == ("erode", 9.0)
    kind, mn = O.outcome(p, 2 * vf, 9.999, 1.0, 0.5)
    assert kind == "frag" and m0 <= mn <= 9.999
    kind, mn = O.outcome(p, 2 * vf, 1.0, 10.0, 0.5)
    assert kind == "eroded_small" and m0 <= mn <= 1.0
    assert O.outcome(p, 2 * vf, 1.05 * m0, 0.1 * m0, 0.5) == ("erode", m0)
    # grouped erosion removes dm_max m_i
    kind, mn = O.outcome(p, 2 * vf, 1e6, 1.0, 0.5)
    assert kind == "erode" and rel(mn, 1e6 - 1e3) < 1e-15
    # the test kernels always stick
    pc = P(kernel="constant")
    assert O.outcome(pc, 1e9, 2.0, 1.0, 0.5)[0] == "stick"


def test_frag_draw_inverse_cdf():
    # mass-weighted fragment distribution ~ m^(1 - 11/6) = m^(-5/6) on [lo, hi]:
    # the draw at u must sit at the u-quantile of the numerically integrated pdf
    # (integrated over t = ln m, where the integrand m^(-5/6) dm = e^(t/6) dt is smooth)
    lo, hi = 6.7e-12, 3.0e-3
    pdf_t = lambda t: np.exp(t) ** (-5.0 / 6.0) * np.exp(t)
    norm = integrate.quad(pdf_t, np.log(lo), np.log(hi), epsabs=0, epsrel=1e-13)[0]
    for u in (1e-6, 0.01, 0.25, 0.5, 0.75, 0.99, 1 - 1e-9):
        m = O.frag_draw(lo, hi, u)
        assert lo <= m <= hi
        F = integrate.quad(pdf_t, np.log(lo), np.log(m), epsabs=0, epsrel=1e-13)[0] / norm
        assert abs(F - u) < 1e-8, (u, F)
    assert O.frag_draw(lo, lo, 0.3) == lo
    assert O.frag_draw(1.0, 0.5, 0.3) == 1.0


def test_select_rule():
    assert O.select([1, 2, 3, 4], 0.5) == 0
    assert O.select([1, 2, 3, 4], 1.0) == 1        # prefix must exceed the target
    assert O.select([1, 2, 3, 4], 9.99) == 3
    assert O.select([1, 2, 3, 4], 10.0) == 3       # rounding fallback: last nonzero
    assert O.select([0, 1, 0, 2], 0.0) == 1        # zero entries are never chosen
    assert O.select([0, 1, 0, 2, 0], 3.5) == 3
    assert O.select([0, 0], 0.0) == -1

"""Pins of the oracle's transport step (paper, Summary: transport in the
vertical and radial directions) against closed forms: the stationary
vertical profile of the settling-mixing Fokker-Planck equation, the
well-mixed limit of tracers, the radial drift speed, the diffusive spread
of a ring, the planar diffusion law of a radial walk in a uniform gas
(power-law and gridded), tracers that stay distributed like the gas, and
removal at the inner edge."""
import numpy as np
from scipy import integrate

import oracle as O
from paper_2507_21239_amd import workloads as W

AU, YR = W.AU, W.YR


def _column(N, a, z0_scale, flags, seed):
    p = W.benchmark_params(column=1, n_r=1, n_z=1, flags=flags)
    rng = np.random.default_rng(seed)
    H = O.disk_local(p, AU, 0.0)["H"]
    m = 4.0 / 3.0 * np.pi * p["rho_s"] * a ** 3
    part = dict(r=np.full(N, AU), z=np.abs(rng.standard_normal(N)) * z0_scale * H,
                m=np.full(N, m), M=np.ones(N), active=np.ones(N, dtype=np.uint8))
    return p, part, H


def _run(p, part, steps, dt, sample_from):
    acc = []
    for s in range(steps):
        O.transport(p, part, s, dt)
        if s >= sample_from:
            acc.append(np.mean(part["z"] ** 2))
    return np.mean(acc)


def test_tracers_stay_well_mixed():
    p, part, H = _column(10000, 1e-4, 1.0, ["tr_settle", "tr_mix_z"], seed=1)
    x2 = _run(p, part, 300, 1.0 * YR, 100) / H ** 2
    assert abs(x2 - 1.0) < 0.04, x2


def test_settling_mixing_equilibrium():
    # St(z) = St0 exp(z^2 / 2H^2) (Epstein drag in a Gaussian gas column);
    # the zero-flux solution of the Fokker-Planck equation of
    # dz = -z (Omega St/(1+St) + D/H^2) dt + sqrt(2D) dW, D = alpha Omega H^2/(1+St^2):
    # p(x) ~ (1+St^2) exp(-int_0^x x' [1 + St (1+St^2) / (alpha (1+St))] dx'), x = z/H
    alpha, St0 = 1e-3, 1e-3
    Sigma = 1000.0
    a = 2.0 * Sigma * St0 / (np.pi * 1.6)
    p, part, H = _column(10000, a, 0.7, ["tr_settle", "tr_mix_z"], seed=2)

    def St(x):
        return St0 * np.exp(0.5 * x * x)

    def phi(x):
        return integrate.quad(lambda y: y * (1 + St(y) * (1 + St(y) ** 2) / (alpha * (1 + St(y)))), 0, x)[0]

    dens = lambda x: (1 + St(x) ** 2) * np.exp(-phi(x))
    norm = integrate.quad(dens, 0, 8)[0]
    x2_exact = integrate.quad(lambda x: x * x * dens(x), 0, 8)[0] / norm
    # Dubrulle et al. (1995) estimate with constant St0: alpha/(alpha+St0) = 0.5
    assert 0.35 < x2_exact < 0.5
    x2 = _run(p, part, 1200, 0.5 * YR, 400) / H ** 2
    assert abs(x2 - x2_exact) / x2_exact < 0.03, (x2, x2_exact)


def test_radial_drift_speed():
    # one step, drift only: dr = -2 eta v_K St/(1+St^2) dt with eta v_K = 45.6 m/s
    # at every radius of the benchmark disk (q = 0.5) and the midplane Epstein
    # Stokes number St = pi a rho_s / (2 Sigma_g(r))
    p = W.benchmark_params(flags=["tr_drift"])
    r0 = 10 * AU
    a = 0.01
    m = 4.0 / 3.0 * np.pi * p["rho_s"] * a ** 3
    part = dict(r=np.array([r0]), z=np.array([0.0]), m=np.array([m]), M=np.ones(1),
                active=np.ones(1, dtype=np.uint8))
    O.transport(p, part, 0, YR)
    St = np.pi * a * 1.6 / (2.0 * 1000.0 * (r0 / AU) ** -1)
    dr = -2.0 * 4560.0 * St / (1 + St * St) * YR
    assert abs((part["r"][0] - r0) - dr) / abs(dr) < 2e-3
    assert part["z"][0] == 0.0


def test_radial_spread_of_a_ring():
    # tracers, radial mixing only: variance grows by 2 D dt per step with
    # D = alpha c_s H; c_s(10 AU) = 993.6 m/s 10^-1/4, H(10 AU) = 0.0334 AU 10^1.25
    p = W.benchmark_params(flags=["tr_mix_r"])
    N, steps = 20000, 50
    r0 = 10 * AU
    m = 4.0 / 3.0 * np.pi * p["rho_s"] * 1e-4 ** 3
    part = dict(r=np.full(N, r0), z=np.zeros(N), m=np.full(N, m), M=np.ones(N),
                active=np.ones(N, dtype=np.uint8))
    for s in range(steps):
        O.transport(p, part, s, YR)
    D = 1e-3 * 99360.0 * 10 ** -0.25 * 0.0334 * AU * 10 ** 1.25
    var = np.var(part["r"])
    assert abs(var / (2 * D * steps * YR) - 1.0) < 0.04


def _tracers(p, r, seed=0):
    m = 4.0 / 3.0 * np.pi * p["rho_s"] * p["a_mono"] ** 3
    N = len(r)
    return dict(r=np.array(r, dtype=np.float64), z=np.zeros(N), m=np.full(N, m), M=np.ones(N),
                active=np.ones(N, dtype=np.uint8))


def _planar_diffusion(p, steps=100, N=400_000, r0=2 * AU):
    """Mean growth of r^2 of tracers released at r0 and the diffusivity D
    (constant in r for the disks used here)."""
    part = _tracers(p, np.full(N, r0))
    for s in range(steps):
        O.transport(p, part, s, YR)
    assert part["active"].all()
    g = O.local_gas(p, r0, 0.0)
    D = g["alpha"] * g["cs"] * g["H"]
    x = part["r"] ** 2 - r0 ** 2
    return x.mean(), x.std() / np.sqrt(N), 4.0 * D * steps * YR


def test_radial_walk_follows_the_planar_diffusion_law():
    # Sigma_g and D independent of r (p = 0, q = 3/2: c_s H ~ r^(3/2 - q)):
    # tracers in a uniform gas diffuse like a planar random walk, for which
    # E[r^2] - r0^2 = E[x^2 + y^2] - r0^2 = 4 D t exactly; a walk with no
    # geometric drift would give 2 D t, one with the opposite sign 0
    p = W.benchmark_params(p=0.0, q=1.5, alpha=0.1, r_in=0.0, flags=["tr_mix_r"])
    got, se, want = _planar_diffusion(p)
    assert abs(got - want) < 4.0 * se, (got / want, se / want)
    assert abs(got / want - 1.0) < 0.03, got / want


def test_gridded_gas_walk_follows_the_planar_diffusion_law():
    # the same law through the gridded gas: a slab of constant density and
    # turbulence with T ~ r^-3/2 (so alpha c_s H is constant), sampled on nodes
    p = W.benchmark_params(p=0.0, q=1.5, alpha=0.1, r_in=0.0, flags=["tr_mix_r"])
    rn = AU * np.geomspace(0.05, 20.0, 30)
    zn = np.linspace(0.0, 0.5 * AU, 4)
    ones = np.ones(len(zn))
    grid = dict(r_nodes=rn, z_nodes=zn, rho=np.full((len(rn), len(zn)), 1e-9),
                T=np.outer(280.0 * (rn / AU) ** -1.5, ones), alpha=np.full((len(rn), len(zn)), 0.1))
    got, se, want = _planar_diffusion(dict(p, gas_grid=grid))
    assert abs(got - want) < 4.0 * se, (got / want, se / want)
    assert abs(got / want - 1.0) < 0.03, got / want


def test_tracers_distributed_like_the_gas_stay_so_radially():
    # a passive tracer whose surface density is proportional to the gas's
    # stays so: per unit r the particles are distributed ~ r Sigma_g.  Here
    # Sigma_g ~ r^-1/2 and D ~ r (p = q = 1/2); particles start ~ r^1/2 on
    # [0.2, 12] AU and the count inside [1, 3] AU, far from both edges, must
    # not change beyond its sampling noise (at most the square root of the
    # number of particles that entered or left).  Dropping the walk's
    # geometric drift moves the count by ~5 % (12 times that noise)
    p = W.benchmark_params(p=0.5, q=0.5, alpha=0.3, r_in=0.0, flags=["tr_mix_r"])
    N, steps = 400_000, 100
    a, b = 0.2, 12.0
    u = np.random.default_rng(5).random(N)
    r = AU * (a ** 1.5 + u * (b ** 1.5 - a ** 1.5)) ** (2.0 / 3.0)   # density ~ r^1/2
    part = _tracers(p, r)
    inside = lambda x: (x > AU) & (x < 3 * AU)
    i0 = inside(part["r"])
    for s in range(steps):
        O.transport(p, part, s, YR)
    i1 = inside(part["r"])
    n0, n1 = int(i0.sum()), int(i1.sum())
    moved = np.count_nonzero(i0 != i1)
    expect = N * (3 ** 1.5 - 1) / (b ** 1.5 - a ** 1.5)
    assert abs(n0 - expect) < 4 * np.sqrt(expect)
    assert moved > 0.1 * n0                     # the walk did mix across the window's edges
    assert abs(n1 - n0) < 4 * np.sqrt(moved), (n0, n1, moved)


def test_inner_edge_removes_particles():
    p = W.benchmark_params(flags=["tr_drift"], r_in=AU)
    m = 4.0 / 3.0 * np.pi * p["rho_s"] * 30.0 ** 3
    part = dict(r=np.array([1.0000001 * AU, 50 * AU, 2 * AU]), z=np.zeros(3), m=np.full(3, m),
                M=np.ones(3), active=np.array([1, 1, 0], dtype=np.uint8))
    O.transport(p, part, 0, YR)
    assert list(part["active"]) == [0, 1, 0]
    assert part["r"][2] == 2 * AU                       # inactive particles are not moved
    r_after = part["r"].copy()
    O.transport(p, part, 1, YR)
    assert part["r"][0] == r_after[0]

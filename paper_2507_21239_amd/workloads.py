"""Seeded synthetic workloads shaped like the paper's benchmark.

This module only draws inputs: parameter sets, particle arrays and explicit
cells.  It holds none of the method's arithmetic (no rates, no gas-state
derivation, no selection, no outcomes) and imports nothing else from this
package, so that the GPU library and the CPU oracle can both consume the very
same inputs.

Parameter values follow the paper's Benchmark table (arXiv 2507.21239):
Sigma_g(1 AU) = 1000 g/cm^2, T(1 AU) = 280 K, alpha = 1e-3, v_frag = 10 m/s,
erosion mass ratio 10, p = 1, q = 0.5.  Values the paper does not give (monomer
radius, material density, mean molecular weight, stellar mass, grouping
threshold, eroded-mass factor) are stated readings.

Flags are given by name; each side maps the names onto its own bit layout.
"""
from __future__ import annotations

import numpy as np

AU = 1.495978707e13   # cm
YR = 3.15576e7        # s (Julian year)
MSUN = 1.98847e33     # g

VELOCITY_SOURCES = ("brownian", "turb", "radial", "azimuthal", "settling")
ALL_FLAG_NAMES = VELOCITY_SOURCES + ("tr_drift", "tr_settle", "tr_mix_r", "tr_mix_z", "coag")

# scale height of the benchmark disk at 1 AU for T = 280 K, mu = 2.34, 1 Msun
# (c_s / Omega = 993.6 m/s / 1.991e-7 s^-1); used only to place initial
# particles, with H ~ r^((3 - q)/2) = r^1.25
H_1AU_BENCH = 0.0334 * AU


def benchmark_params(**over) -> dict:
    """Parameters of the paper's benchmark disk plus the stated readings."""
    p = dict(
        sigma_g0=1000.0, T0=280.0, p=1.0, q=0.5, alpha=1e-3,
        v_frag=1000.0, erosion_ratio=10.0,
        a_mono=1e-4, rho_s=1.6, mu=2.34, m_star=MSUN, r_ref=AU,
        dm_max=1e-3, erosion_chi=1.0, r_in=AU, r_col=AU, k0=1.0,
        kernel="physical", n_r=1, n_z=1, column=0,
        flags=list(VELOCITY_SOURCES) + ["coag"],
        n_comp=0, seed=0, frag_mode="sharp", frag_width=0.2,
    )
    p.update(over)
    return p


def _explicit_cells(counts: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    cell_start = np.zeros(len(counts) + 1, dtype=np.int32)
    cell_start[1:] = np.cumsum(counts)
    order = np.arange(int(cell_start[-1]), dtype=np.int32)
    return cell_start, order


def _particles(N: int) -> dict:
    return dict(
        r=np.zeros(N), z=np.zeros(N), m=np.zeros(N), M=np.zeros(N),
        active=np.ones(N, dtype=np.uint8), comp=None,
    )


def c1_single_cell(seed: int = 0, n: int = 200, t_end: float = 1998.0) -> dict:
    """One cell, constant kernel K = 1, monomers of mass 1, equal swarm masses
    (total mass density 1 in a unit volume), run to dimensionless time 1998
    where the number-mean mass of the Smoluchowski solution is 1 + T/2 = 1000."""
    params = benchmark_params(kernel="constant", k0=1.0, dm_max=0.0, flags=["coag"], seed=seed)
    part = _particles(n)
    part["m"][:] = 1.0
    part["M"][:] = 1.0 / n
    cell_start, order = _explicit_cells(np.array([n]))
    gas = np.array([[1.0, 1.0, 1.0, 1.0, AU, 0.0]])   # only V = 1 enters the test kernels
    return dict(name="c1_single_cell", params=params, particles=part,
                cells=dict(cell_start=cell_start, order=order, gas=gas),
                dt=t_end, max_events=0)


def linear_single_cell(seed: int = 0, n: int = 200, t_end: float = 2.0) -> dict:
    """One cell, linear kernel K = m_i + m_j, monomers of mass 1, total mass
    density 1, run to dimensionless time T = t_end."""
    out = c1_single_cell(seed=seed, n=n, t_end=t_end)
    out["params"]["kernel"] = "linear"
    out["name"] = "linear_single_cell"
    return out


def _half_normal(rng: np.random.Generator, scale: np.ndarray) -> np.ndarray:
    return np.abs(rng.standard_normal(scale.shape)) * scale


def c2_column(seed: int = 0, n_z: int = 20, per_cell: int = 200) -> dict:
    """One vertical column at 1 AU, full physical kernel, settling and vertical
    mixing on, 20 equal-count cells of 200 particles; masses per unit area."""
    rng = np.random.default_rng(seed)
    N = n_z * per_cell
    params = benchmark_params(
        n_r=1, n_z=n_z, column=1, seed=seed,
        flags=list(VELOCITY_SOURCES) + ["coag", "tr_settle", "tr_mix_z"])
    part = _particles(N)
    m0 = 4.0 / 3.0 * np.pi * params["a_mono"] ** 3 * params["rho_s"]
    part["r"][:] = AU
    part["z"][:] = _half_normal(rng, np.full(N, H_1AU_BENCH))
    part["m"][:] = m0
    part["M"][:] = 0.01 * params["sigma_g0"] / N     # dust-to-gas 0.01, per unit area
    return dict(name="c2_column", params=params, particles=part, cells=None,
                dt=1.0 * YR, max_events=0, n_steps=1000)


def c3_disk(seed: int = 0, N: int = 100_000, n_r: int = 50, n_z: int = 10,
            n_comp: int = 0) -> dict:
    """2-D disk from 1 to 100 AU with log-spaced start radii, Sigma ~ r^-1,
    T ~ r^-0.5; drift, settling, turbulent mixing and coagulation."""
    rng = np.random.default_rng(seed)
    params = benchmark_params(
        n_r=n_r, n_z=n_z, column=0, seed=seed, n_comp=n_comp, r_in=AU,
        flags=list(VELOCITY_SOURCES) + ["coag", "tr_drift", "tr_settle", "tr_mix_r", "tr_mix_z"])
    part = _particles(N)
    k = np.arange(N)
    r = AU * 100.0 ** ((k + 0.5) / N)
    part["r"][:] = r
    part["z"][:] = _half_normal(rng, H_1AU_BENCH * (r / AU) ** 1.25)
    m0 = 4.0 / 3.0 * np.pi * params["a_mono"] ** 3 * params["rho_s"]
    part["m"][:] = m0
    # swarm masses ~ Sigma_d(r) r^2 (log spacing), normalised to 1% of the gas
    # mass between 1 and 100 AU: 2 pi Sigma0 AU^2 (100 - 1)
    w = (r / AU) ** (-params["p"]) * (r / AU) ** 2
    m_dust = 0.01 * 2.0 * np.pi * params["sigma_g0"] * AU * AU * 99.0
    part["M"][:] = m_dust * w / w.sum()
    if n_comp:
        comp = np.zeros((n_comp, N), dtype=np.float32)
        octile = np.minimum((np.log(r / AU) / np.log(100.0) * n_comp).astype(int), n_comp - 1)
        comp[octile, k] = 1.0
        part["comp"] = comp
    return dict(name="c3_disk", params=params, particles=part, cells=None,
                dt=1.0 * YR, max_events=0, n_steps=10_000)


def c5_large_disk(seed: int = 0, N: int = 2_000_000, n_r: int = 1000, n_z: int = 10) -> dict:
    """The 2-D disk at 2e6 particles, ~1e4 cells of ~200, with 8 FP32
    composition fractions initialised one-hot by the octile of log r."""
    out = c3_disk(seed=seed, N=N, n_r=n_r, n_z=n_z, n_comp=8)
    out["name"] = "c5_large_disk"
    return out


def gridded_gas(params: dict, n_r: int = 48, n_z: int = 24, r_lo: float = 0.5 * AU,
                r_hi: float = 200.0 * AU, seed: int = 0) -> dict:
    """A synthetic gas state on a grid (standing in for hydrodynamic output):
    the power-law disk's midplane density and temperature with a Gaussian
    pressure bump near 10 AU and a gap near 30 AU, scale heights from the
    local temperature, a vertical density floor, turbulence rising outwards
    and a small seeded ripple.  Node values only; no physics of the method."""
    rng = np.random.default_rng(seed)
    rn = np.geomspace(r_lo, r_hi, n_r)
    x = rn / params["r_ref"]
    T = params["T0"] * x ** -params["q"]
    cs2 = 1.380649e-16 * T / (params["mu"] * 1.6735575e-24)
    Om = np.sqrt(6.67430e-8 * params["m_star"] / rn ** 3)
    H = np.sqrt(cs2) / Om
    sig = params["sigma_g0"] * x ** -params["p"]
    sig *= 1.0 + 1.5 * np.exp(-0.5 * ((np.log(rn / (10 * AU))) / 0.15) ** 2)
    sig *= 1.0 - 0.9 * np.exp(-0.5 * ((np.log(rn / (30 * AU))) / 0.1) ** 2)
    zn = np.linspace(0.0, 5.0 * H.max(), n_z)
    rho_mid = sig / (np.sqrt(2 * np.pi) * H)
    rho = rho_mid[:, None] * np.exp(-0.5 * (zn[None, :] / H[:, None]) ** 2)
    rho = np.maximum(rho, 1e-12 * rho_mid[:, None])
    rho *= 1.0 + 0.02 * rng.standard_normal(rho.shape)
    Tg = np.repeat(T[:, None], n_z, axis=1) * (1.0 + 0.3 * (zn[None, :] / zn[-1]) ** 2)
    alpha = np.repeat((params["alpha"] * (1.0 + 0.5 * np.log10(x / x[0])))[:, None], n_z, axis=1)
    return dict(r_nodes=rn, z_nodes=zn, rho=rho, T=Tg, alpha=alpha)


def c4_batched(seed: int = 0, n_cells: int = 4096, n_lo: int = 64, n_hi: int = 1024,
               events: int = 1000, philox_seed: int = 0, V: float = 1e36,
               counts=None) -> dict:
    """Independent cells with log-uniform particle counts in [n_lo, n_hi]
    (or the given counts), log-uniform masses 1e-12 .. 1e2 g, random local
    gas (rho_g, T, alpha, radius, height in scale heights); exactly `events`
    collisions per cell."""
    rng = np.random.default_rng(seed)
    if counts is None:
        counts = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), n_cells))).astype(np.int32)
    else:
        counts = np.asarray(counts, dtype=np.int32)
        n_cells = len(counts)
    cell_start, order = _explicit_cells(counts)
    N = int(cell_start[-1])
    params = benchmark_params(seed=philox_seed, flags=list(VELOCITY_SOURCES) + ["coag"])
    part = _particles(N)
    part["m"][:] = 10.0 ** rng.uniform(-12.0, 2.0, N)
    rho_g = 10.0 ** rng.uniform(-14.0, -9.0, n_cells)
    T = 10.0 ** rng.uniform(np.log10(20.0), np.log10(300.0), n_cells)
    alpha = 10.0 ** rng.uniform(-5.0, -2.0, n_cells)
    r_c = AU * 10.0 ** rng.uniform(0.0, 2.0, n_cells)
    zeta = rng.uniform(0.0, 2.0, n_cells)
    gas = np.stack([np.full(n_cells, V), rho_g, T, alpha, r_c, zeta], axis=1)
    Mc = 0.01 * rho_g * V / np.maximum(counts, 1)
    part["M"][:] = np.repeat(Mc, counts)
    return dict(name="c4_batched", params=params, particles=part,
                cells=dict(cell_start=cell_start, order=order, gas=gas),
                dt=0.0, max_events=events)


def subset_cells(work: dict, cells: np.ndarray) -> dict:
    """Restrict an explicit-cell workload to the given cells (renumbered)."""
    cs = work["cells"]["cell_start"]
    counts = (cs[cells + 1] - cs[cells]).astype(np.int32)
    idx = np.concatenate([np.arange(cs[c], cs[c + 1]) for c in cells]).astype(np.int64)
    part = {k: (v[idx].copy() if isinstance(v, np.ndarray) and v.ndim == 1 else v)
            for k, v in work["particles"].items()}
    if work["particles"].get("comp") is not None:
        part["comp"] = work["particles"]["comp"][:, idx].copy()
    new_start, order = _explicit_cells(counts)
    out = dict(work)
    out["particles"] = part
    out["cells"] = dict(cell_start=new_start, order=order, gas=work["cells"]["gas"][cells].copy())
    out["name"] = work["name"] + f"[{len(cells)} cells]"
    return out

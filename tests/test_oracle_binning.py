"""Pins of the oracle's equal-count adaptive binning (paper, Summary: every
cell holds the same number of representative particles) against a library
sort, and of the cell geometry against tiling properties."""
import numpy as np
import pytest

import oracle as O
from paper_2507_21239_amd import workloads as W

AU = W.AU


def _inputs(N, seed, ties=True):
    rng = np.random.default_rng(seed)
    r = AU * 10.0 ** rng.uniform(0, 2, N)
    z = np.abs(rng.standard_normal(N)) * 0.05 * r
    if ties:
        k = rng.choice(N, N // 5, replace=False)
        r[k[: len(k) // 2]] = r[k[len(k) // 2: 2 * (len(k) // 2)]]   # duplicated radii
        z[k[::3]] = z[k[0]]                                           # duplicated heights
        z[k[1::7]] = 0.0
    active = (rng.random(N) > 0.1).astype(np.uint8)
    return r, z, active


def _library_binning(r, z, active, n_r, n_z):
    idx = np.nonzero(active)[0]
    na = len(idx)
    by_r = idx[np.lexsort((idx, r[idx]))]                 # ascending (r, index)
    order = np.empty(na, dtype=np.int64)
    cell_start = np.zeros(n_r * n_z + 1, dtype=np.int64)
    for k in range(n_r):
        b0, b1 = k * na // n_r, (k + 1) * na // n_r
        zone = by_r[b0:b1]
        zone = zone[np.lexsort((zone, z[zone]))]          # ascending (|z|, index)
        order[b0:b1] = zone
        nk = b1 - b0
        for l in range(n_z):
            cell_start[k * n_z + l] = b0 + l * nk // n_z
    cell_start[-1] = na
    return cell_start, order


@pytest.mark.parametrize("N,n_r,n_z,seed", [(203, 5, 4, 0), (1000, 7, 3, 1), (4000, 1, 20, 2),
                                            (97, 3, 3, 3), (12, 4, 5, 4)])
def test_binning_matches_library_sort(N, n_r, n_z, seed):
    r, z, active = _inputs(N, seed)
    p = W.benchmark_params(n_r=n_r, n_z=n_z)
    out = O.bin_particles(p, r, z, active)
    cs, order = _library_binning(r, z, active, n_r, n_z)
    assert out["n_active"] == int(active.sum())
    assert np.array_equal(out["cell_start"], cs)
    assert np.array_equal(out["order"], order)
    counts = np.diff(out["cell_start"])
    # equal count per zone up to the floor rule
    for k in range(n_r):
        c = counts[k * n_z:(k + 1) * n_z]
        assert c.max() - c.min() <= 1


def test_geometry_tiles_the_disk():
    r, z, active = _inputs(5000, 11, ties=False)
    n_r, n_z = 8, 6
    p = W.benchmark_params(n_r=n_r, n_z=n_z)
    out = O.bin_particles(p, r, z, active)
    geom = out["geom"].reshape(n_r, n_z, 5)
    cs, order = out["cell_start"], out["order"]
    for k in range(n_r):
        assert np.all(geom[k, :, 0] == geom[k, 0, 0]) and np.all(geom[k, :, 1] == geom[k, 0, 1])
        if k + 1 < n_r:
            assert geom[k, 0, 1] == geom[k + 1, 0, 0]          # shared radial edge
        assert geom[k, 0, 2] == 0.0                              # grid starts at the midplane
        assert np.all(geom[k, :-1, 3] == geom[k, 1:, 2])        # shared vertical edges
        ztop = geom[k, -1, 3]
        # cell volumes of a zone add up to the annulus volume 2 pi (r_hi^2 - r_lo^2) z_top
        vol = 2 * np.pi * (geom[k, 0, 1] ** 2 - geom[k, 0, 0] ** 2) * ztop
        assert abs(geom[k, :, 4].sum() - vol) / vol < 1e-12
        for l in range(n_z):
            c = k * n_z + l
            mem = order[cs[c]:cs[c + 1]]
            assert np.all(r[mem] >= geom[k, l, 0]) and np.all(r[mem] <= geom[k, l, 1])
            assert np.all(z[mem] >= geom[k, l, 2]) and np.all(z[mem] <= geom[k, l, 3])
    assert geom[0, 0, 0] == r[active == 1].min() and geom[-1, 0, 1] == r[active == 1].max()


def test_cell_gas_at_cell_centre():
    r, z, active = _inputs(3000, 12, ties=False)
    p = W.benchmark_params(n_r=6, n_z=5)
    out = O.bin_particles(p, r, z, active)
    for c in (0, 7, 29):
        g = out["geom"][c]
        rc, zc = 0.5 * (g[0] + g[1]), 0.5 * (g[2] + g[3])
        d = O.disk_local(p, rc, zc)
        V, rho, T, alpha, r_c, zeta = out["gas"][c]
        assert V == g[4] and rho == d["rho_g"] and T == d["T"] and r_c == rc
        assert abs(zeta * d["H"] - zc) <= 1e-15 * zc + 1e-300


def test_column_mode_volume_per_unit_area():
    w = W.c2_column(seed=0)
    part = w["particles"]
    out = O.bin_particles(w["params"], part["r"], part["z"], part["active"])
    assert np.all(np.diff(out["cell_start"]) == 200)
    g = out["geom"]
    assert np.allclose(g[:, 4], 2.0 * (g[:, 3] - g[:, 2]), rtol=0, atol=0)
    assert np.all(out["gas"][:, 4] == W.AU)


def test_empty_and_tiny_inputs():
    p = W.benchmark_params(n_r=3, n_z=2)
    r = np.array([2.0, 1.0]) * AU
    z = np.array([0.1, 0.2]) * AU
    out = O.bin_particles(p, r, z, np.array([1, 1], dtype=np.uint8))
    assert out["n_active"] == 2
    assert out["cell_start"][-1] == 2 and np.all(np.diff(out["cell_start"]) >= 0)
    assert np.diff(out["cell_start"]).sum() == 2
    out = O.bin_particles(p, r, z, np.array([0, 0], dtype=np.uint8))
    assert out["n_active"] == 0 and np.all(out["cell_start"] == 0)

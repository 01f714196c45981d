"""Gridded gas on the GPU against the oracle with the same grid: binning
and the cell gas, then bin -> collide -> transport steps of a small disk in
FP64 (event counts equal, masses and positions within 1e-11), and the
power-law disk restored by clearing the grid."""
import numpy as np
import pytest

import oracle as O
from paper_2507_21239_amd import workloads as W

from gpu_common import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _api():
    from paper_2507_21239_amd import api
    return api


def test_binning_cell_gas_from_the_grid():
    api = _api()
    work = W.c3_disk(seed=3, N=30000, n_r=15, n_z=8)
    grid = W.gridded_gas(work["params"], seed=1)
    p = dict(work["params"], gas_grid=grid)
    say("grid binning")
    sim = api.Simulation(work["params"], api.to_device(work["particles"]), precision="fp64")
    sim.set_gas_grid(grid)
    sim.bin()
    cells = {k: v.cpu().numpy() for k, v in sim.cells().items()}
    part = work["particles"]
    ref = O.bin_particles(p, part["r"], part["z"], part["active"])
    assert np.array_equal(cells["cell_start"], ref["cell_start"])
    assert np.array_equal(cells["order"], ref["order"])
    occ = np.diff(ref["cell_start"]) > 0
    g, gr = cells["gas"][occ], ref["gas"][occ]
    assert np.all(np.abs(g - gr) <= 1e-13 * np.abs(gr) + 1e-300)
    # the grid's gas differs from the power-law disk's (bump, gap, ripple)
    pl = O.bin_particles(work["params"], part["r"], part["z"], part["active"])
    assert np.max(np.abs(pl["gas"][occ][:, 1] / gr[:, 1] - 1.0)) > 0.05
    sim.close()


@pytest.mark.parametrize("schedule", ["batched", "plain"])
def test_disk_steps_with_the_grid_fp64(schedule):
    api = _api()
    work = W.c3_disk(seed=8, N=20000, n_r=20, n_z=10, n_comp=8)
    grid = W.gridded_gas(work["params"], seed=2)
    p = dict(work["params"], gas_grid=grid)
    dt = 30.0 * W.YR
    ref = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in work["particles"].items()}
    dev = api.to_device(work["particles"])
    say("grid disk steps", schedule)
    sim = api.Simulation(work["params"], dev, precision="fp64", schedule=schedule)
    sim.set_gas_grid(grid)
    sim.bin()
    sim.step(dt, 0, 3)
    st = sim.stats()
    ev = 0
    for s in range(3):
        out = O.step(p, ref, s, dt, 0, threads=8)
        ev += int(out["stats"]["events"].sum())
    assert st["events"] == ev and ev > 0
    g = {k: v.cpu().numpy() for k, v in dev.items()}
    assert np.array_equal(g["active"], ref["active"])
    for k in ("m", "r", "z"):
        assert np.all(np.abs(g[k] - ref[k]) <= 1e-11 * np.abs(ref[k]) + 1e-300), k
    assert np.max(np.abs(g["comp"] - ref["comp"])) <= 1e-6
    sim.close()


def test_clearing_the_grid_restores_the_power_law_and_bad_grids_are_rejected():
    api = _api()
    work = W.c3_disk(seed=4, N=5000, n_r=5, n_z=5)
    grid = W.gridded_gas(work["params"], seed=3)
    sim = api.Simulation(work["params"], api.to_device(work["particles"]), precision="fp64")
    sim.set_gas_grid(grid)
    sim.set_gas_grid(None)
    sim.bin()
    cells = {k: v.cpu().numpy() for k, v in sim.cells().items()}
    part = work["particles"]
    ref = O.bin_particles(work["params"], part["r"], part["z"], part["active"])
    occ = np.diff(ref["cell_start"]) > 0
    assert np.all(np.abs(cells["gas"][occ] - ref["gas"][occ]) <= 1e-13 * np.abs(ref["gas"][occ]))
    bad = [dict(grid, rho=-grid["rho"]), dict(grid, r_nodes=grid["r_nodes"][::-1]),
           dict(grid, z_nodes=grid["z_nodes"] - 1.0), dict(grid, T=grid["T"] * np.nan)]
    for b in bad:
        with pytest.raises(api.MCDError):
            sim.set_gas_grid(b)
    sim.close()

"""mcd_collide_noalloc -- the entry point for callers that cannot allocate
device memory -- against the context path it stands for (mcd_init,
mcd_bin with explicit cells, one mcd_step), through the C ABI: two calls in
a row, the second on a smaller input, in both precisions.  The two run the
same kernels and schedule, so masses, compositions and counts must be
identical (FP64: the oracle's event decisions; mixed: the same FP32
arithmetic)."""
import numpy as np
import pytest

from paper_2507_21239_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _work(seed, n_cells, events):
    w = W.c4_batched(seed=seed, n_cells=n_cells, events=events)
    N = len(w["particles"]["m"])
    rng = np.random.default_rng(seed)
    comp = np.zeros((2, N), dtype=np.float32)
    comp[0] = rng.random(N) < 0.5
    comp[1] = 1.0 - comp[0]
    w["particles"]["comp"] = comp
    w["params"] = dict(w["params"], n_comp=2)
    return w


def _context_path(work, precision, max_cell):
    from paper_2507_21239_amd import api
    dev = api.to_device(work["particles"])
    sim = api.Simulation(work["params"], dev, precision=precision, schedule="batched")
    sim.bin(api.cells_to_device(work["cells"]), max_cell=max_cell)
    sim.step(0.0, work["max_events"], 1)
    st = sim.stats()
    sim.close()
    return {k: v.cpu().numpy() for k, v in dev.items()}, st


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_the_context_path(precision):
    from paper_2507_21239_amd import api
    for seed, n_cells, events in ((2, 300, 200), (3, 40, 120)):   # the second call is smaller
        work = _work(seed, n_cells, events)
        max_cell = int(np.diff(work["cells"]["cell_start"]).max())
        print("[case] noalloc", precision, "cells", n_cells, "max_cell", max_cell, flush=True)
        ref, st = _context_path(work, precision, max_cell)
        dev = api.to_device(work["particles"])
        counts = api.collide_noalloc(work["params"], dev, api.cells_to_device(work["cells"]), 0.0,
                                     events, step=0, precision=precision, max_cell=max_cell)
        c = counts.cpu().numpy()
        assert c[0] == st["events"] == events * n_cells
        assert list(c[1:5]) == st["outcomes"]
        assert c[5] == 0
        g = {k: v.cpu().numpy() for k, v in dev.items()}
        assert np.array_equal(g["m"], ref["m"])
        assert np.array_equal(g["comp"], ref["comp"])
        assert np.array_equal(g["M"], work["particles"]["M"])


def test_noalloc_rejects_sizes_beyond_its_scratch():
    from paper_2507_21239_amd import api
    work = _work(4, 8, 10)
    dev = api.to_device(work["particles"])
    cells = api.cells_to_device(work["cells"])
    with pytest.raises(api.MCDError) as e:
        api.collide_noalloc(work["params"], dev, cells, 0.0, 10, max_cell=0)
    assert e.value.status == -1 and "max_cell" in str(e.value)
    big = dict(cells, cell_start=torch.zeros((1 << 20) + 2, dtype=torch.int32, device="cuda"))
    with pytest.raises(api.MCDError) as e:
        api.collide_noalloc(work["params"], dev, big, 0.0, 10, max_cell=64)
    assert e.value.status == -1 and "1048576" in str(e.value)

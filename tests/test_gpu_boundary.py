"""The C-ABI boundary on the GPU: the library works in the caller's
workspace and allocates no device memory in mcd_init, mcd_bin, mcd_step or
mcd_tune; explicit cells are planned on the device, with a size bound
(asynchronous, validated on the device) or without one (measured); a grid
that fails validation collides nothing and is reported; and the largest
cells of each precision run while larger ones are rejected."""
import numpy as np
import pytest

import oracle as O
from paper_2507_21239_amd import workloads as W

from gpu_common import compare_logs, edge_size_work, run_oracle_explicit, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _api():
    from paper_2507_21239_amd import api
    return api


def test_library_allocates_no_device_memory():
    api = _api()
    work = W.c5_large_disk(seed=0)
    dev = api.to_device(work["particles"])
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    say("large disk: workspace from torch, init / bin / tune / steps")
    sim = api.Simulation(work["params"], dev, precision="mixed", schedule="batched")
    ws = sim.workspace.numel()
    assert ws > 100 * 2 ** 20              # grid, binning buffers, backups of 2e6 particles
    sim.bin()
    sim.tune(W.YR, 0)
    sim.step(W.YR, 0, 3)                   # graph capture and replays
    sim.step(W.YR, 0, 1)
    st = sim.stats()
    assert st["events"] > 0 and st["steps"] == 4
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    # torch's own allocation of the workspace (cached blocks) aside, nothing
    # of the size of the library's buffers was taken
    used = free0 - free1
    say("device memory taken", used, "workspace", ws)
    assert used <= ws + 64 * 2 ** 20, (used, ws)
    sim.close()


def test_explicit_cells_with_a_bound_plan_asynchronously_and_match():
    work = edge_size_work(events=100)
    opart, oout = run_oracle_explicit(work, log_per_cell=120, threads=8)
    api = _api()
    for schedule in ("batched", "plain"):
        say("bounded explicit cells", schedule)
        dev = api.to_device(work["particles"])
        sim = api.Simulation(work["params"], dev, precision="fp64", schedule=schedule)
        sim.bin(api.cells_to_device(work["cells"]), max_cell=1024)
        nc = len(work["cells"]["cell_start"]) - 1
        log = torch.full((nc * 120 * 4,), -7, dtype=torch.int32, device="cuda")
        sim.set_event_log(log, 120)
        sim.step(0.0, 100, 1)
        st = sim.stats()
        assert st["n_active"] == int(work["cells"]["cell_start"][-1])
        assert st["max_cell"] == 1024
        glog = log.cpu().numpy().reshape(nc, 120, 4)
        assert compare_logs(oout["log"], oout["stats"], glog) == []
        g = dev["m"].cpu().numpy()
        assert np.max(np.abs(g - opart["m"]) / opart["m"]) <= 1e-12
        sim.close()


def test_invalid_grid_is_rejected_on_the_device_and_reported():
    api = _api()
    work = edge_size_work(events=5)
    dev = api.to_device(work["particles"])
    m0 = dev["m"].clone()
    sim = api.Simulation(work["params"], dev, precision="mixed")
    bad = api.cells_to_device(work["cells"])
    bad["order"][7] = len(work["particles"]["m"]) + 3
    say("bad member index, bounded grid")
    sim.bin(bad, max_cell=1024)            # async: accepted, validated on the device
    sim.step(0.0, 5, 1)
    with pytest.raises(api.MCDError) as e:
        sim.stats()
    assert e.value.status == -5 and "explicit cells rejected" in str(e.value)
    assert torch.equal(dev["m"], m0)       # nothing collided
    # a cell above the stated bound is rejected the same way
    sim.bin(api.cells_to_device(work["cells"]), max_cell=1000)
    sim.step(0.0, 5, 1)
    with pytest.raises(api.MCDError):
        sim.stats()
    assert torch.equal(dev["m"], m0)
    # without a bound the same grid is rejected at once
    with pytest.raises(api.MCDError) as e:
        sim.bin(bad)
    assert e.value.status == -1
    # a valid grid clears the bad-grid flag
    sim.bin(api.cells_to_device(work["cells"]), max_cell=1024)
    sim.step(0.0, 5, 1)
    st = sim.stats()
    assert st["status"] == 0 and st["device_flags"] == 0
    sim.close()


@pytest.mark.parametrize("precision,largest", [("fp64", 1536), ("mixed", 2048)])
def test_largest_cells_run_and_larger_ones_are_rejected(precision, largest):
    api = _api()
    for schedule in ("batched", "plain"):
        work = W.c4_batched(seed=5, counts=[largest + 1, 100], events=10)
        dev = api.to_device(work["particles"])
        sim = api.Simulation(work["params"], dev, precision=precision, schedule=schedule)
        with pytest.raises(api.MCDError) as e:
            sim.bin(api.cells_to_device(work["cells"]))
        assert e.value.status == -1
        msg = str(e.value)
        assert (str(largest) in msg) or ("2048" in msg), msg
        with pytest.raises(api.MCDError):
            sim.bin(api.cells_to_device(work["cells"]), max_cell=largest + 1)
        sim.close()
    # the largest cell itself: FP64 event sequence bit-exact, mixed row sums in tolerance
    work = W.c4_batched(seed=6, counts=[largest, 37], events=60)
    say("largest cell", precision, largest)
    if precision == "fp64":
        from gpu_common import run_gpu_explicit
        opart, oout = run_oracle_explicit(work, log_per_cell=60, threads=8)
        for schedule in ("batched", "plain"):
            gpart, gstats, glog = run_gpu_explicit(work, "fp64", schedule, log_per_cell=60)
            assert compare_logs(oout["log"], oout["stats"], glog) == []
            assert gstats["device_flags"] == 0
    else:
        dev = api.to_device(work["particles"])
        sim = api.Simulation(work["params"], dev, precision="mixed")
        sim.bin(api.cells_to_device(work["cells"]))
        got = sim.row_sums(largest + 37).cpu().numpy()
        cs = work["cells"]["cell_start"]
        for c in range(2):
            members = work["cells"]["order"][cs[c]:cs[c + 1]]
            _, rs = O.cell_rates(work["params"], work["cells"]["gas"][c], members,
                                 work["particles"]["m"], work["particles"]["M"])
            assert np.max(np.abs(got[cs[c]:cs[c + 1]] - rs) / rs) <= 1e-5
        sim.step(0.0, 60, 1)
        st = sim.stats()
        assert st["events"] == 120 and st["device_flags"] == 0
        sim.close()

"""The batched schedule (single-wave threshold, workgroups per compute unit)
and its autotuner: tuning leaves the particle state and counters as they
were, and every schedule gives the FP64 event sequence of the oracle."""
import numpy as np
import pytest

from paper_2507_21239_amd import workloads as W

from gpu_common import compare_logs, run_gpu_explicit, run_oracle_explicit, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# cells on both sides of every candidate threshold, including empty ones
COUNTS = [1, 0, 40, 64, 65, 128, 129, 192, 193, 256, 257, 384, 385, 512, 513, 700, 1024]
EVENTS = 150


def _work():
    return W.c4_batched(seed=21, counts=COUNTS, events=EVENTS)


def test_tune_restores_state_and_picks_a_valid_schedule():
    from paper_2507_21239_amd import api
    work = _work()
    dev = api.to_device(work["particles"])
    m0 = dev["m"].cpu().numpy().copy()
    sim = api.Simulation(work["params"], dev, precision="mixed", schedule="batched")
    sim.bin(api.cells_to_device(work["cells"]))
    say("tune", len(COUNTS), "cells")
    r = sim.tune(0.0, EVENTS)
    assert r["small_max"] in (0, 64, 128, 192, 256, 384, 512)
    assert r["grid_per_cu"] in (0, 1, 2)
    assert r["trials"] >= 2 and r["ms_best"] > 0.0 and r["ms_best"] <= r["ms_default"] * 1.0001
    st = sim.stats()
    assert st["events"] == 0 and st["steps"] == 0 and st["outcomes"] == [0, 0, 0, 0]
    assert np.array_equal(dev["m"].cpu().numpy(), m0)
    sim.step(0.0, EVENTS, 1)
    assert sim.stats()["events"] == EVENTS * sum(1 for n in COUNTS if n > 0)
    sim.close()


# FP64 records are 96 bytes: four single-wave regions of 384 fit the 160 KB
# of LDS, of 512 they do not (tested below)
@pytest.mark.parametrize("small_max,grid_per_cu", [(0, 0), (64, 1), (256, 2), (384, 0), (128, 1)])
def test_every_schedule_matches_the_oracle_fp64(small_max, grid_per_cu):
    work = _work()
    say("schedule", small_max, grid_per_cu)
    opart, oout = run_oracle_explicit(work, log_per_cell=EVENTS + 10, threads=8)
    gpart, gstats, glog = run_gpu_explicit(work, "fp64", "batched", log_per_cell=EVENTS + 10,
                                           batched_schedule=(small_max, grid_per_cu))
    assert compare_logs(oout["log"], oout["stats"], glog) == []
    assert gstats["events"] == int(oout["stats"]["events"].sum())
    rel = np.abs(gpart["m"] - opart["m"]) / opart["m"]
    assert rel.max() <= 1e-12, rel.max()
    assert gstats["device_flags"] == 0


def test_set_schedule_rejects_out_of_range():
    from paper_2507_21239_amd import api
    work = _work()
    dev = api.to_device(work["particles"])
    sim = api.Simulation(work["params"], dev, precision="fp64", schedule="batched")
    sim.bin(api.cells_to_device(work["cells"]))
    for bad in ((-1, 0), (513, 0), (256, -1), (512, 0)):
        with pytest.raises(api.MCDError):
            sim.set_schedule(*bad)
    sim.step(0.0, EVENTS, 1)    # the schedule in force before is kept
    assert sim.stats()["events"] == EVENTS * sum(1 for n in COUNTS if n > 0)
    plain = api.Simulation(work["params"], api.to_device(work["particles"]), precision="fp64",
                           schedule="plain")
    plain.bin(api.cells_to_device(work["cells"]))
    with pytest.raises(api.MCDError):
        plain.tune(0.0, EVENTS)
    sim.close()
    plain.close()

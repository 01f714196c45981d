"""The batched collision kernel exists in two variants: with the composition
mix and the event log compiled in (a launch with fractions to track or an
event log set) and without them.  Apart from those two side effects they
evaluate the same arithmetic in the same order, so on the same inputs they
must take the same events: final masses bit-identical, in both precisions,
with a fixed event count and with time-limited steps.  In the mixed form
the variant without them is also instantiated for fixed event counts only
(no waiting times) and built with another instruction schedule; the
fixed-count case compares that instantiation with the variant compiled for
either event budget."""
import numpy as np
import pytest

from paper_2507_21239_amd import workloads as W

from gpu_common import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run(work, precision, log, dt, max_events, steps, explicit):
    from paper_2507_21239_amd import api
    dev = api.to_device(work["particles"])
    sim = api.Simulation(work["params"], dev, precision=precision, schedule="batched")
    if explicit:
        counts = np.diff(work["cells"]["cell_start"])
        sim.bin(api.cells_to_device(work["cells"]), max_cell=int(counts.max()))
        n_cells = len(counts)
    else:
        sim.bin()
        n_cells = work["params"]["n_r"] * work["params"]["n_z"]
    buf = None
    if log:
        buf = torch.full((n_cells * 64 * 4,), -2, dtype=torch.int32, device="cuda")
        sim.set_event_log(buf, 64)
    sim.step(dt, max_events, steps)
    torch.cuda.synchronize()
    st = sim.stats()
    out = {k: dev[k].cpu().numpy().copy() for k in ("m", "r", "z", "active")}
    sim.close()
    return out, st["events"], buf


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_variants_take_the_same_events_fixed_count(precision):
    counts = [1, 2, 63, 64, 65, 200, 256, 257, 300, 512, 700, 1024] * 4
    work = W.c4_batched(seed=5, counts=counts, events=300)
    say("kernel variants, fixed count", precision, len(counts), "cells")
    a, ea, _ = _run(work, precision, False, 0.0, 300, 1, True)
    b, eb, buf = _run(work, precision, True, 0.0, 300, 1, True)
    assert ea == eb
    assert np.array_equal(a["m"], b["m"])
    if precision == "fp64":
        # the kernel without the log (the fixed-count instantiation) against
        # the oracle directly, on the same cells and events
        import oracle as O
        part = {k: (v.copy() if isinstance(v, np.ndarray) else v)
                for k, v in work["particles"].items()}
        O.collide_all(work["params"], work["cells"], 0, part, 0.0, 300)
        assert np.max(np.abs(a["m"] - part["m"]) / part["m"]) <= 1e-12
    # the log variant recorded events, with cell-local indices
    log = buf.view(len(counts), 64, 4).cpu().numpy()
    n = np.asarray(counts)[:, None]
    i, j = log[:, :, 0], log[:, :, 1]
    assert (i >= 0).sum() > 0
    assert np.all((i == -2) | ((i >= 0) & (i < n)))
    assert np.all((i == -2) | ((j >= -1) & (j < n)))


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_variants_take_the_same_events_time_limited(precision):
    work = W.c3_disk(seed=4, N=20_000, n_r=20, n_z=5)
    say("kernel variants, disk steps", precision)
    a, ea, _ = _run(work, precision, False, 2.0 * W.YR, 0, 3, False)
    b, eb, _ = _run(work, precision, True, 2.0 * W.YR, 0, 3, False)
    assert ea == eb
    for f in ("m", "r", "z", "active"):
        assert np.array_equal(a[f], b[f]), f

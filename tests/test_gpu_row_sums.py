"""The collision launch's own starting row sums, read back through
mcd_row_sums, against the oracle's row sums r_i = sum_j r_ij (Zsom &
Dullemond 2008; the paper, Summary), cell by cell on cells of every boundary
size of the kernel's layout, for every team shape: one-wave cells (the FP32
form adds each unordered pair once, the reverse rates riding in lane-rotated
accumulators), four-wave teams (the same over 256 lanes with partner sums
exchanged through LDS), the eight-slot kernel and the plain schedule.

Bars: FP64 within 1e-13 relative (canonical order on both sides, a few ulps
from the libraries' cbrt / pow); mixed within 1e-5 relative (FP32 pair
rates with the hardware reciprocal and square root, ~1e-7 per operation, and
FP32 sums of up to 1024 terms).  A wrong partner sum, a lane rotation off by
one or a dropped pair moves a row by about one term in n, far outside both."""
import numpy as np
import pytest

import oracle as O
from paper_2507_21239_amd import workloads as W

from gpu_common import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIZES = [1, 2, 3, 63, 64, 65, 127, 128, 129, 200, 255, 256, 257, 300, 383, 384, 385,
         511, 512, 513, 700, 1023, 1024]


def _work(seed=4):
    return W.c4_batched(seed=seed, counts=SIZES, events=1)


def _oracle_rows(work):
    cs = work["cells"]["cell_start"]
    out = np.zeros(int(cs[-1]))
    for c in range(len(cs) - 1):
        members = work["cells"]["order"][cs[c]:cs[c + 1]]
        _, rs = O.cell_rates(work["params"], work["cells"]["gas"][c], members,
                             work["particles"]["m"], work["particles"]["M"])
        out[cs[c]:cs[c + 1]] = rs
    return out


@pytest.mark.parametrize("precision,schedule,small_max,tol", [
    ("mixed", "batched", 256, 1e-5),    # one-wave cells up to 256, four-wave teams above
    ("mixed", "batched", 0, 1e-5),      # every cell on a four-wave team
    ("mixed", "batched", 64, 1e-5),
    ("mixed", "batched", 512, 1e-5),    # one-wave cells up to 512: eight slots per lane
    ("mixed", "plain", None, 1e-5),
    ("fp64", "batched", 256, 1e-13),
    ("fp64", "batched", 0, 1e-13),
    ("fp64", "plain", None, 1e-13),
])
def test_starting_row_sums_match_the_oracle(precision, schedule, small_max, tol):
    from paper_2507_21239_amd import api
    work = _work()
    ref = _oracle_rows(work)
    say("row sums", precision, schedule, small_max)
    dev = api.to_device(work["particles"])
    m0 = dev["m"].clone()
    sim = api.Simulation(work["params"], dev, precision=precision, schedule=schedule)
    sim.bin(api.cells_to_device(work["cells"]))
    if small_max is not None:
        sim.set_schedule(small_max, 0)
    got = sim.row_sums(len(ref)).cpu().numpy()
    st = sim.stats()
    assert st["events"] == 0 and st["device_flags"] == 0
    assert torch.equal(dev["m"], m0)
    rel = np.abs(got - ref) / ref
    cs = work["cells"]["cell_start"]
    for c in range(len(cs) - 1):
        worst = rel[cs[c]:cs[c + 1]].max()
        assert worst <= tol, (SIZES[c], worst)
    say("worst relative row-sum error", float(rel.max()))
    sim.close()

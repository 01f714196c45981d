"""Asynchronous particle snapshots (histories): each snapshot equals the
state at its place in the stream -- after the steps queued before it, before
the ones queued after -- bit for bit, with both staging slots reused."""
import numpy as np
import pytest

from paper_2507_21239_amd import workloads as W

from gpu_common import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _sim(precision="mixed"):
    from paper_2507_21239_amd import api
    work = W.c3_disk(seed=11, N=20_000, n_r=20, n_z=5, n_comp=8)
    dev = api.to_device(work["particles"])
    sim = api.Simulation(work["params"], dev, precision=precision, schedule="batched")
    sim.bin()
    return sim, dev


def _state(dev):
    out = {k: dev[k].cpu().numpy().copy() for k in ("r", "z", "m", "active")}
    out["comp"] = dev["comp"].cpu().numpy().copy()
    return out


def test_snapshots_match_the_state_at_their_place_in_the_stream():
    sim, dev = _sim()
    dt = 5.0 * W.YR
    snaps, refs = [], []
    say("snapshots eager and graph steps")
    for k in range(5):
        if k % 2:
            sim.step(dt, 0, 3)        # graph replay
        else:
            sim.step(dt, 0, 1)        # eager step
        snaps.append(sim.snapshot())
        refs.append(_state(dev))      # synchronous copy at the same place
    sim.step(dt, 0, 2)                # later work must not leak into the snapshots
    for s, ref in zip(snaps, refs):
        got = s.wait()
        for f in ("r", "z", "m", "active", "comp"):
            assert np.array_equal(got[f], ref[f]), f
    assert sim.stats()["steps"] == 1 + 3 + 1 + 3 + 1 + 2
    sim.close()


def test_snapshot_subsets_and_errors():
    from paper_2507_21239_amd import api
    sim, dev = _sim("fp64")
    s = sim.snapshot(fields=("m",))
    m = s.wait()["m"]
    assert np.array_equal(m, dev["m"].cpu().numpy())
    with pytest.raises(ValueError):
        sim.snapshot(fields=("r",), out=torch.empty(8, dtype=torch.uint8))
    with pytest.raises(api.MCDError):
        sim._check(sim.lib.mcd_snapshot_wait(sim.ctx, 99), "mcd_snapshot_wait")
    assert sim.lib.mcd_snapshot(sim.ctx, 0, 1, 8, None) != 0          # no fields
    assert sim.lib.mcd_snapshot(sim.ctx, 1 << 6, 1, 8, None) != 0     # unknown field
    sim.close()


def test_fp64_snapshots_match_the_oracle_state():
    """Histories against the oracle: FP64 snapshots after every pair of
    graph-replayed steps of a small disk equal the oracle's state after the
    same steps (positions and masses within 1e-11, active flags exact,
    composition within 1e-6)."""
    import oracle as O
    sim, dev = _sim("fp64")
    work = W.c3_disk(seed=11, N=20_000, n_r=20, n_z=5, n_comp=8)
    ref = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in work["particles"].items()}
    dt = 5.0 * W.YR
    snaps = []
    for k in range(3):
        say("fp64 snapshot after graph steps", 2 * k + 2)
        sim.step(dt, 0, 2)
        snaps.append(sim.snapshot())
    for k, s in enumerate(snaps):
        for st in (2 * k, 2 * k + 1):
            O.step(work["params"], ref, st, dt, 0, threads=8)
        got = s.wait()
        assert np.array_equal(got["active"], ref["active"]), k
        for f in ("r", "z", "m"):
            assert np.all(np.abs(got[f] - ref[f]) <= 1e-11 * np.abs(ref[f]) + 1e-300), (k, f)
        assert np.max(np.abs(got["comp"] - ref["comp"])) <= 1e-6, k
    sim.close()

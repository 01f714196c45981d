"""The probabilistic fragmentation criteria on the GPU: with FP64 rates the
event sequence (who collides, and whether the collision sticks or
fragments/erodes) equals the oracle's, draw for draw, for the linear ramp and
for Maxwellian collision speeds."""
import numpy as np
import pytest

from paper_2507_21239_amd import workloads as W

from gpu_common import compare_logs, run_gpu_explicit, run_oracle_explicit, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
EVENTS = 150


def _work(mode, vf):
    w = W.c4_batched(seed=5, counts=[1, 40, 130, 256, 257, 300, 700], events=EVENTS)
    w["params"].update(v_frag=vf, frag_mode=mode, frag_width=0.9)
    return w


@pytest.mark.parametrize("mode,vf", [("ramp", 300.0), ("maxwell", 300.0), ("maxwell", 100.0)])
@pytest.mark.parametrize("schedule", ["batched", "plain"])
def test_fp64_event_sequence_matches_oracle(mode, vf, schedule):
    work = _work(mode, vf)
    say("outcome variant", mode, vf, schedule)
    opart, oout = run_oracle_explicit(work, log_per_cell=EVENTS + 10, threads=8)
    oc = oout["stats"]["outcomes"].sum(axis=0)
    assert oc[0] > 0 and oc[1] + oc[2] + oc[3] > 0   # both branches are exercised
    gpart, gstats, glog = run_gpu_explicit(work, "fp64", schedule, log_per_cell=EVENTS + 10)
    assert compare_logs(oout["log"], oout["stats"], glog) == []
    assert gstats["outcomes"] == [int(x) for x in oc]
    rel = np.abs(gpart["m"] - opart["m"]) / opart["m"]
    assert rel.max() <= 1e-12
    assert gstats["device_flags"] == 0


def test_mixed_outcome_fractions_follow_the_oracle():
    work = _work("maxwell", 300.0)
    work = W.c4_batched(seed=6, counts=[200] * 64, events=EVENTS)
    work["params"].update(v_frag=300.0, frag_mode="maxwell")
    say("outcome variant mixed")
    _, oout = run_oracle_explicit(work, threads=8)
    _, gstats, _ = run_gpu_explicit(work, "mixed", "batched")
    o = oout["stats"]["outcomes"].sum(axis=0).astype(float)
    g = np.array(gstats["outcomes"], dtype=float)
    n = o.sum()
    assert g.sum() == n
    # fraction of sticking collisions: binomial standard error, 5 sigma
    po, pg = o[0] / n, g[0] / n
    se = np.sqrt(po * (1 - po) / n)
    assert abs(pg - po) <= 5 * se + 1e-9, (pg, po, se)

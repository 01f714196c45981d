"""Pins of the fragmentation criteria (outcome variants of the literature the
paper cites for its collision physics): the sharp threshold of the paper's
fragmentation velocity, a linear probability ramp below it, and Maxwellian
collision speeds whose mean is the computed relative velocity (checked
against scipy's independent Maxwell distribution)."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
from paper_2507_21239_amd import workloads as W

VF = 1000.0


def _p(mode, width=0.2):
    return W.benchmark_params(frag_mode=mode, frag_width=width, v_frag=VF, dm_max=0.0)


def test_sharp_threshold_ignores_the_extra_uniform():
    P = _p("sharp")
    for uf in (0.0, 0.3, 0.999):
        assert O.outcome(P, VF * (1 - 1e-15), 1.0, 1.0, 0.5, uf)[0] == "stick"
        assert O.outcome(P, VF, 1.0, 1.0, 0.5, uf)[0] == "frag"
    assert O.frag_probability(P, VF * 0.999) == 0.0 and O.frag_probability(P, VF) == 1.0


def test_ramp_is_linear_between_its_ends():
    w = 0.25
    P = _p("ramp", w)
    lo = (1 - w) * VF
    assert O.frag_probability(P, lo) == 0.0
    assert O.frag_probability(P, 0.5 * lo) == 0.0
    assert O.frag_probability(P, VF) == 1.0
    assert O.frag_probability(P, 2 * VF) == 1.0
    for f in (0.1, 0.5, 0.9):
        dv = lo + f * (VF - lo)
        assert abs(O.frag_probability(P, dv) - f) <= 1e-14


def test_maxwell_tail_matches_scipy():
    P = _p("maxwell")
    for dv in (30.0, 300.0, 700.0, 1000.0, 1500.0, 4000.0, 3e4):
        scale = dv * math.sqrt(math.pi / 8.0)
        # the reading: the speed distribution's mean is the computed dv
        assert abs(stats.maxwell.mean(scale=scale) - dv) <= 1e-12 * dv
        ref = stats.maxwell.sf(VF, scale=scale)
        got = O.frag_probability(P, dv)
        assert abs(got - ref) <= 1e-13 + 1e-12 * ref, (dv, got, ref)
    assert O.frag_probability(P, 0.0) == 0.0
    assert O.frag_probability(P, 1e9) == pytest.approx(1.0, abs=1e-12)
    # monotone in dv
    ps = [O.frag_probability(P, dv) for dv in np.geomspace(10, 1e5, 200)]
    assert all(b >= a for a, b in zip(ps, ps[1:]))


@pytest.mark.parametrize("mode", ["ramp", "maxwell"])
def test_decision_uses_the_uniform_against_the_probability(mode):
    P = _p(mode, 0.4)
    dv = 0.9 * VF
    pf = O.frag_probability(P, dv)
    assert 0.0 < pf < 1.0
    below, above = pf * (1 - 1e-12), min(pf * (1 + 1e-12), 1 - 1e-16)
    # equal masses: a fragmenting collision fragments, otherwise they stick
    assert O.outcome(P, dv, 1.0, 1.0, 0.5, below)[0] == "frag"
    assert O.outcome(P, dv, 1.0, 1.0, 0.5, above)[0] == "stick"
    # mass ratio >= 10: the fast branch erodes the larger body
    assert O.outcome(P, dv, 100.0, 1.0, 0.5, below)[0] == "erode"
    assert O.outcome(P, dv, 100.0, 1.0, 0.5, above)[0] == "stick"

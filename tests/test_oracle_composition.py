"""Pins of the oracle's composition mixing (the paper, Statement of Need:
particles carry extra properties such as their composition, followed
collision by collision).

- Hand-worked single collisions (tests/golden/composition_cases.txt) with
  grouping on, for sticking, fragmentation and both kinds of erosion: every
  (i, j) pair of a two-particle cell is reached over seeds, and the new mass
  and composition of i must equal the worked values while j stays as it was.
- Counting monomers: with the constant kernel, monomers of mass 1 and no
  grouping every mass is a whole number of monomers, and mass-weighted mixing
  keeps m * comp_A a whole number of A monomers (up to the FP32 store of the
  fractions); the fractions of each particle add to 1.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_2507_21239_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "composition_cases.txt")

SETUPS = {
    # masses in units, dm_max, kernel
    "stick": dict(m=(8.0, 1.0), dm_max=0.5, kernel="constant"),
    "frag": dict(m=(4.0, 2.0), dm_max=0.75, kernel="physical"),
    "erode": dict(m=(20.0, 1.0), dm_max=0.1, kernel="physical"),
}


def _cases():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            setup, i, j, oc, mnew, ca, cb = line.split()[:7]
            out[(setup, int(i), int(j))] = (oc, mnew, float(Fraction(ca)), float(Fraction(cb)))
    return out


def _params(setup):
    s = SETUPS[setup]
    flags = ["coag"] if s["kernel"] == "constant" else ["brownian", "coag"]
    # v_frag far below every Brownian speed: physical-kernel collisions are all fast
    return W.benchmark_params(kernel=s["kernel"], k0=1.0, dm_max=s["dm_max"], flags=flags,
                              v_frag=1e-6, erosion_ratio=10.0, erosion_chi=1.0, n_comp=2)


def _unit(params, setup):
    if SETUPS[setup]["kernel"] == "constant":
        return 1.0
    return 4.0 / 3.0 * np.pi * params["a_mono"] ** 3 * params["rho_s"]


def _one_event(setup, seed):
    p = dict(_params(setup), seed=seed)
    u = _unit(p, setup)
    part = dict(r=np.zeros(2), z=np.zeros(2), m=np.array(SETUPS[setup]["m"]) * u,
                M=np.array([1.0, 1.0]) * u, active=np.ones(2, dtype=np.uint8),
                comp=np.array([[1.0, 0.0], [0.0, 1.0]], dtype=np.float32))
    cells = dict(cell_start=np.array([0, 2], dtype=np.int32), order=np.array([0, 1], dtype=np.int32),
                 gas=np.array([[1.0, 1e-10, 100.0, 1e-3, W.AU, 0.0]]))
    m_in, comp_in = part["m"].copy(), part["comp"].copy()
    out = O.collide_all(p, cells, 0, part, 0.0, 1, log_per_cell=1)
    ev = out["log"][0][0]
    return int(ev["i"]), int(ev["j"]), O.OUTCOMES[int(ev["outcome"])], part, m_in, comp_in, u


@pytest.mark.parametrize("setup", sorted(SETUPS))
def test_hand_worked_collisions(setup):
    cases = _cases()
    seen = set()
    for seed in range(400):
        i, j, oc, part, m_in, comp_in, u = _one_event(setup, seed)
        want_oc, want_m, want_a, want_b = cases[(setup, i, j)]
        assert oc == want_oc, (setup, i, j, oc)
        m_new = part["m"][i] / u
        if want_m.startswith("draw:"):
            hi = float(want_m[5:])
            assert 1.0 - 1e-12 <= m_new <= hi * (1 + 1e-12), (setup, i, j, m_new)
        else:
            assert m_new == pytest.approx(float(want_m), rel=1e-14), (setup, i, j, m_new)
        assert part["comp"][0, i] == pytest.approx(want_a, abs=1e-7), (setup, i, j)
        assert part["comp"][1, i] == pytest.approx(want_b, abs=1e-7), (setup, i, j)
        if i != j:  # only i changes
            assert part["m"][j] == m_in[j]
            assert np.array_equal(part["comp"][:, j], comp_in[:, j])
        seen.add((i, j))
    assert seen == {(0, 0), (0, 1), (1, 0), (1, 1)}, seen


def test_mixing_counts_whole_monomers():
    n = 200
    for seed in range(6):
        w = W.c1_single_cell(seed=seed, n=n, t_end=1998.0)
        p = dict(w["params"], n_comp=2)
        part = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in w["particles"].items()}
        comp = np.zeros((2, n), dtype=np.float32)
        comp[0, : n // 2] = 1.0      # species A
        comp[1, n // 2:] = 1.0       # species B
        part["comp"] = comp
        out = O.collide_all(p, w["cells"], 0, part, w["dt"], 0)
        assert out["stats"]["events"][0] > 1000
        m = part["m"]
        assert np.array_equal(m, np.rint(m))
        a = m * part["comp"][0].astype(np.float64)
        b = m * part["comp"][1].astype(np.float64)
        assert np.max(np.abs(a - np.rint(a))) < 0.05, np.max(np.abs(a - np.rint(a)))
        assert np.max(np.abs(b - np.rint(b))) < 0.05
        assert np.array_equal(np.rint(a) + np.rint(b), m)
        s = part["comp"].astype(np.float64).sum(axis=0)
        assert np.max(np.abs(s - 1.0)) < 1e-5
        # particles that never met the other species stay pure
        assert np.all((np.rint(a) > 0) | (part["comp"][0] == 0.0))

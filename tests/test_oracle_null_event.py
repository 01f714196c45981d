"""Pin of the degenerate-row rule (the reading that a particle whose stored
row sum is only rounding residue meets nobody: its row sum is cleared and
the event is a null event, logged as j = -1, outcome -1).

A three-particle cell with relative velocities from drift and settling
only, so that equal masses have zero relative velocity: one monomer and two
bodies of 16 monomers (swarm masses 1 and 3), every collision fast.  A big
body hitting the monomer's swarm erodes to 16 - 16 = 0, floored at one
monomer; the monomer hitting a big body is a fragment draw on [m0, m0].  Once
both big bodies have eroded all masses are equal, every true rate is zero and
the run must end; the monomer's row sum, updated incrementally from a + b
minus a minus b, is then left with rounding residue.  The rule must turn that
residue into null events that change nothing and end the run."""
import numpy as np

import oracle as O
from paper_2507_21239_amd import workloads as W


def null_event_work(seed: int) -> dict:
    p = W.benchmark_params(kernel="physical", dm_max=0.0,
                           flags=["radial", "azimuthal", "settling", "coag"],
                           v_frag=1e-6, erosion_ratio=10.0, erosion_chi=16.0, seed=seed)
    m0 = 4.0 / 3.0 * np.pi * p["a_mono"] ** 3 * p["rho_s"]
    part = dict(r=np.zeros(3), z=np.zeros(3), m=np.array([1.0, 16.0, 16.0]) * m0,
                M=np.array([1.0, 1.0, 3.0]), active=np.ones(3, dtype=np.uint8), comp=None)
    cells = dict(cell_start=np.array([0, 3], dtype=np.int32), order=np.array([0, 1, 2], dtype=np.int32),
                 gas=np.array([[1.0, 1e-10, 100.0, 1e-3, 5 * W.AU, 1.0]]))
    return dict(name=f"null_event[{seed}]", params=p, particles=part, cells=cells, dt=0.0,
                max_events=60, m0=m0)


def test_rounding_residue_becomes_null_events():
    with_null = 0
    for seed in range(40):
        w = null_event_work(seed)
        part = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in w["particles"].items()}
        out = O.collide_all(w["params"], w["cells"], 0, part, 0.0, w["max_events"], log_per_cell=60)
        ne = int(out["stats"]["events"][0])
        lg = out["log"][0][:ne]
        assert ne < w["max_events"]                        # the run ended by itself
        assert np.array_equal(part["m"], np.full(3, w["m0"]))  # all eroded to one monomer
        real = lg["j"] >= 0
        erosions = np.flatnonzero(real & (lg["outcome"] == 1))
        assert sorted(lg["i"][erosions].tolist()) == [1, 2]   # each big body eroded once
        last = int(erosions[-1])
        # after the second erosion every true rate is zero: only null events follow,
        # at most one per particle (each clears its row), and they change nothing
        tail = lg[last + 1:]
        assert np.all(tail["j"] == -1) and np.all(tail["outcome"] == -1)
        assert len(tail) <= 3 and len(set(tail["i"].tolist())) == len(tail)
        assert np.all(lg["j"][: last + 1] >= 0)
        assert int(out["stats"]["outcomes"][0].sum()) == last + 1
        with_null += len(tail) > 0
    assert with_null >= 10, with_null

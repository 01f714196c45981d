"""The sigma_d comparison of two benchmark-shaped runs (host code, no GPU)."""
import numpy as np
import pytest

from paper_2507_21239_amd.disk_run import compare


def _run(sigma):
    return dict(sigma=np.asarray(sigma, dtype=np.float64), m_edges=10.0 ** np.arange(5.0),
                r_edges=np.arange(3.0))


def test_identical_results_compare_as_zero():
    a = _run([[1.0, 2.0, 0.0, 1.0], [0.0, 1.0, 1.0, 0.0]])
    d = compare(a, a)
    assert d["max_cdf_gap"] == 0.0 and d["mean_log_m_diff"] == 0.0 and d["total_rel_diff"] == 0.0
    assert d["profile_median_gap"] == 0.0 and d["profile_max_gap"] == 0.0


def test_mass_moved_up_one_decade():
    # bin centres in log10 m: 0.5, 1.5, 2.5, 3.5; all of a's mass one bin above b's
    a = _run([[0.0, 2.0, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0]])
    b = _run([[2.0, 0.0, 0.0, 0.0], [0.0, 1.0, 0.0, 0.0]])
    d = compare(a, b)
    assert d["mean_log_m_diff"] == pytest.approx(1.0)
    assert d["total_rel_diff"] == pytest.approx(0.0)
    assert d["max_cdf_gap"] == pytest.approx(2.0 / 3.0)
    assert d["profile_median_gap"] == pytest.approx(1.0) and d["profile_max_gap"] == pytest.approx(1.0)


def test_empty_radial_bins_are_skipped_and_bins_must_match():
    a = _run([[1.0, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 0.0]])
    b = _run([[0.0, 1.0, 0.0, 0.0], [0.0, 0.0, 0.0, 0.0]])
    assert compare(a, b)["profile_max_gap"] == pytest.approx(1.0)
    c = dict(b, m_edges=10.0 ** np.arange(1.0, 6.0))
    with pytest.raises(ValueError):
        compare(a, c)

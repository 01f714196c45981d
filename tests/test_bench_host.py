"""Host-side logic of bench.py (no GPU): the work counts behind the roofline
figures, the ensemble comparisons behind the error report, and the refusal of
more than one GPU."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_pair_evaluation_counts():
    counts = np.array([1, 64, 65, 300])
    # algorithmic: n(n+1)/2 per build plus n per event
    assert bench.pair_evals(counts, 10) == sum(n * (n + 1) / 2 + 10 * n for n in (1, 64, 65, 300))
    # executed, lane by lane: one wave (64 lanes) up to 256 particles, four above
    def one(n, events):
        if n <= 256:
            lanes, K, offs = 64, -(-n // 64), 32
        else:
            lanes, K, offs = 256, -(-n // 256), 128
        return lanes * (K * (K + 1) // 2 + offs * K * K) + events * 2 * lanes * K
    assert bench.executed_pair_evals(counts, 10) == sum(one(n, 10) for n in (1, 64, 65, 300))
    # the kernel never executes fewer evaluations than the method needs
    c = np.arange(1, 1025)
    assert bench.executed_pair_evals(c, 1000) > bench.pair_evals(c, 1000)


def _runs(rng, n_runs, shift=0.0, n=20000):
    runs = []
    for _ in range(n_runs):
        logm = rng.normal(-10.0 + shift, 1.0, n)
        m = 10.0 ** logm
        M = np.ones(n)
        runs.append({"summary": bench.swarm_summary(m, M, np.ones(n, dtype=bool)), "logm": logm,
                     "hist": bench._logm_hist(logm)})
    return runs


def test_ensemble_comparison_accepts_equal_and_flags_shifted_distributions():
    rng = np.random.default_rng(1)
    a, b = _runs(rng, 16), _runs(rng, 16)
    assert bench.compare_ensembles(a, b, "a", "b")["within_tolerance"]
    c = _runs(rng, 16, shift=0.05)
    out = bench.compare_ensembles(a, c, "a", "c")
    assert not out["within_tolerance"]
    assert abs(out["quantities"]["mass-weighted mean log10 m"]["z"]) > 3


def test_histogram_comparison_matches_the_sample_comparison():
    rng = np.random.default_rng(2)
    a, b = _runs(rng, 8), _runs(rng, 8, shift=0.01)
    for r in a + b:
        r["summary"] = np.array([r["summary"][q] for q in bench.SUMMARY_KEYS])
    hist = bench.compare_ensembles_hist(a, b, "a", "b")
    for r in a + b:
        r["summary"] = dict(zip(bench.SUMMARY_KEYS, r["summary"]))
    samp = bench.compare_ensembles(a, b, "a", "b")
    # 1e-4 dex bins: the binned KS distance is the sample one within one bin's mass
    assert abs(hist["logm_ks"]["D"] - samp["logm_ks"]["D"]) < 2e-4
    for q in bench.SUMMARY_KEYS:
        assert abs(hist["quantities"][q]["z"] - samp["quantities"][q]["z"]) < 1e-9


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_run_permutation_reference_accounts_for_run_to_run_spread():
    """Runs whose whole distribution wanders from seed to seed (as the disk's
    largest particles do): both sides draw the per-run offset from the same
    law, so they agree, although the particle-level KS p-value says
    otherwise; a real offset between the sides is still found."""
    rng = np.random.default_rng(3)

    def runs(n_runs, shift):
        out = []
        for _ in range(n_runs):
            logm = rng.normal(-10.0 + shift + rng.normal(0.0, 0.02), 1.0, 20000)
            out.append({"summary": bench.swarm_summary(10.0 ** logm, np.ones(len(logm)),
                                                         np.ones(len(logm), dtype=bool)),
                        "logm": logm})
        return out

    a, b = runs(16, 0.0), runs(16, 0.0)
    out = bench.compare_ensembles(a, b, "a", "b")
    assert out["logm_ks"]["p_particles"] < 0.01          # particles taken as independent
    assert out["logm_ks"]["p_runs_permutation"] > 0.01   # runs as the sampling unit
    assert out["within_tolerance"]
    c = runs(16, 0.06)
    assert bench.compare_ensembles(a, c, "a", "c")["logm_ks"]["p_runs_permutation"] < 0.01


def test_parts_combine_against_the_oracle(tmp_path):
    """Ensemble parts saved apart (the oracle's runs on the host, the mixed
    runs from the GPU) combine into one comparison against the oracle; a part
    set without a reference side is refused, and so is an unknown side."""
    rng = np.random.default_rng(4)

    def save(path, side, seeds, shift):
        rec = {}
        for s in seeds:
            logm = rng.normal(-10.0 + shift, 1.0, 20000)
            summ = bench.swarm_summary(10.0 ** logm, np.ones(len(logm)), np.ones(len(logm), dtype=bool))
            key = f"{side}_{s}"
            rec[key + "_summary"] = np.array([summ[q] for q in bench.SUMMARY_KEYS])
            rec[key + "_events"] = np.array(100)
            rec[key + "_wall"] = np.array(1.0)
            rec[key + "_hist"] = bench._logm_hist(logm)
        np.savez_compressed(path, years=np.array(5), **rec)

    save(tmp_path / "o.npz", "oracle", range(8), 0.0)
    save(tmp_path / "m.npz", "mixed", range(8, 16), 0.0)
    out = bench.large_disk_ensemble_combine([str(tmp_path / "o.npz"), str(tmp_path / "m.npz")])
    assert out["oracle_seeds"] == list(range(8)) and out["mixed_seeds"] == list(range(8, 16))
    assert out["within_tolerance"] and out["horizon_yr"] == 5
    assert "paired_collisions" not in out
    with pytest.raises(ValueError):
        bench.large_disk_ensemble_combine([str(tmp_path / "m.npz")])
    # the same seeds on both sides: collisions per run compared run by run
    save(tmp_path / "p.npz", "mixed", range(8), 0.0)
    out = bench.large_disk_ensemble_combine([str(tmp_path / "o.npz"), str(tmp_path / "p.npz")])
    assert out["paired_collisions"]["rel_diff_mean"] == 0.0
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--modes", "ensemble-part",
                        "--sides", "oracle,gpu"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "--sides" in r.stderr

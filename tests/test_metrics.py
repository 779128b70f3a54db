"""Association and unit conversion of the evaluation helpers, against brute
force over all pairings."""
import itertools

import numpy as np

from paper_2604_19723_amd import metrics


def test_sorted_pairing_is_optimal_on_a_line():
    rng = np.random.default_rng(0)
    for _ in range(50):
        t = rng.uniform(-60, 60, 4)
        e = t + rng.normal(0, 3, 4)
        best = min(sum((e[list(p)] - t) ** 2) for p in itertools.permutations(range(4)))
        assert abs(np.sum(metrics.associated_errors(e, t) ** 2) - best) < 1e-9


def test_hungarian_on_sphere_matches_brute_force():
    rng = np.random.default_rng(1)
    for _ in range(20):
        t = np.stack([rng.uniform(0, 360, 3), rng.uniform(0, 80, 3)], 1)
        e = t + rng.normal(0, 4, (3, 2))
        ue, ut = metrics._unit(e), metrics._unit(t)
        ang = np.rad2deg(np.arccos(np.clip(ue @ ut.T, -1, 1)))
        best = min(sum(ang[list(p), range(3)] ** 2) for p in itertools.permutations(range(3)))
        assert abs(np.sum(metrics.associated_errors(e, t) ** 2) - best) < 1e-9


def test_wrap_and_units():
    assert abs(metrics.associated_errors(np.array([[359.5, 10.0]]), np.array([[0.5, 10.0]]))[0]
               - np.rad2deg(np.arccos(np.cos(np.deg2rad(10)) ** 2 * np.cos(np.deg2rad(1))
                                      + np.sin(np.deg2rad(10)) ** 2))) < 1e-9
    grid = np.linspace(-90, 90, 1801)
    assert abs(metrics.fractional_index_to_deg(1, grid, (1801, 1), np.array([[900.5]]))[0] - 0.05) < 1e-12
    g2 = np.stack([np.repeat(np.linspace(0, 360, 361), 181), np.tile(np.linspace(0, 90, 181), 361)], 1)
    d = metrics.fractional_index_to_deg(2, g2, (361, 181), np.array([[-0.5, 20.25]]))
    assert abs(d[0, 0] - 359.5) < 1e-12 and abs(d[0, 1] - 10.125) < 1e-12


def test_accuracy_summary_counts_failures_as_unresolved():
    errs = [np.array([0.1, -0.2]), None, np.array([3.0, 0.05])]
    s = metrics.accuracy_summary(errs, resolved_deg=1.0, nboot=20)
    assert s["pairs"] == 6 and s["failed_trials"] == 1
    assert s["resolved_frac"] == 3 / 6
    # median over |e| with the failed trial's two sources at infinity: 0.05 0.1 0.2 3 inf inf
    assert s["median_deg"] == (0.2 + 3.0) / 2
    assert np.isclose(s["rmse_resolved_deg"], np.sqrt((0.01 + 0.04 + 0.0025) / 3))
    assert np.isclose(s["rmse_all_deg"], np.sqrt((0.01 + 0.04 + 9.0 + 0.0025) / 4))


def test_paired_comparison_detects_a_small_systematic_change():
    rng = np.random.default_rng(3)
    errs = [rng.normal(0, 0.01, 4) for _ in range(2000)] + [np.array([4.0, 0.0, 0.0, 0.0])] * 40
    same = metrics.compare_accuracy(errs, errs, nboot=50)
    assert same["equal_accuracy"]
    # 3 % larger errors everywhere: far inside either side's own RMSE spread
    # (outliers dominate it), caught by the paired median and resolved RMSE
    worse = metrics.compare_accuracy([e * 1.03 for e in errs], errs, nboot=50)
    assert not worse["equal"]["median_deg"] and not worse["equal"]["rmse_resolved_deg"]
    # losing resolution on 1 % of trials is caught by the resolved fraction
    lost = [np.array([5.0, 5.0, 5.0, 5.0]) if i % 100 == 0 else e for i, e in enumerate(errs)]
    assert not metrics.compare_accuracy(lost, errs, nboot=50)["equal"]["resolved_frac"]


def test_index_identity_ignores_order():
    a = np.array([[3, 1], [5, 7], [2, 2]])
    b = np.array([[1, 3], [5, 8], [2, 2]])
    assert metrics.index_identity(a, b) == 2 / 3

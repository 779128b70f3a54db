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

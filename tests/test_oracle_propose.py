"""Pins of the refinement-window oracle (oracle/propose.py): hand-built spectra
whose window maxima, edges, duplicates and thresholds are fixed by
construction, a parabola whose vertex is known, the Cauchy-Schwarz bound that
fixes the normalisation of the threshold, and exact peaks of orthogonal
sources (closed form) found through windows."""
import numpy as np
import pytest

from oracle import bartlett as ob
from oracle import propose as op

G = 181                      # 1-degree grid over [-90, 90]
TH0, STEP = -90.0, 1.0


def u_of(g):
    return np.sin(np.deg2rad(TH0 + g * STEP))


def bumps(centres, heights, G=G, floor=0.01):
    """Spectrum of separated parabolic bumps of half width 3 on a low floor."""
    P = np.full(G, floor)
    for c, h in zip(centres, heights):
        for d in range(-3, 4):
            if 0 <= c + d < G:
                P[c + d] = max(P[c + d], h - 0.02 * h * d * d)
    return P


def run(P, props, hw=5, tau=0.0, K=None, M=4, tr=4.0):
    K = len(props) if K is None else K
    return op.refine_trial(P, tr, M, np.asarray(props, float), TH0, STEP, hw, tau, K)


def test_nearest_index_inverts_the_grid():
    # every grid point's own sine maps back to it, on a fine and a coarse grid
    for G_, th0, st in [(7201, -90.0, 0.025), (181, -90.0, 1.0)]:
        g = np.arange(G_)
        u = np.sin(np.deg2rad(th0 + g * st))
        assert all(op.nearest_index(u[i], th0, st, G_) == i for i in range(G_))
    # halfway between two points of the 1-degree grid: halves go to the even index
    assert op.nearest_index(np.sin(np.deg2rad(-89.5)), TH0, STEP, G) in (0, 1)
    assert op.nearest_index(2.0, TH0, STEP, G) == G - 1 and op.nearest_index(-2.0, TH0, STEP, G) == 0


def test_windows_pick_the_bumps_in_value_order():
    P = bumps([40, 100, 150], [1.0, 3.0, 2.0])
    o = run(P, [u_of(41), u_of(98), u_of(152)])
    assert not o["fell_back"]
    assert list(o["idx"]) == [100, 150, 40]
    assert list(o["val"]) == [3.0, 2.0, 1.0]
    # symmetric bumps: the parabola through a peak and its neighbours has its vertex on the peak
    assert list(o["refined"]) == [100.0, 150.0, 40.0]
    assert o["windows"] == [(36, 46), (93, 103), (147, 157)]


def test_refinement_is_the_vertex_of_an_off_grid_parabola():
    v = 70.3                                   # true vertex between grid points
    P = np.full(G, 0.01)
    for g in range(64, 77):
        P[g] = 5.0 - 0.1 * (g - v) ** 2
    o = run(P, [u_of(72)])
    assert not o["fell_back"] and o["idx"][0] == 70
    assert abs(o["refined"][0] - v) < 1e-12


def test_window_clipped_at_a_grid_end_keeps_a_maximum_on_the_grid_end():
    P = bumps([120], [2.0])
    P[:8] = [1.5, 1.4, 1.3, 1.2, 1.1, 1.0, 0.9, 0.8]   # falling away from g = 0
    o = run(P, [-1.0, u_of(121)])
    assert o["windows"][0] == (0, 5)
    assert not o["fell_back"]
    assert list(o["idx"]) == [120, 0] and o["refined"][1] == 0.0   # no parabola on a grid end
    # the same at the other end
    Q = P[::-1].copy()
    o = run(Q, [1.0, u_of(180 - 121)])
    assert not o["fell_back"] and list(o["idx"]) == [60, 180]


def test_maximum_on_an_interior_window_edge_goes_back_to_the_full_grid():
    P = bumps([40, 110], [1.0, 3.0])
    o = run(P, [u_of(40), u_of(100)], hw=5)     # window 95..105: P rises to 105 towards the bump at 110
    assert o["fell_back"]
    i_ref, v_ref = ob.top_k(P, 2, (G, 1), 0)
    assert list(o["idx"]) == list(i_ref) == [110, 40]
    # a wider window holds the bump
    o = run(P, [u_of(40), u_of(100)], hw=12)
    assert not o["fell_back"] and list(o["idx"]) == [110, 40]
    # the lower edge too
    o = run(P, [u_of(40), u_of(120)], hw=5)     # window 115..125: maximum on 115
    assert o["fell_back"]


def test_two_windows_on_one_point_go_back():
    P = bumps([40, 100, 150], [1.0, 3.0, 2.0])
    o = run(P, [u_of(99), u_of(101), u_of(150)], K=3)
    assert o["fell_back"]
    assert list(o["idx"]) == [100, 150, 40]     # the full grid's answer


@pytest.mark.parametrize("tau,fall", [(0.3, False), (0.29999999, False), (0.30000001, True), (0.5, True)])
def test_threshold_on_both_sides_of_the_normalised_cost(tau, fall):
    # peak 0.3 with M = 4 and tr R = 4: P M / tr R = 0.3 exactly
    P = bumps([90], [0.3], floor=0.001)
    o = run(P, [u_of(90)], tau=tau, M=4, tr=4.0)
    assert o["fell_back"] is fall
    # the threshold reads P M / tr R (not P M^2 / tr R): a peak of 0.3 at
    # M = 8, tr R = 4 is 0.6, above 0.5
    o = run(P, [u_of(90)], tau=0.5, M=8, tr=4.0)
    assert not o["fell_back"]


def test_normalised_cost_is_at_most_one_and_reaches_one_for_a_single_source():
    # Cauchy-Schwarz: a^H R a <= |a|^2 lambda_max(R) <= M tr R, with equality
    # for R = a_s a_s^H at the source point
    M = 8
    pos = np.stack([np.zeros(M), (np.arange(M) - (M - 1) / 2) * 0.5, np.zeros(M)], 1)
    grid = TH0 + STEP * np.arange(G)
    A = ob.steering(pos, ob.directions(ob.GRID_ULA_DEG, grid))
    rng = np.random.default_rng(5)
    X = rng.normal(size=(M, 3 * M)) + 1j * rng.normal(size=(M, 3 * M))
    R = X @ X.conj().T / (3 * M)
    c = ob.spectrum(R, A) * M / np.trace(R).real
    assert np.all(c <= 1.0 + 1e-12) and np.all(c >= -1e-12)
    a = A[:, 73]
    Rs = np.outer(a, a.conj())
    cs = ob.spectrum(Rs, A) * M / np.trace(Rs).real
    assert abs(cs[73] - 1.0) < 1e-12
    o = run(ob.spectrum(Rs, A), [u_of(75)], tau=0.999999, M=M, tr=np.trace(Rs).real)
    assert not o["fell_back"] and o["idx"][0] == 73


def test_nan_in_a_window_or_a_proposal_goes_back():
    P = bumps([40, 100], [1.0, 3.0])
    Pn = P.copy()
    Pn[98] = np.nan                             # inside the window around 100
    assert run(Pn, [u_of(40), u_of(100)])["fell_back"]
    Pn = P.copy()
    Pn[70] = np.nan                             # outside every window: no effect
    o = run(Pn, [u_of(40), u_of(100)])
    assert not o["fell_back"] and list(o["idx"]) == [100, 40]
    o = run(P, [u_of(40), np.nan])
    assert o["fell_back"] and list(o["idx"]) == [100, 40]
    # a trial whose windows are all NaN goes back, and the full grid then has no maxima
    o = run(np.full(G, np.nan), [u_of(40)])
    assert o["fell_back"] and o["idx"][0] == -1 and np.isnan(o["val"][0])


def test_proposals_are_taken_in_ascending_order_and_only_the_first_k():
    P = bumps([40, 100, 150], [1.0, 3.0, 2.0])
    o = run(P, [u_of(150), u_of(40), u_of(100), np.nan], K=3)   # the 4th output is not a proposal
    assert not o["fell_back"] and o["windows"] == [(35, 45), (95, 105), (145, 155)]


def test_orthogonal_sources_are_found_exactly_through_windows():
    # P2 of the spectrum oracle: sources at u_2 - u_1 = 2k/M are orthogonal, so
    # the exact covariance's spectrum peaks exactly at them
    M = 16
    th_grid = -90.0 + 0.025 * np.arange(7201)
    pos = np.stack([np.zeros(M), (np.arange(M) - (M - 1) / 2) * 0.5, np.zeros(M)], 1)
    g1 = 3000
    u1 = np.sin(np.deg2rad(th_grid[g1]))
    u2 = u1 + 2 * 3 / M
    g2 = int(np.rint((np.rad2deg(np.arcsin(u2)) + 90) / 0.025))
    u2 = np.sin(np.deg2rad(th_grid[g2]))        # keep both on the grid (orthogonal to ~1e-4)
    A = ob.steering(pos, ob.directions(ob.GRID_ULA_DEG, th_grid))
    a1, a2 = A[:, g1], A[:, g2]
    R = 2.0 * np.outer(a1, a1.conj()) + 1.0 * np.outer(a2, a2.conj())
    P = ob.spectrum(R, A)
    props = np.sin(np.deg2rad(th_grid[[g1, g2]] + np.array([0.6, -0.9])))
    o = op.refine_trial(P, np.trace(R).real, M, props, -90.0, 0.025, 50, 0.2, 2)
    i_ref, v_ref = ob.top_k(P, 2, (7201, 1), 0)
    assert not o["fell_back"]
    assert list(o["idx"]) == list(i_ref) == [g1, g2]
    np.testing.assert_array_equal(o["val"], v_ref)
    np.testing.assert_array_equal(o["refined"], ob.refine(P, i_ref, (7201, 1), 0)[:, 0])


def test_batch_is_the_trials_one_by_one():
    rng = np.random.default_rng(3)
    P = np.stack([bumps([int(c) for c in rng.integers(10, 170, 2)], [1.0, 2.0]) for _ in range(5)])
    U = np.sin(np.deg2rad(rng.uniform(-80, 80, (5, 2))))
    tr = np.full(5, 4.0)
    ob_ = op.refine_batch(P, tr, 4, U, TH0, STEP, 5, 0.0, 2)
    for b in range(5):
        o = op.refine_trial(P[b], 4.0, 4, U[b], TH0, STEP, 5, 0.0, 2)
        assert list(ob_["idx"][b]) == list(o["idx"]) and ob_["fell_back"][b] == o["fell_back"]


def test_plateau_in_a_window_goes_to_its_lower_index():
    # a two-point plateau: the full-grid rule makes only its first point a
    # local maximum, and the window maximum must be that point
    P = bumps([40], [1.0])
    P[99:103] = [2.0, 3.0, 3.0, 2.0]
    assert ob.local_max_mask(P, (G, 1), 0)[100] and not ob.local_max_mask(P, (G, 1), 0)[101]
    o = run(P, [u_of(40), u_of(102)])
    assert not o["fell_back"] and list(o["idx"]) == [100, 40]

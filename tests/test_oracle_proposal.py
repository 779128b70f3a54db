"""Pins for the Gaussian-proposal oracle: the density against scipy, a hand
1-D case, region handling, and self-normalised importance sampling of a
uniform target recovering the region's moments."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import proposal as op


@pytest.mark.parametrize("d", [1, 2, 3])
def test_log_density_matches_scipy(d):
    rng = np.random.default_rng(d)
    A = rng.standard_normal((d, d))
    C = A @ A.T + 0.5 * np.eye(d)
    mu = rng.standard_normal(d)
    p = rng.standard_normal((7, d)) * 2
    np.testing.assert_allclose(op.log_gauss(p, mu, C), stats.multivariate_normal(mu, C).logpdf(p).reshape(-1),
                               rtol=1e-12, atol=1e-12)


def test_hand_one_dimensional():
    # mu 10, sigma 2: particles mu + 2 z; weight proportional to 1 / N(p) = sqrt(2 pi) 2 exp(z^2 / 2)
    z = np.array([[0.0], [1.0], [-2.0]])
    p, w = op.sample_and_weight(np.array([10.0]), np.array([[4.0]]), z, np.array([-90.0]), np.array([90.0]),
                                np.array([False]))
    np.testing.assert_allclose(p[:, 0], [10.0, 12.0, 6.0])
    e = np.array([1.0, math.exp(0.5), math.exp(2.0)])
    np.testing.assert_allclose(w, e / e.sum(), rtol=1e-14)


def test_region_and_wrap():
    mu = np.array([355.0, 45.0])
    C = np.diag([25.0, 400.0])
    z = np.array([[3.0, 0.0], [0.0, 3.0], [0.0, 0.0]])       # az 370 -> 10; el 105 is outside [0, 90]
    p, w = op.sample_and_weight(mu, C, z, np.array([0.0, 0.0]), np.array([360.0, 90.0]), np.array([True, False]))
    np.testing.assert_allclose(p[0], [10.0, 45.0])
    assert w[1] == 0.0
    e0, e2 = math.exp(4.5), 1.0
    np.testing.assert_allclose(w[[0, 2]], [e0 / (e0 + e2), e2 / (e0 + e2)], rtol=1e-14)
    _, w_none = op.sample_and_weight(np.array([0.0]), np.array([[1.0]]), np.array([[50.0]]), np.array([-1.0]),
                                     np.array([1.0]), np.array([False]))
    assert np.isnan(w_none).all()


def test_degenerate_covariance():
    p, w = op.sample_and_weight(np.array([1.0, 2.0]), np.array([[1.0, 1.0], [1.0, 1.0]]),
                                np.ones((4, 2)), np.zeros(2), np.full(2, 90.0), np.array([False, False]))
    assert np.array_equal(p, np.tile([1.0, 2.0], (4, 1)))
    np.testing.assert_allclose(w, 0.25)


def test_importance_weights_recover_uniform_target():
    # a Gaussian proposal wider than the region: weighted moments of the
    # particles approach those of the uniform distribution on [lo, hi]
    rng = np.random.default_rng(7)
    lo, hi = -20.0, 50.0
    z = rng.standard_normal((400000, 1))
    p, w = op.sample_and_weight(np.array([5.0]), np.array([[900.0]]), z, np.array([lo]), np.array([hi]),
                                np.array([False]))
    m1 = np.sum(w * p[:, 0])
    m2 = np.sum(w * p[:, 0] ** 2)
    assert abs(m1 - (lo + hi) / 2) < 0.3
    assert abs(m2 - (lo * lo + lo * hi + hi * hi) / 3) < 15.0

"""FP64 oracle of the Gaussian birth proposal drawn from the Bartlett moments.

Test infrastructure only: the test suite, the smoke check and the CPU-baseline
leg of the benchmark call this module; the product path never does.

What the paper computes (Sec. IV-D.2): the proposal density of a new
feature's spatial parameter is a Gaussian N(mu, C) whose mean is the
Bartlett maximum and whose covariance is the spectrum-weighted second
central moment. Particles are drawn from it, and their importance weights are
proportional to the indicator of the partition the feature is searched in
divided by the proposal density (the target being uniform on that region).

Readings (the paper is silent on these):
  * the standard normal draws z are an input, so a particle is mu + L z with
    C = L L^T (Cholesky), and the proposal density at it is
    N(mu + L z; mu, C) = exp(-|z|^2 / 2) / ((2 pi)^(d/2) det L);
  * the region is the grid's extent per coordinate; an azimuth coordinate
    (grids with a wrapping first axis) is periodic, so every azimuth is
    inside and the particle is reported wrapped into [az_0, az_0 + 360);
    its density is the Gaussian at the unwrapped draw (the wrapped-normal
    images at +-360 deg are neglected);
  * weights are normalised to sum to one per trial (self-normalised
    importance sampling); a trial with no particle inside gets NaN weights;
  * a covariance that is not positive definite gives a degenerate proposal:
    every particle is mu and the weights are equal.
"""
from __future__ import annotations

import numpy as np


def cholesky_or_none(C: np.ndarray):
    """Lower Cholesky factor of C, or None when C is not positive definite."""
    C = np.asarray(C, np.float64)
    if not np.all(np.isfinite(C)):
        return None
    try:
        return np.linalg.cholesky(C)
    except np.linalg.LinAlgError:
        return None


def log_gauss(p: np.ndarray, mu: np.ndarray, C: np.ndarray) -> np.ndarray:
    """log N(p; mu, C) for rows of p, written from the definition."""
    d = mu.shape[0]
    D = np.atleast_2d(p) - mu
    Ci = np.linalg.inv(C)
    q = np.einsum("ni,ij,nj->n", D, Ci, D)
    _, logdet = np.linalg.slogdet(C)
    return -0.5 * q - 0.5 * logdet - 0.5 * d * np.log(2 * np.pi)


def sample_and_weight(mu: np.ndarray, C: np.ndarray, z: np.ndarray, lo: np.ndarray, hi: np.ndarray,
                      periodic: np.ndarray):
    """Particles [N][d] and normalised importance weights [N] for one trial.

    lo, hi: region bounds per coordinate; periodic: bool per coordinate
    (period hi - lo, always inside)."""
    mu = np.asarray(mu, np.float64)
    z = np.asarray(z, np.float64)
    N, d = z.shape
    L = cholesky_or_none(C)
    if L is None:
        return np.repeat(mu[None, :], N, axis=0), np.full(N, 1.0 / N)
    p = mu + z @ L.T
    inside = np.ones(N, dtype=bool)
    out = p.copy()
    for j in range(d):
        if periodic[j]:
            out[:, j] = lo[j] + np.mod(p[:, j] - lo[j], hi[j] - lo[j])
        else:
            inside &= (p[:, j] >= lo[j]) & (p[:, j] <= hi[j])
    logw = np.where(inside, -log_gauss(p, mu, C), -np.inf)
    if not np.any(inside):
        return out, np.full(N, np.nan)
    m = np.max(logw)
    w = np.exp(logw - m)
    return out, w / np.sum(w)

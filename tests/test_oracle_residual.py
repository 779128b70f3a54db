"""Pins for the residual-projector oracle: a hand-derived two-element case,
a closed form for orthogonal sources, a QR route and a least-squares
snapshot route (library routines the oracle's pseudo-inverse does not use),
projector identities, and exact noise-free sequential detection."""
import cmath

import numpy as np
import pytest

from oracle import bartlett as ob
from oracle import residual as orr


def ula(M, d=0.5):
    p = np.zeros((M, 3))
    p[:, 1] = (np.arange(M) - (M - 1) / 2) * d
    return p


def dirs_u(u):
    u = np.asarray(u, float)
    return np.stack([np.sqrt(1 - u * u), u, np.zeros_like(u)], 1)


def steer_u(M, u):
    return ob.steering(ula(M), dirs_u(np.atleast_1d(u)))


def fejer(M, x):
    """|a(u)^H a(u + x)|^2 for a centred half-wavelength ULA."""
    s = np.sin(np.pi * x / 2)
    return np.where(np.abs(s) < 1e-15, float(M * M), np.sin(M * np.pi * x / 2) ** 2 / np.where(s == 0, 1, s) ** 2)


def test_hand_two_elements():
    # a = [exp(-j pi u / 2), exp(+j pi u / 2)]; a a^H = [[1, e^{-j pi u}], [e^{j pi u}, 1]], |a|^2 = 2
    u = 0.3
    Pi = orr.residual_projector(steer_u(2, u))
    e = cmath.exp(1j * np.pi * u)
    want = np.array([[0.5, -0.5 / e], [-0.5 * e, 0.5]])
    np.testing.assert_allclose(Pi, want, atol=1e-15)


def test_projector_identities():
    rng = np.random.default_rng(0)
    M, S = 12, 4
    Psi = rng.standard_normal((M, S)) + 1j * rng.standard_normal((M, S))
    Pi = orr.residual_projector(Psi)
    np.testing.assert_allclose(Pi, Pi.conj().T, atol=1e-14)
    np.testing.assert_allclose(Pi @ Pi, Pi, atol=1e-13)
    np.testing.assert_allclose(Pi @ Psi, 0, atol=1e-13)
    assert abs(np.trace(Pi).real - (M - S)) < 1e-12


def test_matches_qr_route():
    rng = np.random.default_rng(1)
    M, S = 16, 5
    Psi = rng.standard_normal((M, S)) + 1j * rng.standard_normal((M, S))
    Q, _ = np.linalg.qr(Psi)
    np.testing.assert_allclose(orr.residual_projector(Psi), np.eye(M) - Q @ Q.conj().T, atol=1e-13)


def test_matches_snapshot_residuals_by_least_squares():
    # R~ = (1/T) sum_t z_t z_t^H with z_t the least-squares residual of y_t on Psi
    rng = np.random.default_rng(2)
    M, S, T = 10, 3, 7
    Psi = steer_u(M, [-0.4, 0.1, 0.55])
    Y = (rng.standard_normal((T, M)) + 1j * rng.standard_normal((T, M))) / np.sqrt(2)
    Z = np.empty_like(Y)
    for t in range(T):
        c, *_ = np.linalg.lstsq(Psi, Y[t], rcond=None)
        Z[t] = Y[t] - Psi @ c
    np.testing.assert_allclose(orr.residual_covariance(ob.covariance(Y), Psi), ob.covariance(Z), atol=1e-13)


def test_orthogonal_sources_closed_form():
    # a1, a2 orthogonal (u2 - u1 = 2k/M): projecting out a1 from
    # R = p1 a1 a1^H + p2 a2 a2^H + s I leaves p2 a2 a2^H + s (I - a1 a1^H / M), so
    # M^2 P~(u) = p2 F(u - u2) + s (M - F(u - u1) / M)
    M, u1 = 16, -0.2
    u2 = u1 + 2 * 3 / M
    p1, p2, s = 4.0, 1.5, 0.3
    a1, a2 = steer_u(M, u1)[:, 0], steer_u(M, u2)[:, 0]
    R = p1 * np.outer(a1, a1.conj()) + p2 * np.outer(a2, a2.conj()) + s * np.eye(M)
    u = np.linspace(-0.99, 0.99, 401)
    P = ob.spectrum(orr.residual_covariance(R, a1[:, None]), steer_u(M, u))
    want = (p2 * fejer(M, u - u2) + s * (M - fejer(M, u - u1) / M)) / M ** 2
    np.testing.assert_allclose(P, want, atol=1e-13)


def test_residual_spectrum_vanishes_at_projected_points():
    rng = np.random.default_rng(3)
    M, T = 16, 40
    Y = (rng.standard_normal((T, M)) + 1j * rng.standard_normal((T, M))) / np.sqrt(2)
    R = ob.covariance(Y)
    A = steer_u(M, np.linspace(-0.9, 0.9, 181))
    Rt = orr.residual_covariance(R, A[:, [20, 77, 150]])
    P = ob.spectrum(Rt, A)
    assert np.max(np.abs(P[[20, 77, 150]])) < 1e-14 * np.max(P)


def test_duplicate_and_zero_columns_add_nothing():
    M = 8
    a = steer_u(M, [0.25, -0.5])
    one = orr.residual_projector(a)
    dup = orr.residual_projector(np.concatenate([a, a[:, :1], np.zeros((M, 1))], axis=1))
    np.testing.assert_allclose(dup, one, atol=1e-13)
    assert list(orr.independent_columns(np.concatenate([a, a[:, :1]], axis=1))) == [0, 1]
    np.testing.assert_allclose(orr.residual_projector(np.zeros((M, 2))), np.eye(M))


def test_sequential_detection_noise_free_orthogonal():
    # orthogonal sources on grid points: pass k finds the k-th strongest exactly,
    # with the value equal to its power
    M = 16
    G = 321
    u = np.linspace(-1.0, 1.0, G)                       # step 1/160 = (2/M) / 20
    A = steer_u(M, u)
    gi = np.array([60, 100, 200, 260])                  # u spacings multiples of 2/M
    assert np.allclose(((u[gi] - u[gi[0]]) * M / 2) % 1, 0)
    pw = np.array([1.0, 3.0, 0.5, 2.0])
    R = sum(p * np.outer(A[:, g], A[:, g].conj()) for p, g in zip(pw, gi))
    out = orr.sequential_peaks(R, A, 4, (G, 1), 0)
    order = np.argsort(-pw)
    assert list(out["idx"]) == list(gi[order])
    np.testing.assert_allclose(out["val"], pw[order], rtol=1e-12)
    # the other sources sit at double zeros of the kernel, so their pull on the
    # parabola is second order; the last pass sees one source alone
    np.testing.assert_allclose(out["refined"][:, 0], gi[order], atol=1e-3)
    assert abs(out["refined"][-1, 0] - gi[order][-1]) < 1e-9


def test_sequential_first_pass_is_plain_top1():
    rng = np.random.default_rng(4)
    M, T, G = 8, 30, 97
    Y = (rng.standard_normal((T, M)) + 1j * rng.standard_normal((T, M))) / np.sqrt(2)
    R = ob.covariance(Y)
    A = steer_u(M, np.linspace(-1, 1, G))
    out = orr.sequential_peaks(R, A, 3, (G, 1), 0)
    i, v = ob.top_k(ob.spectrum(R, A), 1, (G, 1), 0)
    assert out["idx"][0] == i[0] and out["val"][0] == v[0]
    assert len(set(out["idx"])) == 3

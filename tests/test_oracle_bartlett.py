"""Pins for the FP64 Bartlett oracle: closed forms, library special cases,
invariants, hand-derived values and brute force on tiny inputs. None of these
re-runs the oracle's own formula; each would fail on a plausible slip in it
(a dropped conjugate, a transposed covariance, a wrong sign or normalisation,
a wrong tie rule)."""
import cmath
import json
import math
import os

import numpy as np
import pytest

from oracle import bartlett as ob

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ula(M, d=0.5):
    p = np.zeros((M, 3))
    p[:, 1] = (np.arange(M) - (M - 1) / 2) * d
    return p


def ula_dirs_from_u(u):
    u = np.asarray(u, float)
    return np.stack([np.sqrt(1 - u * u), u, np.zeros_like(u)], 1)


def rand_cov(rng, M, T):
    Y = (rng.standard_normal((T, M)) + 1j * rng.standard_normal((T, M))) / np.sqrt(2)
    return Y, ob.covariance(Y)


# ------------------------------------------------------------------ hand-derived golden values

def test_hand_m2_t1_golden():
    d = json.load(open(os.path.join(GOLDEN, "hand_m2_t1.json")))
    y = np.array(d["y_re"]) + 1j * np.array(d["y_im"])
    A = ob.steering(np.array(d["pos_wl"]), ob.directions(ob.GRID_ULA_DEG, np.array(d["theta_deg"])))
    P = ob.spectrum(ob.covariance(y[None, :]), A)
    np.testing.assert_allclose(P, d["P"], atol=1e-15)
    np.testing.assert_allclose(ob.spectrum_snapshots(y[None, :], A), d["P"], atol=1e-15)


# ------------------------------------------------------------------ P1 closed form, one source

@pytest.mark.parametrize("M", [4, 16, 64])
def test_single_source_fejer_closed_form(M):
    """R = p a_s a_s^H exactly; P(u) = p F_M(u - u_s) / M^2 with the Fejer kernel
    F_M(x) = sin^2(M pi x / 2) / sin^2(pi x / 2) for half-wavelength spacing."""
    p, th_s = 2.5, 17.3
    theta = np.linspace(-90, 90, 1801)
    A = ob.steering(ula(M), ob.directions(ob.GRID_ULA_DEG, theta))
    a_s = ob.steering(ula(M), ob.directions(ob.GRID_ULA_DEG, [th_s]))[:, 0]
    R = p * np.outer(a_s, a_s.conj())
    P = ob.spectrum(R, A)
    x = np.sin(np.deg2rad(theta)) - np.sin(np.deg2rad(th_s))
    with np.errstate(invalid="ignore", divide="ignore"):
        F = np.sin(M * np.pi * x / 2) ** 2 / np.sin(np.pi * x / 2) ** 2
    F[np.abs(x) < 1e-12] = M * M
    np.testing.assert_allclose(P, p * F / M ** 2, atol=1e-12 * p)
    # value at the source is p exactly
    Ps = ob.spectrum(R, a_s[:, None])
    assert abs(Ps[0] - p) < 1e-12
    # the top peak is the grid point nearest in u (main lobe is monotone in |du|)
    idx, val = ob.top_k(P, 1, (len(theta), 1))
    assert idx[0] == np.argmin(np.abs(x))


# ------------------------------------------------------------------ P2 orthogonal sources

def test_orthogonal_sources_exact_peaks():
    M = 16
    u1 = -0.3
    u2 = u1 + 2 * 2 / M                      # a_1^H a_2 = 0
    # a grid uniform in u that contains both sources exactly
    u = -0.9 + 0.001 * np.arange(1801)
    i1, i2 = int(round((u1 + 0.9) / 0.001)), int(round((u2 + 0.9) / 0.001))
    u[i1], u[i2] = u1, u2
    A = ob.steering(ula(M), ula_dirs_from_u(u))
    a1, a2 = A[:, i1], A[:, i2]
    assert abs(np.vdot(a1, a2)) < 1e-12
    p1, p2 = 1.0, 0.6
    R = p1 * np.outer(a1, a1.conj()) + p2 * np.outer(a2, a2.conj())
    P = ob.spectrum(R, A)
    assert abs(P[i1] - p1) < 1e-13 and abs(P[i2] - p2) < 1e-13
    idx, val = ob.top_k(P, 2, (len(u), 1))
    assert list(idx) == [i1, i2]


# ------------------------------------------------------------------ P3 Hermitian / PSD invariants

def test_hermitian_psd_bounds():
    rng = np.random.default_rng(3)
    M, T = 12, 7                                   # T < M: rank deficient on purpose
    Y, R = rand_cov(rng, M, T)
    assert np.max(np.abs(R - R.conj().T)) < 1e-15
    lam = np.linalg.eigvalsh(R)
    assert lam.min() > -1e-13
    theta = np.linspace(-90, 90, 721)
    A = ob.steering(ula(M), ob.directions(ob.GRID_ULA_DEG, theta))
    P = ob.spectrum(R, A)
    assert np.all(P >= -1e-15)
    assert np.max(np.abs(ob.spectrum_imag(R, A))) < 1e-12 * P.max()
    assert P.max() <= lam.max() / M * (1 + 1e-12)


# ------------------------------------------------------------------ P4 route equivalence

def test_covariance_and_snapshot_routes_agree():
    rng = np.random.default_rng(4)
    M, T = 24, 40
    Y, R = rand_cov(rng, M, T)
    A = ob.steering(ula(M), ob.directions(ob.GRID_ULA_DEG, np.linspace(-90, 90, 901)))
    Pc, Ps = ob.spectrum(R, A), ob.spectrum_snapshots(Y, A)
    assert np.max(np.abs(Pc - Ps)) <= 1e-13 * Pc.max()


# ------------------------------------------------------------------ P5 library special cases

def _coarray(R):
    M = R.shape[0]
    r = np.zeros(2 * M - 1, complex)
    for m in range(M):
        for n in range(M):
            r[(n - m) + M - 1] += R[m, n]
    return r                               # r[d + M - 1], d = n - m


@pytest.mark.parametrize("M,N", [(8, 15), (8, 64), (16, 31)])
def test_fft_identity_uniform_u(M, N):
    """On u_k = -1 + 2k/N, M^2 P(u_k) = sum_d (-1)^d r_d exp(j 2 pi d k / N),
    r_d = sum_{n - m = d} R_mn: one inverse FFT of length N >= 2M - 1."""
    rng = np.random.default_rng(5)
    Y, R = rand_cov(rng, M, 9)
    u = -1 + 2 * np.arange(N) / N
    P = ob.spectrum(R, ob.steering(ula(M), ula_dirs_from_u(u)))
    r = _coarray(R)
    c = np.zeros(N, complex)
    for d in range(-(M - 1), M):
        c[d % N] += (-1) ** abs(d) * r[d + M - 1]
    ref = (N * np.fft.ifft(c)).real / M ** 2
    np.testing.assert_allclose(P, ref, atol=1e-12 * P.max())


@pytest.mark.parametrize("M,N", [(8, 8), (8, 21), (5, 40)])
def test_trace_identity_uniform_u(M, N):
    """(1/N) sum_k M^2 P(u_k) = tr R for N >= M (the off-diagonal lags sum to zero
    over a full period)."""
    rng = np.random.default_rng(6)
    Y, R = rand_cov(rng, M, 3)
    u = -1 + 2 * np.arange(N) / N
    P = ob.spectrum(R, ob.steering(ula(M), ula_dirs_from_u(u)))
    assert abs(np.mean(P) * M * M - np.trace(R).real) < 1e-12 * np.trace(R).real


def test_eigen_route():
    rng = np.random.default_rng(7)
    M = 10
    Y, R = rand_cov(rng, M, 30)
    A = ob.steering(ula(M), ob.directions(ob.GRID_ULA_DEG, np.linspace(-90, 90, 181)))
    lam, V = np.linalg.eigh(R)
    ref = np.sum(lam[:, None] * np.abs(V.conj().T @ A) ** 2, axis=0) / M ** 2
    np.testing.assert_allclose(ob.spectrum(R, A), ref, atol=1e-13 * ref.max())


def test_ura_kronecker_factorisation():
    """Horizontal URA: a(u) = a_x(u_x) (x) a_y(u_y) (Supplement S-II Kronecker form),
    so a^H R a with R = R_x (x) R_y factorises into the two 1-D quadratic forms."""
    rng = np.random.default_rng(8)
    nx, ny = 4, 5
    px = (np.arange(nx) - (nx - 1) / 2) * 0.5
    py = (np.arange(ny) - (ny - 1) / 2) * 0.5
    pos = np.zeros((nx * ny, 3))
    pos[:, 0] = np.repeat(px, ny)
    pos[:, 1] = np.tile(py, nx)
    _, Rx = rand_cov(rng, nx, 6)
    _, Ry = rand_cov(rng, ny, 6)
    az = rng.uniform(0, 360, 50)
    el = rng.uniform(0, 90, 50)
    grid = np.stack([az, el], 1)
    d = ob.directions(ob.GRID_AZEL_DEG, grid)
    P = ob.spectrum(np.kron(Rx, Ry), ob.steering(pos, d))
    ax = np.exp(2j * np.pi * np.outer(px, d[:, 0]))
    ay = np.exp(2j * np.pi * np.outer(py, d[:, 1]))
    qx = np.sum(ax.conj() * (Rx @ ax), 0).real
    qy = np.sum(ay.conj() * (Ry @ ay), 0).real
    np.testing.assert_allclose(P, qx * qy / (nx * ny) ** 2, rtol=1e-11)


# ------------------------------------------------------------------ P6 invariances

def test_per_point_phase_and_phase_centre_invariance():
    rng = np.random.default_rng(9)
    M = 16
    Y, R = rand_cov(rng, M, 20)
    d = ob.directions(ob.GRID_ULA_DEG, np.linspace(-90, 90, 361))
    A = ob.steering(ula(M), d)
    P = ob.spectrum(R, A)
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, A.shape[1]))
    np.testing.assert_allclose(ob.spectrum(R, A * ph[None, :]), P, atol=1e-13 * P.max())
    shifted = ula(M) + np.array([0.3, -7.25, 1.1])           # move the phase centre
    np.testing.assert_allclose(ob.spectrum(R, ob.steering(shifted, d)), P, atol=1e-12 * P.max())


def test_scale_permutation_rotation_mirror():
    rng = np.random.default_rng(10)
    M, T = 9, 13
    Y, R = rand_cov(rng, M, T)
    theta = np.linspace(-90, 90, 181)
    A = ob.steering(ula(M), ob.directions(ob.GRID_ULA_DEG, theta))
    P = ob.spectrum(R, A)
    c = 1.7 - 0.4j
    np.testing.assert_allclose(ob.spectrum(ob.covariance(c * Y), A), abs(c) ** 2 * P, rtol=1e-12)
    perm = rng.permutation(T)
    rot = np.exp(1j * rng.uniform(0, 2 * np.pi, T))[:, None]
    np.testing.assert_allclose(ob.covariance(Y[perm] * rot), R, atol=1e-14)
    # mirror: P_{conj R}(t) = P_R(-t); the grid is symmetric so -t is the reversed grid
    np.testing.assert_allclose(ob.spectrum(R.conj(), A), P[::-1], atol=1e-13 * P.max())


# ------------------------------------------------------------------ P7 brute force

@pytest.mark.parametrize("M,T,G", [(1, 1, 5), (2, 1, 7), (3, 2, 11), (4, 3, 16)])
def test_brute_force_tiny(M, T, G):
    rng = np.random.default_rng(100 + M)
    pos = rng.uniform(-2, 2, (M, 3))                 # arbitrary geometry
    dirs = rng.standard_normal((G, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    Y = rng.standard_normal((T, M)) + 1j * rng.standard_normal((T, M))
    P = ob.spectrum(ob.covariance(Y), ob.steering(pos, ob.directions(ob.GRID_DIRS, dirs)))
    for g in range(G):
        a = [cmath.exp(2j * math.pi * sum(pos[m][c] * dirs[g][c] for c in range(3))) for m in range(M)]
        acc = 0j
        for m in range(M):
            for n in range(M):
                r_mn = sum(Y[t][m] * Y[t][n].conjugate() for t in range(T)) / T
                acc += a[m].conjugate() * r_mn * a[n]
        # and the snapshot form, |a^H y_t|^2 averaged
        snap = sum(abs(sum(a[m].conjugate() * Y[t][m] for m in range(M))) ** 2 for t in range(T)) / T
        assert abs(P[g] - acc.real / M ** 2) < 1e-12 * max(1.0, abs(acc))
        assert abs(P[g] - snap / M ** 2) < 1e-12 * max(1.0, snap)


# ------------------------------------------------------------------ peak rule, hand cases

def test_peaks_1d_plateau_endpoints_ties():
    sh = lambda P: (len(P), 1)
    P = np.array([0.0, 1.0, 1.0, 0.0])
    assert list(np.nonzero(ob.local_max_mask(P, sh(P)))[0]) == [1]   # plateau -> lowest index
    P = np.array([2.0, 1.0, 3.0])
    assert list(np.nonzero(ob.local_max_mask(P, sh(P)))[0]) == [0, 2]  # both endpoints
    idx, val = ob.top_k(P, 2, sh(P))
    assert list(idx) == [2, 0] and list(val) == [3.0, 2.0]
    P = np.array([1.0, 5.0, 1.0, 5.0, 1.0, 4.0])
    idx, val = ob.top_k(P, 4, sh(P))                  # equal values -> lower index first
    assert list(idx[:3]) == [1, 3, 5] and idx[3] == -1 and np.isnan(val[3])
    P = np.array([1.0, 1.0, 1.0])
    assert list(np.nonzero(ob.local_max_mask(P, sh(P)))[0]) == [0]
    # every comparison with NaN is false: neither NaN nor its neighbours are maxima
    P = np.array([0.0, np.nan, 2.0, 1.0, 3.0, 1.0])
    assert list(np.nonzero(ob.local_max_mask(P, sh(P)))[0]) == [4]


def test_peaks_1d_wrap():
    P = np.array([3.0, 1.0, 2.0, 0.5, 2.9])
    assert list(np.nonzero(ob.local_max_mask(P, (5, 1), 1))[0]) == [0, 2]
    # wrap0 = 2: last entry duplicates the first and is ignored
    P = np.array([3.0, 1.0, 2.0, 3.5, 3.0])
    assert list(np.nonzero(ob.local_max_mask(P, (5, 1), 2))[0]) == [3]


def test_peaks_2d_hand():
    # 4 x 3 grid (dim0 = rows), no wrap
    P = np.array([[0, 0, 0],
                  [0, 5, 0],
                  [0, 0, 0],
                  [1, 0, 4]], float).reshape(-1)
    assert list(np.nonzero(ob.local_max_mask(P, (4, 3), 0))[0]) == [4, 9, 11]
    # diagonal neighbour decides
    P = np.array([[0, 0, 6],
                  [0, 5, 0],
                  [0, 0, 0]], float).reshape(-1)
    assert list(np.nonzero(ob.local_max_mask(P, (3, 3), 0))[0]) == [2]
    # plateau across rows: the earlier raster element wins
    P = np.array([[0, 7, 0],
                  [0, 7, 0],
                  [0, 0, 0]], float).reshape(-1)
    assert list(np.nonzero(ob.local_max_mask(P, (3, 3), 0))[0]) == [1]
    # wrap0 = 2: rows 0 and 3 are the same azimuth; row 3 is ignored, rows 0/2 are neighbours
    P = np.array([[0, 5, 0],
                  [0, 0, 0],
                  [0, 6, 0],
                  [9, 9, 9]], float).reshape(-1)
    assert list(np.nonzero(ob.local_max_mask(P, (4, 3), 2))[0]) == [7]


# ------------------------------------------------------------------ refinement / moments

def test_parabolic_refinement_exact_on_parabola():
    g = np.arange(50, dtype=float)
    for x0 in (20.0, 20.3, 19.51, 20.49):
        P = 10.0 - 0.3 * (g - x0) ** 2
        idx, _ = ob.top_k(P, 1, (50, 1))
        r = ob.refine(P, idx, (50, 1))
        assert abs(r[0, 0] - x0) < 1e-12
    # endpoint peak keeps offset 0
    P = np.array([5.0, 4.0, 1.0])
    r = ob.refine(P, np.array([0]), (3, 1))
    assert r[0, 0] == 0.0
    # separable 2-D: a product of two 1-D parabolas in log form is separable per axis
    i0, i1 = np.meshgrid(np.arange(9.0), np.arange(7.0), indexing="ij")
    P = 50.0 - 0.5 * (i0 - 4.2) ** 2 - 0.25 * (i1 - 2.7) ** 2
    idx, _ = ob.top_k(P.reshape(-1), 1, (9, 7))
    r = ob.refine(P.reshape(-1), idx, (9, 7))
    np.testing.assert_allclose(r[0], [4.2, 2.7], atol=1e-12)


@pytest.mark.parametrize("wrap0", [1, 2])
def test_parabolic_refinement_across_the_azimuth_wrap(wrap0):
    # a separable parabola in the wrapped azimuth distance: its vertex lies
    # between the last row and the first, so the peak row's neighbour on one
    # side is across the wrap
    s0, s1 = 12, 7
    rows = s0 - 1 if wrap0 == 2 else s0
    i0, i1 = np.meshgrid(np.arange(s0, dtype=float), np.arange(s1, dtype=float), indexing="ij")
    for x0, peak_row in ((-0.3, 0), (rows - 1 + 0.4, rows - 1), (rows - 0.49, 0)):
        d = (i0 - x0 + rows / 2.0) % rows - rows / 2.0
        P = 50.0 - 0.5 * d ** 2 - 0.25 * (i1 - 2.7) ** 2
        if wrap0 == 2:
            P[s0 - 1] = -1e9          # the duplicate row is never a neighbour
        idx, _ = ob.top_k(P.reshape(-1), 1, (s0, s1), wrap0)
        assert idx[0] // s1 == peak_row
        r = ob.refine(P.reshape(-1), idx, (s0, s1), wrap0)
        want0 = x0 if peak_row == 0 and x0 < 0 else (x0 - rows if peak_row == 0 else x0)
        np.testing.assert_allclose(r[0], [want0, 2.7], atol=1e-12)


def test_proposal_moments_on_direction_vectors():
    # mass 2 at the zenith, 1 each at polar angle a towards +x and -x: the mean is
    # the zenith and the covariance of the offsets is diag(sin^2 a, 0, (1 - cos a)^2) / 2
    a = 0.4
    dirs = np.array([[0.0, 0.0, 1.0], [np.sin(a), 0.0, np.cos(a)], [-np.sin(a), 0.0, np.cos(a)]])
    P = np.array([2.0, 1.0, 1.0])
    mu, C = ob.proposal_moments(P, ob.GRID_DIRS, dirs.reshape(-1), (3, 1))
    np.testing.assert_array_equal(mu, [0.0, 0.0, 1.0])
    want = np.diag([np.sin(a) ** 2, 0.0, (1 - np.cos(a)) ** 2]) / 2.0
    np.testing.assert_allclose(C, want, atol=1e-15)
    # random directions: rotating the grid rotates the moments (mu -> Q mu,
    # C -> Q C Q^T), and for unit vectors tr C = sum_g w_g (2 - 2 x_g . mu)
    rng = np.random.default_rng(11)
    X = rng.standard_normal((40, 3))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    P = rng.random(40)
    mu, C = ob.proposal_moments(P, ob.GRID_DIRS, X.reshape(-1), (40, 1))
    w = P / P.sum()
    assert abs(np.trace(C) - np.sum(w * (2.0 - 2.0 * (X @ mu)))) < 1e-13
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    mu2, C2 = ob.proposal_moments(P, ob.GRID_DIRS, (X @ Q.T).reshape(-1), (40, 1))
    np.testing.assert_allclose(mu2, Q @ mu, atol=1e-14)
    np.testing.assert_allclose(C2, Q @ C @ Q.T, atol=1e-14)
    assert np.all(np.linalg.eigvalsh(C) >= -1e-15)


def test_proposal_moments_closed_forms():
    theta = np.linspace(-10, 10, 21)
    P = np.zeros(21)
    P[5] = 2.0
    mu, C = ob.proposal_moments(P, ob.GRID_ULA_DEG, theta, (21, 1))
    assert mu[0] == theta[5] and C[0, 0] == 0.0
    P[15] = 2.0                                            # two equal maxima
    mu, C = ob.proposal_moments(P, ob.GRID_ULA_DEG, theta, (21, 1))
    assert mu[0] == theta[5]
    assert abs(C[0, 0] - 0.5 * (theta[15] - theta[5]) ** 2) < 1e-12
    # az differences wrap: mass at az 359 and mean at az 1 are 2 degrees apart
    grid = np.array([[1.0, 10.0], [359.0, 10.0], [180.0, 10.0]])
    P = np.array([3.0, 1.0, 0.0])
    mu, C = ob.proposal_moments(P, ob.GRID_AZEL_DEG, grid, (3, 1))
    assert list(mu) == [1.0, 10.0]
    assert abs(C[0, 0] - 0.25 * 4.0) < 1e-12 and C[1, 1] == 0.0


def test_fractional_index_to_degrees():
    theta = np.linspace(-90, 90, 1801)
    assert abs(ob.fractional_index_to_deg(ob.GRID_ULA_DEG, theta, (1801, 1), np.array([[900.5]]))[0] - 0.05) < 1e-12

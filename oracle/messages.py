"""FP64 oracle of the particle-based update messages: the MT state message
iota, the PF state message kappa, the PR existence message omega and the noise
variance message nu, evaluated at every particle-array pair.

Test infrastructure only: the test suite, the smoke check and the CPU-baseline
leg of the benchmark call this module; the product path never does.

What the paper computes (Sec. IV-C, update messages; Supplementary Sec. S-V):
each message is a complex Gaussian density CN(z_j; mu, C) of the observation
z_j of array j. Its mean and covariance are moment-matched to the Bernoulli
mixture over feature existences (proposition of Sec. IV-C), then replaced by
the particle representations of Sec. S-V:

  * iota at MT particle p (Sec. S-V, MT state update message):
      mu = sum_s zeta_s rho_s mu_s^p a_s^(j,p),
      C  = eta~ I + sum_s c_s a_s a_s^H,
      c_s = zeta_s rho_s (gamma_s^p + |mu_s^p|^2 (1 - zeta_s rho_s));
  * kappa of feature s at particle p, existence r (Sec. S-V, PF state update
    message):
      mu = r zeta_s mu_s^p a_s^(j,p) + sum_{t != s} m3_t,
      C  = r q a_s a_s^H + eta~ I + M_s M_s^H,
      q  = (gamma_s^p + |mu_s^p|^2 (1 - zeta_s)) zeta_s,
      M_s = the columns m_t of every other feature t;
  * omega of feature s, existence r (Sec. S-V, PR state update message):
      mu = r m4_s + sum_{t != s} m3_t,  C = r w_s w_s^H + eta~ I + M_s M_s^H;
  * nu at noise particle eta^(j,p) (Sec. S-V, noise variance update message):
      mu = sum_s m3_s,  C = eta^(j,p) I + M M^H over all features.

Here rho_s = sum_p w_alpha,s^p (the PF's existence probability), zeta_s =
zeta_s^(j)(r = 1), eta~ = sum_p w_xi^(j,p) eta^(j,p) (the noise prior mean),
a_s^(j,p) is the steering vector of feature s (s = 0: the line-of-sight path)
for MT particle p paired with PF particle p (the SFV/VA geometry and array
response of Secs. II-A and II-B, taken from the coherent-cost oracle), and the
particle averages are

  m_s   = rho_s zeta_s sum_p w_beta^p sqrt(gamma_s^p + |mu_s^p|^2 (1 - zeta_s rho_s)) a_s^(j,p),
  w_s   = rho_s sum_p w_beta^p sqrt(gamma_s^p + |mu_s^p|^2 (1 - rho_s)) a_s^(j,p),
  m3_s  = rho_s zeta_s sum_p w_beta^p mu_s^p a_s^(j,p),
  m4_s  = rho_s sum_p w_beta^p mu_s^p a_s^(j,p).

Readings (where the paper leaves a choice):
  * the means mu_{s,1..4} of eqs. (musnj1)-(musnj4) are represented with the
    same particle pairing and the same weights as the low-rank columns of
    Sec. S-V (their particle forms are not printed): mu_{s,1}(x^p) and
    mu_{s,2}(phi^p) use particle p's own mu_s^p a_s^(j,p), and mu_{s,3},
    mu_{s,4} are the w_beta-weighted averages m3_s, m4_s above;
  * the low-rank columns m_s and w_s are taken as printed: the factor
    rho_s zeta_s (rho_s for w_s) multiplies the particle average linearly;
  * every message is the full log-density, normalisation included (the paper
    drops det A because it cancels in the weights; it is cheap to keep).

This oracle forms each N_z x N_z covariance densely and takes the log-density
with numpy's LU-based solve and log-determinant; the matrix inversion and
determinant lemmas of Sec. S-V are the kernels' business, not the oracle's.
"""
from __future__ import annotations

import math

import numpy as np

from . import coherent as oc


def geometry(ms):
    lam = oc.C_LIGHT / ms.fc
    return (oc.frequencies(ms.n_f, ms.bandwidth), oc.ura_support(ms.n_y, lam), oc.ura_support(ms.n_z, lam))


def steering(ms, s: int, p: int, j: int) -> np.ndarray:
    """a_s^(j,p): feature s (0 = line of sight) for MT particle p paired with
    PF particle p, at array j [N_z] (Secs. II-A and II-B)."""
    f, py, pz = geometry(ms)
    sfv = None if s == 0 else ms.sfv[s, p]
    r = oc.local_vector(ms.mt_pos[p], sfv, ms.pa_pos[j], ms.pa_rot[j])
    return oc.array_response(r, f, py, pz, ms.fc)


def noise_mean(ms) -> np.ndarray:
    """eta~_j = sum_p w_xi^(j,p) eta^(j,p) [J] (Sec. S-V, definitions)."""
    return np.sum(np.asarray(ms.w_xi, np.float64) * np.asarray(ms.eta, np.float64), axis=1)


def existence(ms) -> np.ndarray:
    """rho_s = sum_p w_alpha,s^p [S] (Sec. S-V, definitions)."""
    return np.sum(np.asarray(ms.w_alpha, np.float64), axis=1)


def particle_averages(ms):
    """m_s, w_s, m3_s, m4_s, each [S][J][N_z] (Sec. S-V; readings above)."""
    S, P, J = ms.n_feat, ms.n_part, len(ms.pa_pos)
    N = ms.n_f * ms.n_y * ms.n_z
    rho = existence(ms)
    m = np.zeros((S, J, N), np.complex128)
    w = np.zeros_like(m)
    u = np.zeros_like(m)
    for s in range(S):
        for j in range(J):
            zeta = ms.zeta[s, j]
            pdd = 1.0 - zeta * rho[s]
            pd = 1.0 - rho[s]
            for p in range(P):
                a = steering(ms, s, p, j)
                g, mu = ms.gamma[s, p], ms.mu[s, p]
                m[s, j] += ms.w_beta[p] * math.sqrt(g + abs(mu) ** 2 * pdd) * a
                w[s, j] += ms.w_beta[p] * math.sqrt(g + abs(mu) ** 2 * pd) * a
                u[s, j] += ms.w_beta[p] * mu * a
            m[s, j] *= rho[s] * zeta
            w[s, j] *= rho[s]
            u[s, j] *= rho[s]
    m3 = u * np.asarray(ms.zeta, np.float64)[:, :, None]
    return m, w, m3, u


def log_cn(z: np.ndarray, mean: np.ndarray, C: np.ndarray) -> float:
    """log CN(z; mean, C) = -N log(pi) - log det C - (z - mean)^H C^{-1} (z - mean)."""
    e = np.asarray(z, np.complex128) - mean
    sign, logdet = np.linalg.slogdet(C)
    if not sign.real > 0:
        raise np.linalg.LinAlgError("covariance is not positive definite")
    quad = np.vdot(e, np.linalg.solve(C, e)).real
    return float(-len(e) * math.log(math.pi) - logdet - quad)


def mt_message(ms, parts=None, arrays=None) -> np.ndarray:
    """log iota(x^p; z_j) [len(arrays)][len(parts)] (Sec. S-V, MT state update
    message; the mean per the readings above)."""
    S, J = ms.n_feat, len(ms.pa_pos)
    parts = range(ms.n_part) if parts is None else parts
    arrays = range(J) if arrays is None else arrays
    rho, eta = existence(ms), noise_mean(ms)
    N = ms.n_f * ms.n_y * ms.n_z
    out = np.zeros((len(arrays), len(parts)))
    for jj, j in enumerate(arrays):
        for pp, p in enumerate(parts):
            mean = np.zeros(N, np.complex128)
            C = eta[j] * np.eye(N, dtype=np.complex128)
            for s in range(S):
                a = steering(ms, s, p, j)
                pe = ms.zeta[s, j] * rho[s]
                mean += pe * ms.mu[s, p] * a
                c = pe * (ms.gamma[s, p] + abs(ms.mu[s, p]) ** 2 * (1.0 - pe))
                C += c * np.outer(a, np.conj(a))
            out[jj, pp] = log_cn(ms.z[j], mean, C)
    return out


def _rest(ms, avg, s, j):
    """eta~ I + M_s M_s^H and sum_{t != s} m3_t for feature s at array j."""
    m, _, m3, _ = avg
    eta = noise_mean(ms)
    N = m.shape[2]
    A = eta[j] * np.eye(N, dtype=np.complex128)
    mean = np.zeros(N, np.complex128)
    for t in range(ms.n_feat):
        if t != s:
            A += np.outer(m[t, j], np.conj(m[t, j]))
            mean += m3[t, j]
    return A, mean


def pf_message(ms, parts=None, avg=None):
    """log kappa(phi_s^p, r = 1; z_j) [S][J][len(parts)] and log kappa(r = 0)
    [S][J] (Sec. S-V, PF state update message)."""
    S, J = ms.n_feat, len(ms.pa_pos)
    parts = range(ms.n_part) if parts is None else parts
    avg = particle_averages(ms) if avg is None else avg
    k1 = np.zeros((S, J, len(parts)))
    k0 = np.zeros((S, J))
    for s in range(S):
        for j in range(J):
            A, rest = _rest(ms, avg, s, j)
            k0[s, j] = log_cn(ms.z[j], rest, A)
            zeta = ms.zeta[s, j]
            for pp, p in enumerate(parts):
                a = steering(ms, s, p, j)
                mu = ms.mu[s, p]
                q = (ms.gamma[s, p] + abs(mu) ** 2 * (1.0 - zeta)) * zeta
                k1[s, j, pp] = log_cn(ms.z[j], rest + zeta * mu * a, A + q * np.outer(a, np.conj(a)))
    return k1, k0


def pr_message(ms, avg=None) -> np.ndarray:
    """log omega(r; z_j) [S][J][2], r = 0, 1 (Sec. S-V, PR state update message)."""
    S, J = ms.n_feat, len(ms.pa_pos)
    avg = particle_averages(ms) if avg is None else avg
    _, w, _, m4 = avg
    out = np.zeros((S, J, 2))
    for s in range(S):
        for j in range(J):
            A, rest = _rest(ms, avg, s, j)
            out[s, j, 0] = log_cn(ms.z[j], rest, A)
            out[s, j, 1] = log_cn(ms.z[j], rest + m4[s, j], A + np.outer(w[s, j], np.conj(w[s, j])))
    return out


def noise_message(ms, parts=None, arrays=None, avg=None) -> np.ndarray:
    """log nu(eta^(j,p); z_j) [len(arrays)][len(parts)] (Sec. S-V, noise
    variance update message)."""
    J = len(ms.pa_pos)
    parts = range(ms.n_part) if parts is None else parts
    arrays = range(J) if arrays is None else arrays
    avg = particle_averages(ms) if avg is None else avg
    m, _, m3, _ = avg
    N = m.shape[2]
    out = np.zeros((len(arrays), len(parts)))
    for jj, j in enumerate(arrays):
        MM = sum(np.outer(m[t, j], np.conj(m[t, j])) for t in range(ms.n_feat))
        mean = m3[:, j].sum(axis=0)
        for pp, p in enumerate(parts):
            out[jj, pp] = log_cn(ms.z[j], mean, ms.eta[j, p] * np.eye(N) + MM)
    return out

"""FP64 oracle of the paper's own birth-proposal cost: the coherent Bartlett
spectrum over J arrays for candidate surface-feature-vector (SFV) positions.

Test infrastructure only: the test suite, the smoke check and the CPU-baseline
leg of the benchmark call this module; the product path never does.

What the paper computes:
  * geometry (Sec. II-A): an SFV position s is the mirror image of the origin
    across a flat surface; the virtual anchor of array j is that array's
    position mirrored across the same surface, eq. (posPA-SB); the
    Householder matrix of eq. (house) mirrors the vector from the virtual
    anchor to the mobile terminal, and the array's rotation takes it into the
    array's local frame, eq. (rangep);
  * array response (Sec. II-B): path-loss compensated, eq. (array-response),
    times the unit-modulus response of eq. (unit-modulus-array-response): the
    Kronecker product of the delay response over the baseband frequencies,
    eq. (delay-array-response), and the spatial responses of the URA's
    horizontal and vertical element positions, eqs. (spatial-response-y/z),
    times the carrier phase of the path length;
  * cost (Sec. IV-D.2): for candidate s, the squared magnitude of the sum over
    arrays of the 1/N_z-normalised inner products between each array's
    (residual) observation and the steering vector of s at that array.

Readings (where the paper is silent):
  * the pilot spectrum is flat, S(f) = 1 (the paper assumes unit modulus);
  * the N_f baseband frequencies are equally spaced over the bandwidth and
    symmetric around zero, f_k = (k - (N_f - 1)/2) B / (N_f - 1);
  * the inverse of a rotation is its transpose;
  * the element index of a steering vector runs frequency slowest, then the
    horizontal element, then the vertical one (the Kronecker order b (x) a_y
    (x) a_z).
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299792458.0


def householder(s: np.ndarray) -> np.ndarray:
    s = np.asarray(s, np.float64)
    return np.eye(3) - 2.0 * np.outer(s, s) / float(s @ s)


def virtual_anchor(p_pa: np.ndarray, s: np.ndarray) -> np.ndarray:
    s = np.asarray(s, np.float64)
    return np.asarray(p_pa, np.float64) - (2.0 * float(p_pa @ s) / float(s @ s) - 1.0) * s


def local_vector(p_mt, s, p_pa, rot) -> np.ndarray:
    """Vector from array j to the (virtual) source in the array's frame;
    s = None is the line-of-sight path."""
    p_mt = np.asarray(p_mt, np.float64)
    p_pa = np.asarray(p_pa, np.float64)
    rot = np.asarray(rot, np.float64)
    if s is None:
        return rot.T @ (p_mt - p_pa)
    return rot.T @ (householder(s) @ (p_mt - virtual_anchor(p_pa, s)))


def frequencies(n_f: int, bandwidth: float) -> np.ndarray:
    if n_f == 1:
        return np.zeros(1)
    return (np.arange(n_f) - (n_f - 1) / 2.0) * (bandwidth / (n_f - 1))


def ura_support(n: int, wavelength: float) -> np.ndarray:
    """Element positions of one URA axis at half-wavelength spacing, centred."""
    return (np.arange(n) - (n - 1) / 2.0) * (wavelength / 2.0)


def array_response(r: np.ndarray, f_base: np.ndarray, p_y: np.ndarray, p_z: np.ndarray, fc: float,
                   unit_modulus: bool = False) -> np.ndarray:
    """psi(r) [N_f * N_y * N_z] for a local vector r."""
    r = np.asarray(r, np.float64)
    lam = C_LIGHT / fc
    d = float(np.sqrt(r @ r))
    tau = d / C_LIGHT
    el = np.arccos(r[2] / d)
    az = np.arctan2(r[1], r[0])
    b = np.exp(-2j * np.pi * f_base * tau)
    a_y = np.exp(2j * np.pi / lam * p_y * np.sin(el) * np.sin(az))
    a_z = np.exp(2j * np.pi / lam * p_z * np.cos(el))
    psi = np.kron(b, np.kron(a_y, a_z)) * np.exp(-2j * np.pi / C_LIGHT * fc * d)
    if unit_modulus:
        return psi
    return lam / np.sqrt(4 * np.pi) / (np.sqrt(4 * np.pi) * d) * psi


def steering(p_mt, s, pas, rots, f_base, p_y, p_z, fc) -> np.ndarray:
    """Steering vectors of candidate s at every array: [J][N_z]."""
    return np.stack([array_response(local_vector(p_mt, s, pas[j], rots[j]), f_base, p_y, p_z, fc)
                     for j in range(len(pas))])


def coherent_cost(Z: np.ndarray, Psi: np.ndarray) -> float:
    """|sum_j (1/N_z) z_j^H psi_j|^2 for observations Z [J][N_z]."""
    Z = np.asarray(Z, np.complex128)
    n_z = Z.shape[1]
    return float(abs(np.sum(np.conj(Z) * Psi) / n_z) ** 2)


def coherent_spectrum(Z, candidates, p_mt, pas, rots, f_base, p_y, p_z, fc) -> np.ndarray:
    """The cost for every candidate SFV position [N_g][3]."""
    return np.array([coherent_cost(Z, steering(p_mt, s, pas, rots, f_base, p_y, p_z, fc)) for s in candidates])

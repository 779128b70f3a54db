"""FP64 oracle of the residual projector and of project-out-and-rescan detection.

Test infrastructure only: the test suite, the smoke check and the CPU-baseline
leg of the benchmark call this module; the product path never does.

What the paper computes (Sec. IV-D.2, "An Efficient Birth Proposal PDF"):
before the Bartlett cost is evaluated, the observation is replaced by its
residual, the component orthogonal to the span of the steering vectors of
the features already known (the line-of-sight and legacy features),

    z~ = Pi_perp z,   Pi_perp = I - Psi Psi^+   (Psi^+ the pseudo-inverse).

With T snapshots the residuals' sample covariance is

    R~ = (1/T) sum_t Pi_perp y_t y_t^H Pi_perp^H = Pi_perp R Pi_perp,

since Pi_perp is Hermitian. The residual Bartlett spectrum is the usual
spectrum of R~.

Sequential detection (a reading: the paper projects out known features once;
applying the same step to the sources found so far gives the classical
project-out-and-rescan search): pass 0 takes the largest local maximum of
the plain spectrum; pass k projects out the steering vectors of the k points
found so far, recomputes the spectrum of the residual covariance, and takes
its largest local maximum. Outputs are in detection order.

Numerical rank: a column whose component orthogonal to the earlier kept
columns has squared norm at most RANK_EPS times its own squared norm is
treated as dependent and adds nothing to the span (exact duplicates are the
case that matters: projecting out the same direction twice).
"""
from __future__ import annotations

import numpy as np

from oracle import bartlett as ob

RANK_EPS = 1e-10


def independent_columns(Psi: np.ndarray) -> np.ndarray:
    """Indices of the columns kept under the numerical-rank rule, in order."""
    Psi = np.asarray(Psi, np.complex128)
    kept = []
    for s in range(Psi.shape[1]):
        a = Psi[:, s]
        n2 = float(np.vdot(a, a).real)
        if n2 == 0.0:
            continue
        if kept:
            B = Psi[:, kept]
            # least-squares fit of a on the kept columns; the residual is the
            # orthogonal component
            c, *_ = np.linalg.lstsq(B, a, rcond=None)
            r = a - B @ c
        else:
            r = a
        if float(np.vdot(r, r).real) > RANK_EPS * n2:
            kept.append(s)
    return np.array(kept, dtype=np.int64)


def residual_projector(Psi: np.ndarray) -> np.ndarray:
    """Pi_perp = I - Psi Psi^+ over the independent columns of Psi [M][S]."""
    Psi = np.asarray(Psi, np.complex128)
    M = Psi.shape[0]
    keep = independent_columns(Psi)
    if len(keep) == 0:
        return np.eye(M, dtype=np.complex128)
    B = Psi[:, keep]
    return np.eye(M, dtype=np.complex128) - B @ np.linalg.pinv(B)


def residual_covariance(R: np.ndarray, Psi: np.ndarray) -> np.ndarray:
    """R~ = Pi_perp R Pi_perp for one trial."""
    Pi = residual_projector(Psi)
    return Pi @ np.asarray(R, np.complex128) @ Pi


def sequential_peaks(R: np.ndarray, A: np.ndarray, K: int, shape, wrap0: int = 0) -> dict:
    """K passes of project-out-and-rescan over the grid whose steering matrix
    is A [M][G]. Returns idx [K] (detection order, -1 when a pass finds no
    local maximum), val [K] (the residual spectrum at the point, in the pass
    that found it) and refined [K][ndim] (parabolic vertex on that pass's
    spectrum)."""
    s1 = int(shape[1])
    ndim = 1 if s1 == 1 else 2
    idx = np.full(K, -1, dtype=np.int64)
    val = np.full(K, np.nan)
    ref = np.full((K, ndim), np.nan)
    found = []
    for k in range(K):
        Rk = residual_covariance(R, A[:, found]) if found else np.asarray(R, np.complex128)
        Pk = ob.spectrum(Rk, A)
        i, v = ob.top_k(Pk, 1, shape, wrap0)
        if i[0] < 0:
            continue
        idx[k], val[k] = i[0], v[0]
        ref[k] = ob.refine(Pk, i, shape, wrap0)[0]
        found.append(int(i[0]))
    return dict(idx=idx, val=val, refined=ref)

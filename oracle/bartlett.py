"""FP64 oracle of the birth-proposal Bartlett step, read as a batched grid search.

Test infrastructure only: the test suite, the smoke check and the CPU-baseline
leg of the benchmark call this module; the product path never does.

What the paper computes (Sec. IV-D.2, "An Efficient Birth Proposal PDF"): a set
of candidates, a cost per candidate (the coherent Bartlett spectrum, the squared
magnitude of the 1/N_z-normalised inner product between the residual
observation and the candidate's steering vector, summed over arrays inside the
magnitude), weights proportional to that cost, the candidate of maximum cost as
the proposal mean, and the cost-weighted second central moment as the proposal
covariance.

Reading for one array (J = 1, N_z = M): there are no legacy features, so the
residual projector is the identity and the residual is the snapshot itself;
T snapshots carry independent source phases and are averaged incoherently:

    P(u_g) = (1/T) sum_t |a_g^H y_t|^2 / M^2 = Re(a_g^H R a_g) / M^2,
    R = (1/T) sum_t y_t y_t^H   (no mean removal, 1/T).

Steering vectors follow the unit-modulus spatial response (eq.
(spatial-response-y), eq. (spatial-response-z) and the directional-cosine form
of Supplement S-II): a_m(u) = exp(+j 2 pi p_m . u), p_m in wavelengths.

Peaks generalise the single argmax to the K largest local maxima. A point is a
local maximum when it is strictly greater than every neighbour that comes
before it in raster order and greater than or equal to every neighbour after
it; missing neighbours (grid edges without wrap) are not compared. Ties in
value go to the lower index. Parabolic refinement and the grid-unit output
are a reading beyond the paper (it keeps the raw candidate); the moments
follow the paper's weight normalisation and mode / moment matching.

Everything is complex128 / float64 numpy, written for readability, not speed.
"""
from __future__ import annotations

import numpy as np

GRID_DIRS = 0
GRID_ULA_DEG = 1
GRID_AZEL_DEG = 2


# --------------------------------------------------------------------------- geometry

def directions(grid_kind: int, grid: np.ndarray) -> np.ndarray:
    """Unit propagation directions [G][3] for a grid (directional cosines,
    Supplement S-II). ULA grids: u = (cos t, sin t, 0), t from broadside.
    Az/el grids: u = (cos el cos az, cos el sin az, sin el)."""
    g = np.asarray(grid, dtype=np.float64)
    if grid_kind == GRID_ULA_DEG:
        t = np.deg2rad(g.reshape(-1))
        return np.stack([np.cos(t), np.sin(t), np.zeros_like(t)], axis=1)
    if grid_kind == GRID_AZEL_DEG:
        g = g.reshape(-1, 2)
        az, el = np.deg2rad(g[:, 0]), np.deg2rad(g[:, 1])
        return np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], axis=1)
    if grid_kind == GRID_DIRS:
        return g.reshape(-1, 3).copy()
    raise ValueError("unknown grid kind %r" % grid_kind)


def steering(pos_wl: np.ndarray, dirs: np.ndarray) -> np.ndarray:
    """Steering matrix A [M][G], A[m, g] = exp(+j 2 pi p_m . u_g)."""
    return np.exp(2j * np.pi * (np.asarray(pos_wl, np.float64) @ np.asarray(dirs, np.float64).T))


# --------------------------------------------------------------------------- covariance / spectrum

def covariance(Y: np.ndarray) -> np.ndarray:
    """Sample covariance of one trial. Y is snapshot-major [T][M]; returns
    R[m, n] = (1/T) sum_t y_t[m] conj(y_t[n])."""
    Y = np.asarray(Y, dtype=np.complex128)
    T = Y.shape[0]
    return (Y.T @ Y.conj()) / T


def spectrum(R: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Bartlett spectrum P[g] = Re(a_g^H R a_g) / M^2 (covariance route)."""
    M = A.shape[0]
    quad = np.sum(A.conj() * (R @ A), axis=0)
    return quad.real / (M * M)


def spectrum_imag(R: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Imaginary part of a_g^H R a_g / M^2 (zero for Hermitian R up to rounding)."""
    M = A.shape[0]
    return np.sum(A.conj() * (R @ A), axis=0).imag / (M * M)


def spectrum_snapshots(Y: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Snapshot route: P[g] = (1/T) sum_t |a_g^H y_t|^2 / M^2, Y is [T][M]."""
    M = A.shape[0]
    Z = np.asarray(Y, np.complex128).conj() @ A       # [T][G] = conj(y_t)^T a_g = conj(a_g^H y_t)
    return np.mean(np.abs(Z) ** 2, axis=0) / (M * M)


# --------------------------------------------------------------------------- peaks

def _rows(shape, wrap0):
    s0, s1 = int(shape[0]), int(shape[1])
    rows = s0 - 1 if wrap0 == 2 else s0
    return s0, s1, rows


def local_max_mask(P: np.ndarray, shape, wrap0: int = 0) -> np.ndarray:
    """Boolean mask [G] of local maxima under the raster-order rule.

    shape = (shape0, shape1), flat index g = i0*shape1 + i1; shape1 = 1 is a 1-D
    grid. wrap0: 0 no wrap; 1 dim0 periodic with period shape0; 2 dim0 periodic
    with period shape0 - 1 (its last row duplicates the first and is never a
    candidate nor a neighbour). Dim1 never wraps."""
    s0, s1, rows = _rows(shape, wrap0)
    P2 = np.asarray(P, np.float64).reshape(s0, s1)[:rows]
    mask = np.ones((rows, s1), dtype=bool)
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            if di == 0 and dj == 0:
                continue
            if s1 == 1 and dj != 0:
                continue
            earlier = di < 0 or (di == 0 and dj < 0)
            j0 = np.arange(rows) + di
            if wrap0:
                v0 = np.ones(rows, dtype=bool)
                j0 = j0 % rows
            else:
                v0 = (j0 >= 0) & (j0 < rows)
                j0 = np.clip(j0, 0, rows - 1)
            j1 = np.arange(s1) + dj
            v1 = (j1 >= 0) & (j1 < s1)
            j1 = np.clip(j1, 0, s1 - 1)
            nb = P2[j0][:, j1]
            cmp = (P2 > nb) if earlier else (P2 >= nb)
            # a missing neighbour is not compared
            mask &= cmp | ~(v0[:, None] & v1[None, :])
    # NaN is never a maximum (every comparison with NaN is false, so its
    # neighbours are not maxima either)
    mask &= ~np.isnan(P2)
    full = np.zeros((s0, s1), dtype=bool)
    full[:rows] = mask
    return full.reshape(-1)


def top_k(P: np.ndarray, K: int, shape, wrap0: int = 0):
    """K largest local maxima, by value then lower index. Missing entries are
    index -1 and value NaN."""
    P = np.asarray(P, np.float64).reshape(-1)
    cand = np.nonzero(local_max_mask(P, shape, wrap0))[0]
    order = np.lexsort((cand, -P[cand]))
    sel = cand[order][:K]
    idx = np.full(K, -1, dtype=np.int64)
    val = np.full(K, np.nan)
    idx[:len(sel)] = sel
    val[:len(sel)] = P[sel]
    return idx, val


def _parabolic(pm, p0, pp):
    den = pm - 2.0 * p0 + pp
    if den == 0.0 or not np.isfinite(den):
        return 0.0
    d = 0.5 * (pm - pp) / den
    return min(0.5, max(-0.5, d))


def refine(P: np.ndarray, idx: np.ndarray, shape, wrap0: int = 0) -> np.ndarray:
    """Parabolic vertex through each peak and its two neighbours, per axis, in
    grid units: [K][ndim] with ndim = 1 for 1-D grids and 2 otherwise. A peak on
    a non-wrapping edge keeps offset 0 on that axis; missing peaks give NaN."""
    s0, s1, rows = _rows(shape, wrap0)
    P2 = np.asarray(P, np.float64).reshape(s0, s1)
    ndim = 1 if s1 == 1 else 2
    out = np.full((len(idx), ndim), np.nan)
    for k, g in enumerate(idx):
        if g < 0:
            continue
        i0, i1 = divmod(int(g), s1)
        p0 = P2[i0, i1]
        if wrap0:
            d0 = _parabolic(P2[(i0 - 1) % rows, i1], p0, P2[(i0 + 1) % rows, i1])
        elif 0 < i0 < rows - 1:
            d0 = _parabolic(P2[i0 - 1, i1], p0, P2[i0 + 1, i1])
        else:
            d0 = 0.0
        out[k, 0] = i0 + d0
        if ndim == 2:
            if 0 < i1 < s1 - 1:
                d1 = _parabolic(P2[i0, i1 - 1], p0, P2[i0, i1 + 1])
            else:
                d1 = 0.0
            out[k, 1] = i1 + d1
    return out


# --------------------------------------------------------------------------- proposal moments

def grid_coords(grid_kind: int, grid: np.ndarray) -> np.ndarray:
    """Coordinates the proposal moments are taken in: degrees for angle grids,
    the unit vector for direction grids. [G][d]."""
    g = np.asarray(grid, np.float64)
    if grid_kind == GRID_ULA_DEG:
        return g.reshape(-1, 1)
    if grid_kind == GRID_AZEL_DEG:
        return g.reshape(-1, 2)
    return g.reshape(-1, 3)


def proposal_moments(P: np.ndarray, grid_kind: int, grid: np.ndarray, shape, wrap0: int = 0):
    """Weights w = P / sum P, mean = coordinates of the global maximum (lowest
    index among equal maxima), covariance = sum_g w_g (x_g - mu)(x_g - mu)^T
    (Sec. IV-D.2 weight normalisation, mode match and moment match). Azimuth
    differences are wrapped into [-180, 180). The duplicate row of a wrap0 = 2
    grid is left out."""
    s0, s1, rows = _rows(shape, wrap0)
    P = np.asarray(P, np.float64).reshape(-1)[:rows * s1]
    X = grid_coords(grid_kind, grid)[:rows * s1]
    w = P / np.sum(P)
    gstar = int(np.argmax(P))            # first occurrence of the maximum
    mu = X[gstar].copy()
    D = X - mu
    if grid_kind == GRID_AZEL_DEG:
        D[:, 0] = (D[:, 0] + 180.0) % 360.0 - 180.0
    C = (w[:, None] * D).T @ D
    return mu, C


# --------------------------------------------------------------------------- whole trial / batch

def grid_search(Y: np.ndarray, pos_wl: np.ndarray, grid_kind: int, grid: np.ndarray, shape,
                wrap0: int, K: int, A: np.ndarray = None) -> dict:
    """One trial: covariance, spectrum, top-K peaks, refinement."""
    if A is None:
        A = steering(pos_wl, directions(grid_kind, grid))
    R = covariance(Y)
    P = spectrum(R, A)
    idx, val = top_k(P, K, shape, wrap0)
    return dict(R=R, P=P, idx=idx, val=val, refined=refine(P, idx, shape, wrap0))


def grid_search_batch(Y: np.ndarray, pos_wl: np.ndarray, grid_kind: int, grid: np.ndarray,
                      shape, wrap0: int, K: int) -> dict:
    """B trials of the same geometry. Y is [B][T][M]."""
    A = steering(pos_wl, directions(grid_kind, grid))
    outs = [grid_search(Y[b], pos_wl, grid_kind, grid, shape, wrap0, K, A=A)
            for b in range(Y.shape[0])]
    return {k: np.stack([o[k] for o in outs]) for k in outs[0]}


def fractional_index_to_deg(grid_kind: int, grid: np.ndarray, shape, refined: np.ndarray):
    """Map fractional grid indices to degrees on uniform angle grids."""
    g = np.asarray(grid, np.float64)
    if grid_kind == GRID_ULA_DEG:
        step = (g[-1] - g[0]) / (len(g) - 1)
        return g[0] + refined[..., 0] * step
    if grid_kind == GRID_AZEL_DEG:
        s0, s1 = shape
        G2 = g.reshape(s0, s1, 2)
        az0, el0 = G2[0, 0]
        daz = (G2[-1, 0, 0] - az0) / (s0 - 1)
        delv = (G2[0, -1, 1] - el0) / (s1 - 1)
        return np.stack([(az0 + refined[..., 0] * daz) % 360.0, el0 + refined[..., 1] * delv], -1)
    raise ValueError("fractional indices have no angle meaning on a direction grid")

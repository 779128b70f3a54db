"""Host-side evaluation of grid-search estimates: grid units to degrees and
association of estimates with the true directions.

The paper associates estimates with the ground truth by the Hungarian method
and leaves missed detections and false alarms out of the error (Sec. VI-A,
caption of its estimation-error figures); on a line the optimal assignment
for a squared cost is the sorted pairing.
"""
import numpy as np

GRID_ULA_DEG = 1
GRID_AZEL_DEG = 2


def fractional_index_to_deg(grid_kind, grid, shape, refined):
    """Fractional grid indices [..., ndim] on a uniform angle grid -> degrees:
    [...] for 1-D grids, [..., 2] (az in [0, 360), el) for az/el grids."""
    g = np.asarray(grid, np.float64)
    r = np.asarray(refined, np.float64)
    if grid_kind == GRID_ULA_DEG:
        step = (g[-1] - g[0]) / (len(g) - 1)
        return g[0] + r[..., 0] * step
    if grid_kind == GRID_AZEL_DEG:
        s0, s1 = shape
        G2 = g.reshape(s0, s1, 2)
        az0, el0 = G2[0, 0]
        daz = (G2[-1, 0, 0] - az0) / (s0 - 1)
        delv = (G2[0, -1, 1] - el0) / (s1 - 1)
        return np.stack([(az0 + r[..., 0] * daz) % 360.0, el0 + r[..., 1] * delv], -1)
    raise ValueError("fractional indices have no angle meaning on this grid kind")


def _unit(azel_deg):
    a = np.deg2rad(np.asarray(azel_deg, np.float64))
    return np.stack([np.cos(a[..., 1]) * np.cos(a[..., 0]), np.cos(a[..., 1]) * np.sin(a[..., 0]),
                     np.sin(a[..., 1])], -1)


def associated_errors(est, truth):
    """Per-source errors in degrees after optimal association: signed
    differences of sorted lists on a line ([K] inputs), great-circle angles
    after a Hungarian assignment on the sphere ([K][2] (az, el) inputs)."""
    est = np.asarray(est, np.float64)
    truth = np.asarray(truth, np.float64)
    if truth.ndim == 1:
        return np.sort(est) - np.sort(truth)
    from scipy.optimize import linear_sum_assignment
    ue, ut = _unit(est), _unit(truth)
    ang = np.rad2deg(np.arccos(np.clip(ue @ ut.T, -1.0, 1.0)))
    r, c = linear_sum_assignment(ang ** 2)
    return ang[r, c]

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


_KEYS = ("median_deg", "resolved_frac", "rmse_resolved_deg", "rmse_all_deg")


def _pair_rows(errors):
    """[trials][max sources] |errors|: a trial with fewer peaks than sources
    (None) is a row of infinities; sources a trial does not have are NaN."""
    per = [None if e is None else np.abs(np.asarray(e, np.float64)).reshape(-1) for e in errors]
    n_src = max([len(e) for e in per if e is not None] or [1])
    rows = np.full((len(per), n_src), np.nan)
    for i, e in enumerate(per):
        if e is None:
            rows[i] = np.inf
        else:
            rows[i, :len(e)] = e
    return rows


def _stats(rows, sel, resolved_deg):
    """(median |e|, resolved fraction, RMSE over resolved pairs, RMSE over the
    pairs of trials with every peak found) over the trials `sel`."""
    if len(sel) == 0:
        return (np.nan,) * 4
    pairs = rows[sel].ravel()
    pairs = pairs[~np.isnan(pairs)]
    if pairs.size == 0:
        return (np.nan,) * 4
    ok = pairs <= resolved_deg
    fin = pairs[np.isfinite(pairs)]
    return (float(np.median(pairs)), float(np.mean(ok)),
            float(np.sqrt(np.mean(pairs[ok] ** 2))) if ok.any() else np.nan,
            float(np.sqrt(np.mean(fin ** 2))) if fin.size else np.nan)


def accuracy_summary(errors, resolved_deg=1.0, nboot=200, seed=0):
    """Accuracy of a set of trials that outliers do not dominate.

    errors: one entry per trial, the associated per-source errors in degrees
    (associated_errors), or None for a trial with fewer peaks than sources,
    whose sources all count as unresolved. Over (trial, source) pairs:
      median_deg         median |error| (unresolved pairs count as infinite)
      resolved_frac      fraction of pairs with |error| <= resolved_deg
      rmse_resolved_deg  RMSE over the resolved pairs
      rmse_all_deg       RMSE over the pairs of trials with every peak found
    each with a bootstrap standard error over trials (nboot resamples)."""
    rows = _pair_rows(errors)
    n = len(rows)
    out = dict(zip(_KEYS, _stats(rows, np.arange(n), resolved_deg)))
    rng = np.random.default_rng(seed)
    boots = np.array([_stats(rows, rng.integers(0, n, n), resolved_deg) for _ in range(nboot)]) \
        if n else np.full((1, 4), np.nan)
    out.update({k + "_se": float(s) for k, s in zip(_KEYS, np.nanstd(boots, axis=0))})
    out["pairs"] = int(np.sum(~np.isnan(rows)))
    out["failed_trials"] = int(sum(e is None for e in errors))
    out["resolved_deg"] = float(resolved_deg)
    return out


def compare_accuracy(errors_v, errors_ref, resolved_deg=1.0, nboot=200, seed=0):
    """A variant against the reference on the same trials (paired).

    Both summaries (accuracy_summary), their differences variant - reference,
    and the bootstrap SE of each difference with both sides resampled over the
    same trials, which is far below either side's own SE when the two agree
    trial by trial. Verdict per quantity: the median error and the RMSE over
    resolved sources are equal when |difference| <= max(1 % of the reference,
    2 paired SE); the resolved fraction when |difference| <= max(0.001,
    2 paired SE)."""
    rv, rr = _pair_rows(errors_v), _pair_rows(errors_ref)
    if len(rv) != len(rr):
        raise ValueError("paired comparison needs the same trials on both sides")
    n = len(rv)
    sv = accuracy_summary(errors_v, resolved_deg, nboot, seed)
    sr = accuracy_summary(errors_ref, resolved_deg, nboot, seed)
    rng = np.random.default_rng(seed + 1)
    d = []
    for _ in range(nboot):
        sel = rng.integers(0, n, n)
        d.append(np.subtract(_stats(rv, sel, resolved_deg), _stats(rr, sel, resolved_deg)))
    dse = np.nanstd(np.array(d), axis=0) if n else np.full(4, np.nan)
    diff = {k: sv[k] - sr[k] for k in _KEYS}
    diff_se = {k: float(s) for k, s in zip(_KEYS, dse)}
    eq = {}
    for k in ("median_deg", "rmse_resolved_deg"):
        eq[k] = bool(abs(diff[k]) <= max(0.01 * abs(sr[k]), 2.0 * diff_se[k]))
    eq["resolved_frac"] = bool(abs(diff["resolved_frac"]) <= max(0.001, 2.0 * diff_se["resolved_frac"]))
    return dict(variant=sv, reference=sr, diff=diff, diff_se=diff_se, equal=eq,
                equal_accuracy=all(eq.values()),
                rule="paired over the same trials: median error and RMSE over resolved sources "
                     "within max(1 %%, 2 paired bootstrap SE), resolved fraction within "
                     "max(0.1 pp, 2 paired SE); resolved = |error| <= %g deg" % resolved_deg)


def index_identity(idx_a, idx_b):
    """Fraction of trials whose sets of peak indices are identical (order of
    equal-valued peaks aside)."""
    a = np.sort(np.asarray(idx_a).reshape(len(idx_a), -1), axis=1)
    b = np.sort(np.asarray(idx_b).reshape(len(idx_b), -1), axis=1)
    return float(np.mean(np.all(a == b, axis=1))) if len(a) else float("nan")

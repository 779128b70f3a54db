"""FP64 oracle of the learned proposal's refinement windows and fallback rule.

Test infrastructure only: the test suite, the smoke check and the CPU-baseline
leg of the benchmark call this module; the product path never does.

The paper has no learned part (it names hybrid learned / model-based
processing as future work, Sec. VII). What a network changes is only the
candidate set of the birth proposal's mode match (Sec. IV-D.2: the candidate
of maximum cost): instead of every full-grid point, narrow windows of full-grid
points around the network's coarse directions are scored, and the trial goes
back to the full candidate set whenever the windows cannot be trusted. The
rule, step by step, for one trial of a uniform 1-D angle grid
theta_g = theta_0 + g * step, g = 0 .. G-1:

  1. Proposals are the first K network outputs, read as u_k = sin(theta_k) and
     taken in ascending order. A NaN proposal sends the trial back.
  2. Proposal k maps to the full-grid index c_k nearest to asin(u_k) (u clamped
     to [-1, 1], halves rounded to even, c clipped to the grid); its window is
     the full-grid indices c_k - hw .. c_k + hw that exist.
  3. The window maximum is the largest spectrum value in the window, ties to
     the lower index. Strictly inside a window it is a local maximum of the
     full spectrum under the full-grid peak rule (it is above its earlier
     neighbour and not below its later one); on a grid end it is one too,
     since a missing neighbour is not compared.
  4. The trial goes back to the full grid when any value in a window is NaN,
     when a window maximum lies on an end of its window that is not an end of
     the grid (the spectrum may still rise outside the window), when two
     windows select the same grid point, or when a selected value's
     normalised cost P M / tr R = a^H R a / (M tr R), which lies in [0, 1], is
     not at least tau (a comparison with NaN is false).
  5. Otherwise the K window maxima, ordered by value with ties to the lower
     index, are the peaks, each refined by the parabolic vertex through its
     full-grid neighbours (bartlett.refine).
  6. A trial that goes back takes the full-grid top-K and its refinement
     (bartlett.top_k, bartlett.refine) on the same spectrum.

Written from the rule above; FP64 numpy, plain loops.
"""
from __future__ import annotations

import numpy as np

from . import bartlett as ob


def nearest_index(u: float, theta0: float, step: float, G: int) -> int:
    """Full-grid index nearest to asin(u) in degrees (step 2)."""
    uc = min(1.0, max(-1.0, float(u)))
    th = np.rad2deg(np.arcsin(uc))
    c = int(np.rint((th - theta0) / step))
    return min(G - 1, max(0, c))


def window_maximum(P: np.ndarray, lo: int, hi: int):
    """Largest value of P[lo..hi], ties to the lower index (step 3). Returns
    (index, value, saw_nan)."""
    best_g, best_v, saw_nan = -1, -np.inf, False
    for g in range(lo, hi + 1):
        v = float(P[g])
        if np.isnan(v):
            saw_nan = True
            continue
        if best_g < 0 or v > best_v:
            best_g, best_v = g, v
    return best_g, best_v, saw_nan


def refine_trial(P: np.ndarray, trace_R: float, M: int, u: np.ndarray, theta0: float, step: float,
                 hw: int, tau: float, K: int) -> dict:
    """One trial of the window rule on the full spectrum P [G] (only window
    points are read unless the trial goes back). u holds at least K proposals.
    Returns idx [K] int, val [K], refined [K] (grid units), fell_back bool,
    and the windows (lo, hi) in proposal order."""
    P = np.asarray(P, np.float64).reshape(-1)
    G = P.shape[0]
    props = np.asarray(u, np.float64).reshape(-1)[:K]
    windows, picks = [], []
    fall = bool(np.any(np.isnan(props)))
    if not fall:
        for uk in np.sort(props):
            c = nearest_index(uk, theta0, step, G)
            lo, hi = max(0, c - hw), min(G - 1, c + hw)
            windows.append((lo, hi))
            g, v, saw_nan = window_maximum(P, lo, hi)
            if saw_nan or g < 0:
                fall = True
                continue
            if (g == lo and g > 0) or (g == hi and g < G - 1):
                fall = True
            if not (v * M / trace_R >= tau):
                fall = True
            if any(g == gp for gp, _ in picks):
                fall = True
            picks.append((g, v))
    if fall:
        idx, val = ob.top_k(P, K, (G, 1), 0)
        ref = ob.refine(P, idx, (G, 1), 0)[:, 0]
        return dict(idx=idx, val=val, refined=ref, fell_back=True, windows=windows)
    picks.sort(key=lambda gv: (-gv[1], gv[0]))
    idx = np.array([g for g, _ in picks], dtype=np.int64)
    val = np.array([v for _, v in picks])
    ref = ob.refine(P, idx, (G, 1), 0)[:, 0]
    return dict(idx=idx, val=val, refined=ref, fell_back=False, windows=windows)


def refine_batch(P: np.ndarray, trace_R: np.ndarray, M: int, U: np.ndarray, theta0: float, step: float,
                 hw: int, tau: float, K: int) -> dict:
    """refine_trial over B trials: P [B][G], trace_R [B], U [B][>= K]."""
    outs = [refine_trial(P[b], trace_R[b], M, U[b], theta0, step, hw, tau, K) for b in range(P.shape[0])]
    return dict(idx=np.stack([o["idx"] for o in outs]), val=np.stack([o["val"] for o in outs]),
                refined=np.stack([o["refined"] for o in outs]),
                fell_back=np.array([o["fell_back"] for o in outs]))

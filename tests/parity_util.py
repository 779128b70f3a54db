"""Parity definitions shared by the GPU tests.

Spectrum gate: per trial, the normwise error e = max_g |P - P*| / max_g P*
against the FP64 oracle must stay below the precision's tolerance (1e-5 for
FP32, 1e-3 for the BF16 hi/lo split). Pointwise relative error is reported
only: near the spectrum's nulls its condition number
sum |conj(a_m) R_mn a_n| / |a^H R a| grows to thousands.

Peak gate, two parts:
  * same-precision decision: the oracle's peak rule applied to the GPU's own
    FP32 spectrum must give bit-identical indices and values, and the same FP64
    refinement (the decision is taken in the kernel's precision on both sides);
  * against the FP64 oracle: identical indices on every trial that is not a
    tie, where a tie means two candidate values (the selected ones, or the
    K-th against the best unselected one, or a peak against its grid
    neighbours) closer than 4 * tol * max P*.
"""
import numpy as np

from oracle import bartlett as ob

TOL = {1: 1e-5, 2: 1e-3, 3: 3e-2}


def normwise_err(P, Pref):
    P = np.asarray(P, np.float64)
    Pref = np.asarray(Pref, np.float64)
    return np.max(np.abs(P - Pref), axis=-1) / np.max(Pref, axis=-1)


def is_tie(Pref, K, shape, wrap0, tol):
    """Tie test on the FP64 spectrum of one trial."""
    thr = 4.0 * tol * np.max(Pref)
    mask = ob.local_max_mask(Pref, shape, wrap0)
    cand = np.nonzero(mask)[0]
    vals = np.sort(Pref[cand])[::-1]
    top = vals[:K + 1]
    if len(top) >= 2 and np.min(np.abs(np.diff(top))) <= thr:
        return True
    # near-plateau at a selected peak, or near-peaks just below the threshold of a neighbour
    idx, _ = ob.top_k(Pref, K, shape, wrap0)
    s0, s1 = shape
    rows = s0 - 1 if wrap0 == 2 else s0
    P2 = np.asarray(Pref).reshape(s0, s1)
    for g in idx:
        if g < 0:
            continue
        i0, i1 = divmod(int(g), s1)
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                if (di, dj) == (0, 0) or (s1 == 1 and dj):
                    continue
                j0, j1 = i0 + di, i1 + dj
                if wrap0:
                    j0 %= rows
                if 0 <= j0 < rows and 0 <= j1 < s1 and abs(P2[j0, j1] - P2[i0, i1]) <= thr:
                    return True
    # a non-maximum that is within thr of being one (a shoulder) can flip too
    return False


def check_peaks_same_precision(P_gpu, idx, val, refined, K, shape, wrap0):
    """Oracle peak rule on the GPU's FP32 spectrum: exact equality."""
    B = P_gpu.shape[0]
    for b in range(B):
        Pb = P_gpu[b].astype(np.float64)
        i_ref, v_ref = ob.top_k(Pb, K, shape, wrap0)
        assert np.array_equal(idx[b], i_ref), (b, idx[b], i_ref)
        np.testing.assert_array_equal(val[b], v_ref.astype(np.float32))
        if refined is not None:
            r_ref = ob.refine(Pb, i_ref, shape, wrap0)
            np.testing.assert_allclose(refined[b], r_ref, rtol=0, atol=1e-12, equal_nan=True)


def peak_agreement_fp64(P_ref, idx, K, shape, wrap0, tol):
    """Indices against the FP64 oracle; returns (n_compared, n_ties, mismatches)."""
    n_cmp, n_tie, bad = 0, 0, []
    for b in range(P_ref.shape[0]):
        if is_tie(P_ref[b], K, shape, wrap0, tol):
            n_tie += 1
            continue
        i_ref, _ = ob.top_k(P_ref[b], K, shape, wrap0)
        n_cmp += 1
        if not np.array_equal(idx[b], i_ref):
            bad.append((b, list(idx[b]), list(i_ref)))
    return n_cmp, n_tie, bad

"""Spectrum with peak candidates from the projection epilogue, merged per trial
(ba_spectrum_candidates + ba_peaks_merge, and ba_run on the plans they serve).

Gates: P bit-identical to ba_spectrum; idx, val and refined bit-identical to
ba_peaks on that P; and the oracle's peak rule on the same FP32 values gives
the same indices and values, with its FP64 refinement within 1e-12. Sizes span
one to 64 column ranges per trial, ragged chunk tails, every padded element
count of the FP32 register-resident kernel (8, 16, 32, 64) and the BF16
split kernel (two trials per workgroup), wrap0 = 0, 1 and 2, k = 1 to 16,
and degenerate spectra (all zero: one plateau; NaN)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bartlett as ob
from paper_2604_19723_amd import bartlett as bb
from paper_2604_19723_amd import workload as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"


def plan_dirs_1d(M, G, wrap0, precision=bb.BA_PREC_F32):
    """Line array along x (half-wavelength spacing), azimuth sweep as a 1-D
    direction grid; wrap0 = 2 repeats the first direction at the end."""
    az = np.linspace(0.0, 2 * np.pi, G, endpoint=(wrap0 == 2))
    dirs = np.stack([np.cos(az), np.sin(az), np.zeros_like(az)], axis=1)
    pos = np.zeros((M, 3))
    pos[:, 0] = 0.5 * np.arange(M)
    return bb.ba_plan_create(M, pos, bb.BA_GRID_DIRS, G, dirs, G, 1, wrap0, precision)


def noise_snapshots(B, T, M, seed):
    rng = np.random.default_rng(seed)
    y = rng.standard_normal((B, T, M)) + 1j * rng.standard_normal((B, T, M))
    return torch.from_numpy(y.astype(np.complex64)).to(DEV)


def staged(plan, B, R, K):
    G = plan.G
    P = torch.empty((B, G), dtype=torch.float32, device=DEV)
    bb.ba_spectrum(plan, B, R, P)
    idx = torch.empty((B, K), dtype=torch.int32, device=DEV)
    val = torch.empty((B, K), dtype=torch.float32, device=DEV)
    ref = torch.empty((B, K, 1), dtype=torch.float64, device=DEV)
    bb.ba_peaks(plan, B, P, K, idx, val, ref)
    return P, idx, val, ref


def fused(plan, B, R, K, write_p=True):
    cand = bb.candidates_for(plan, B, K, DEV)
    cand.fill_(0xFF)  # every record byte the call needs is written
    P = torch.full((B, plan.G), 7.0, dtype=torch.float32, device=DEV) if write_p else None
    bb.ba_spectrum_candidates(plan, B, R, K, P, cand)
    idx = torch.full((B, K), -7, dtype=torch.int32, device=DEV)
    val = torch.empty((B, K), dtype=torch.float32, device=DEV)
    ref = torch.empty((B, K, 1), dtype=torch.float64, device=DEV)
    bb.ba_peaks_merge(plan, B, K, cand, idx, val, ref)
    return P, idx, val, ref


def bits(t):
    a = t.cpu().numpy()
    return a.view(np.int32 if a.dtype in (np.float32, np.int32) else np.int64)


def check_against_staged_and_oracle(plan, B, R, K, wrap0, n_oracle=None):
    Ps, i_s, v_s, r_s = staged(plan, B, R, K)
    Pf, i_f, v_f, r_f = fused(plan, B, R, K)
    _, i_n, v_n, r_n = fused(plan, B, R, K, write_p=False)
    torch.cuda.synchronize()
    assert np.array_equal(bits(Pf), bits(Ps))
    for got in ((i_f, v_f, r_f), (i_n, v_n, r_n)):
        assert np.array_equal(bits(got[0]), bits(i_s))
        assert np.array_equal(bits(got[1]), bits(v_s))
        assert np.array_equal(bits(got[2]), bits(r_s))
    P_h, idx_h, val_h, ref_h = Ps.cpu().numpy(), i_f.cpu().numpy(), v_f.cpu().numpy(), r_f.cpu().numpy()
    G = plan.G
    trials = range(B) if n_oracle is None else np.unique(np.linspace(0, B - 1, n_oracle).astype(int))
    for b in trials:
        Pb = P_h[b].astype(np.float64)
        i_ref, v_ref = ob.top_k(Pb, K, (G, 1), wrap0)
        assert np.array_equal(idx_h[b], i_ref), (b, idx_h[b], i_ref)
        np.testing.assert_array_equal(val_h[b], v_ref.astype(np.float32))
        r_ref = ob.refine(Pb, i_ref, (G, 1), wrap0)
        np.testing.assert_allclose(ref_h[b, :, 0], r_ref.reshape(-1), rtol=0, atol=1e-12, equal_nan=True)
    return idx_h


@pytest.mark.parametrize("M", [3, 12, 24, 64])
@pytest.mark.parametrize("G", [1, 2, 17, 1000, 7201])
@pytest.mark.parametrize("wrap0", [0, 1, 2])
def test_candidates_match_staged_path(M, G, wrap0):
    rows = G - 1 if wrap0 == 2 else G
    if wrap0 and rows < 3:
        pytest.skip("a plan rejects a wrapping dimension with a period below 3")
    with plan_dirs_1d(M, G, wrap0) as plan:
        for B, K in ((1, 16), (5, 4), (3, 1)):
            Y = noise_snapshots(B, 2 * M, M, 7919 * M + 31 * G + wrap0 + B)
            R = torch.empty((B, M, M), dtype=torch.complex64, device=DEV)
            bb.ba_covariance(plan, B, 2 * M, Y, R)
            check_against_staged_and_oracle(plan, B, R, K, wrap0)


# One trial splits its columns into up to 64 ranges of whole 16-column chunks.
# At 64 elements, G = 33265..33267 leaves the last range 0, 1 and 2 candidate
# columns when wrap0 = 2 drops the repeated last direction (1, 2, 3 without),
# and 70 001 points reach the cap on the number of ranges.
@pytest.mark.parametrize("G", [33265, 33266, 33267, 70001])
@pytest.mark.parametrize("wrap0", [0, 2])
def test_candidates_many_ranges(G, wrap0):
    M = 64
    with plan_dirs_1d(M, G, wrap0) as plan:
        for B in (1, 3):
            Y = noise_snapshots(B, 96, M, 104729 + G + wrap0 + B)
            R = torch.empty((B, M, M), dtype=torch.complex64, device=DEV)
            bb.ba_covariance(plan, B, 96, Y, R)
            check_against_staged_and_oracle(plan, B, R, 16, wrap0)


@pytest.mark.parametrize("M", [3, 64])
@pytest.mark.parametrize("wrap0", [0, 1])
def test_candidates_degenerate_spectra(M, wrap0):
    G, B, K = 1000, 2, 4
    with plan_dirs_1d(M, G, wrap0) as plan:
        R = torch.zeros((B, M, M), dtype=torch.complex64, device=DEV)
        R[1] = float("nan")
        idx = check_against_staged_and_oracle(plan, B, R, K, wrap0)
    # zero spectrum: one plateau, whose first point is the only maximum
    # without wrap (no earlier neighbour) and no point is one with wrap
    want0 = [-1] * K if wrap0 else [0] + [-1] * (K - 1)
    assert idx[0].tolist() == want0
    assert idx[1].tolist() == [-1] * K  # NaN compares false


@pytest.mark.parametrize("precision", [bb.BA_PREC_BF16X3, bb.BA_PREC_BF16])
@pytest.mark.parametrize("M", [5, 64])
@pytest.mark.parametrize("G", [1, 2, 17, 1000, 7201])
@pytest.mark.parametrize("wrap0", [0, 1, 2])
def test_split_precision_candidates_match_staged_path(precision, M, G, wrap0):
    """The BF16 register-resident kernel (two trials per workgroup, 64-column
    windows): odd batches (a pair with one trial), one range per pair up to
    the 64-range cap, against its own staged spectrum and ba_peaks."""
    rows = G - 1 if wrap0 == 2 else G
    if wrap0 and rows < 3:
        pytest.skip("a plan rejects a wrapping dimension with a period below 3")
    with plan_dirs_1d(M, G, wrap0, precision) as plan:
        for B, K in ((1, 16), (5, 4), (2, 1)):
            Y = noise_snapshots(B, 2 * M, M, 6007 * M + 37 * G + wrap0 + B + precision)
            R = torch.empty((B, M, M), dtype=torch.complex64, device=DEV)
            bb.ba_covariance(plan, B, 2 * M, Y, R)
            check_against_staged_and_oracle(plan, B, R, K, wrap0)


def test_unsupported_plans_are_rejected():
    ts = wl.config3(1)
    with bb.plan_for(ts) as plan:   # 2-D grid
        with pytest.raises(bb.BartlettError) as e:
            bb.ba_candidates_size(plan, 1, 3)
        assert e.value.status == bb.BA_ERR_UNSUPPORTED
    with plan_dirs_1d(100, 500, 0, bb.BA_PREC_BF16X3) as plan:   # streamed kernel (more than 64 elements)
        with pytest.raises(bb.BartlettError) as e:
            bb.ba_candidates_size(plan, 1, 4)
        assert e.value.status == bb.BA_ERR_UNSUPPORTED
    with plan_dirs_1d(8, 500, 0, bb.BA_PREC_F32_VALU) as plan:   # vector-ALU reference
        with pytest.raises(bb.BartlettError) as e:
            bb.ba_candidates_size(plan, 1, 4)
        assert e.value.status == bb.BA_ERR_UNSUPPORTED


def test_run_uses_candidates_at_the_full_ula_launch():
    """10 000 ULA trials (two column ranges per trial, the bench's launch):
    ba_run without P against the staged path on every trial, the oracle's
    rule on a sample."""
    ts = wl.config2(10000)
    B, T, M, K = ts.n_trials, ts.n_snap, ts.n_elem, ts.K
    with bb.plan_for(ts) as plan:
        Y = torch.from_numpy(ts.y_c64()).to(DEV)
        out = bb.run_grid_search(plan, Y, K, with_spectrum=False)
        R = torch.empty((B, M, M), dtype=torch.complex64, device=DEV)
        bb.ba_covariance(plan, B, T, Y, R)
        Ps, i_s, v_s, r_s = staged(plan, B, R, K)
        torch.cuda.synchronize()
        assert out["P"] is None
        assert np.array_equal(bits(out["idx"]), bits(i_s))
        assert np.array_equal(bits(out["val"]), bits(v_s))
        assert np.array_equal(bits(out["refined"]), bits(r_s))
        P_h, idx_h = Ps.cpu().numpy(), out["idx"].cpu().numpy()
        for b in np.linspace(0, B - 1, 40).astype(int):
            i_ref, _ = ob.top_k(P_h[b].astype(np.float64), K, ts.grid_shape, ts.wrap0)
            assert np.array_equal(idx_h[b], i_ref), b

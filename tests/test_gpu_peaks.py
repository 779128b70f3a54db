"""Peak pick through the C-ABI on synthetic spectra, against the oracle's peak
rule on the same FP32 values (bit-exact indices and values, refinement to
1e-12). The spectra are quantised to a few levels so that plateaus and equal
values are common, and carry NaNs; 1-D rows up to 7680 candidates are staged
in LDS whole, longer rows and 2-D grids in bands of rows (2-D rows of more than
2560 points meet their neighbours in global memory), and wrap0 = 2 drops a
duplicated last row."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bartlett as ob
from paper_2604_19723_amd import bartlett as bb

pytestmark = pytest.mark.gpu
DEV = "cuda"


def plan_1d(G, wrap0):
    az = np.linspace(0.0, 2 * np.pi, G, endpoint=(wrap0 == 2))
    dirs = np.stack([np.cos(az), np.sin(az), np.zeros_like(az)], axis=1)
    pos = np.zeros((4, 3))
    pos[:, 0] = 0.5 * np.arange(4)
    return bb.ba_plan_create(4, pos, bb.BA_GRID_DIRS, G, dirs, G, 1, wrap0)


def synthetic(B, G, seed):
    rng = np.random.default_rng(seed)
    P = rng.integers(0, 6, size=(B, G)).astype(np.float32) * np.float32(0.25)
    P += rng.standard_normal((B, G)).astype(np.float32) * (rng.random((B, G)) < 0.5) * np.float32(1e-3)
    P[rng.random((B, G)) < 0.02] = np.nan
    return P


@pytest.mark.parametrize("G", [1, 2, 3, 5, 64, 257, 7201, 7680, 7681, 9000])
@pytest.mark.parametrize("wrap0", [0, 1, 2])
def test_peaks_1d_match_oracle(G, wrap0):
    rows = G - 1 if wrap0 == 2 else G
    if wrap0 and rows < 3:
        pytest.skip("a plan rejects a wrapping dimension with a period below 3")
    B = 3
    P = synthetic(B, G, 1000 * G + wrap0)
    with plan_1d(G, wrap0) as plan:
        for K in (1, 3, 16):
            idx = torch.empty((B, K), dtype=torch.int32, device=DEV)
            val = torch.empty((B, K), dtype=torch.float32, device=DEV)
            ref = torch.empty((B, K, 1), dtype=torch.float64, device=DEV)
            bb.ba_peaks(plan, B, torch.from_numpy(P).to(DEV), K, idx, val, ref)
            torch.cuda.synchronize()
            idx_h, val_h, ref_h = idx.cpu().numpy(), val.cpu().numpy(), ref.cpu().numpy()
            for b in range(B):
                Pb = P[b].astype(np.float64)
                i_ref, v_ref = ob.top_k(Pb, K, (G, 1), wrap0)
                assert np.array_equal(idx_h[b], i_ref), (G, wrap0, K, b, idx_h[b], i_ref)
                np.testing.assert_array_equal(val_h[b], v_ref.astype(np.float32))
                r_ref = ob.refine(Pb, i_ref, (G, 1), wrap0)
                np.testing.assert_allclose(ref_h[b, :, 0], r_ref.reshape(-1), rtol=0, atol=1e-12, equal_nan=True)


def plan_2d(rows0, s1, wrap0):
    """Az/el grid of rows0 x s1 points (dim 0 azimuth; wrap0 = 2 repeats the
    first azimuth as the last row)."""
    az = np.linspace(0.0, 360.0, rows0, endpoint=(wrap0 == 2))
    el = np.linspace(0.0, 60.0, s1)
    grid = np.stack(np.meshgrid(az, el, indexing="ij"), axis=-1).reshape(-1, 2)
    pos = np.zeros((4, 3))
    pos[:, 0] = 0.5 * np.arange(4)
    return bb.ba_plan_create(4, pos, bb.BA_GRID_AZEL_DEG, rows0 * s1, grid, rows0, s1, wrap0)


# 2-D grids are walked in bands of whole dim-0 rows staged in LDS with the
# rows on either side: 181 columns give bands of 40 rows (shapes on both sides
# of one and two bands, and the 361 x 181 URA grid), 2560 columns bands of a
# single row, 1920 columns bands of two; at 2561 columns no band fits and the
# points meet their neighbours in global memory.
@pytest.mark.parametrize("shape", [(3, 2), (5, 7), (40, 181), (41, 181), (42, 181), (82, 181), (361, 181),
                                   (4, 2560), (6, 1920), (4, 2561)])
@pytest.mark.parametrize("wrap0", [0, 1, 2])
def test_peaks_2d_match_oracle(shape, wrap0):
    rows0, s1 = shape
    rows = rows0 - 1 if wrap0 == 2 else rows0
    if wrap0 and rows < 3:
        pytest.skip("a plan rejects a wrapping dimension with a period below 3")
    B, G = 3, rows0 * s1
    P = synthetic(B, G, 7 * G + wrap0)
    with plan_2d(rows0, s1, wrap0) as plan:
        for K in (1, 4, 16):
            idx = torch.empty((B, K), dtype=torch.int32, device=DEV)
            val = torch.empty((B, K), dtype=torch.float32, device=DEV)
            ref = torch.empty((B, K, 2), dtype=torch.float64, device=DEV)
            bb.ba_peaks(plan, B, torch.from_numpy(P).to(DEV), K, idx, val, ref)
            torch.cuda.synchronize()
            idx_h, val_h, ref_h = idx.cpu().numpy(), val.cpu().numpy(), ref.cpu().numpy()
            for b in range(B):
                Pb = P[b].astype(np.float64)
                i_ref, v_ref = ob.top_k(Pb, K, (rows0, s1), wrap0)
                assert np.array_equal(idx_h[b], i_ref), (shape, wrap0, K, b, idx_h[b], i_ref)
                np.testing.assert_array_equal(val_h[b], v_ref.astype(np.float32))
                r_ref = ob.refine(Pb, i_ref, (rows0, s1), wrap0)
                np.testing.assert_allclose(ref_h[b], r_ref, rtol=0, atol=1e-12, equal_nan=True)

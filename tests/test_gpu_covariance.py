"""GPU parity of the sample covariance R = (1/T) sum_t y_t y_t^H (Sec. IV-D.2,
covariance form) against the FP64 oracle: every array size class (one
workgroup per trial up to 64 elements, pairs of 64-element blocks above),
snapshot counts around the 32- and 64-snapshot stages, odd sizes and
unaligned snapshot buffers (the 8-byte load route), and the 256-element URA
launch at its full batch on sampled trials."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bartlett as ob
from paper_2604_19723_amd import bartlett as bb

pytestmark = pytest.mark.gpu

DEV = "cuda"


def plan_line(M):
    """Any plan of M elements: covariance does not depend on the grid."""
    pos = np.zeros((M, 3))
    pos[:, 0] = 0.5 * np.arange(M)
    az = np.linspace(-np.pi / 2, np.pi / 2, 33)
    dirs = np.stack([np.cos(az), np.sin(az), np.zeros_like(az)], axis=1)
    return bb.ba_plan_create(M, pos, bb.BA_GRID_DIRS, 33, dirs, 33, 1, 0)


def snapshots(B, T, M, seed, offset=0):
    """Seeded complex normal snapshots [B][T][M]; offset > 0 places them that
    many complex values into a larger buffer (a start that is not 16-byte
    aligned when offset is odd)."""
    rng = np.random.default_rng(seed)
    y = (rng.standard_normal((B, T, M)) + 1j * rng.standard_normal((B, T, M))).astype(np.complex64)
    buf = torch.zeros(B * T * M + offset, dtype=torch.complex64, device=DEV)
    buf[offset:] = torch.from_numpy(y.reshape(-1)).to(DEV)
    return y, buf[offset:].view(B, T, M)


def check(R, y, tol=1e-5):
    R = R.cpu().numpy()
    for b in range(R.shape[0]):
        ref = ob.covariance(y[b].astype(np.complex128))
        e = np.max(np.abs(R[b] - ref)) / np.max(np.abs(ref))
        assert e < tol, (b, e)
    assert np.array_equal(R, np.conj(np.transpose(R, (0, 2, 1))))   # exactly Hermitian
    d = np.diagonal(R, axis1=1, axis2=2)
    assert np.all(d.imag == 0) and np.all(d.real > 0)


@pytest.mark.parametrize("M", [1, 7, 63, 64, 65, 96, 100, 127, 128, 129, 200, 256])
@pytest.mark.parametrize("T", [1, 31, 33, 100])
def test_covariance_matches_oracle(M, T):
    B = 3
    with plan_line(M) as plan:
        for offset in (0, 1):
            y, Y = snapshots(B, T, M, 1009 * M + T + offset, offset)
            R = torch.full((B, M, M), float("nan"), dtype=torch.complex64, device=DEV)
            bb.ba_covariance(plan, B, T, Y, R)
            torch.cuda.synchronize()
            check(R, y)


def test_covariance_ura256_full_batch_sampled():
    """The 256-element launch at the 2000-trial batch plus one, so the
    XCD-ordered grid is padded, on trials spread over the batch and the last."""
    B, T, M = 2001, 512, 256
    gen = torch.Generator(device=DEV)
    gen.manual_seed(20261203)
    Y = torch.complex(torch.randn((B, T, M), generator=gen, device=DEV),
                      torch.randn((B, T, M), generator=gen, device=DEV))
    with plan_line(M) as plan:
        R = torch.full((B, M, M), float("nan"), dtype=torch.complex64, device=DEV)
        bb.ba_covariance(plan, B, T, Y, R)
        torch.cuda.synchronize()
        pick = [0, 1, 7, 8, 999, 1600, 1999, 2000]
        y = Y[pick].cpu().numpy()
        check(R[pick], y)
        assert not torch.isnan(torch.view_as_real(R)).any()

"""The allocation-free whole path (ba_run_noalloc) against ba_run through the
C-ABI: two calls in a row on the library's fixed scratch array, the second
with a smaller batch, each bit-identical to ba_run on the same inputs (same
kernels, same launch shapes) and within the FP32 gate of the FP64 oracle."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bartlett as ob
from paper_2604_19723_amd import bartlett as bb
from paper_2604_19723_amd import workload as wl

from parity_util import TOL, normwise_err

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _outputs(B, K, plan, with_P):
    P = torch.full((B, plan.G), np.nan, dtype=torch.float32, device=DEV) if with_P else None
    idx = torch.full((B, K), -7, dtype=torch.int32, device=DEV)
    val = torch.full((B, K), np.nan, dtype=torch.float32, device=DEV)
    ref = torch.full((B, K, plan.ndim), np.nan, dtype=torch.float64, device=DEV)
    return P, idx, val, ref


def _compare(ts, plan, Y, B, with_P):
    K = ts.K
    T = ts.n_snap
    P0, i0, v0, r0 = _outputs(B, K, plan, True)
    ws = bb.workspace_for(plan, B, T, True, DEV)
    bb.ba_run(plan, B, T, Y[:B], K, P0, i0, v0, r0, ws)
    P1, i1, v1, r1 = _outputs(B, K, plan, with_P)
    bb.ba_run_noalloc(plan, B, T, Y[:B], K, P1, i1, v1, r1)
    torch.cuda.synchronize()
    assert torch.equal(i0, i1)
    assert torch.equal(v0, v1)
    assert np.array_equal(r0.cpu().numpy(), r1.cpu().numpy(), equal_nan=True)
    if with_P:
        assert torch.equal(P0, P1)
    # and against the FP64 oracle, on the first trials
    A = ob.steering(ts.pos_wl, ob.directions(ts.grid_kind, ts.grid))
    n = min(B, 4)
    Pref = np.stack([ob.spectrum(ob.covariance(ts.Y[b]), A) for b in range(n)])
    assert normwise_err(P0[:n].cpu().numpy(), Pref).max() <= TOL[bb.BA_PREC_F32]


@pytest.mark.parametrize("with_P", [True, False])
def test_noalloc_two_calls_second_smaller(with_P):
    ts = wl.config2(24).rounded()
    print("noalloc: ULA 64, trials 24 then 9, with_P", with_P, flush=True)
    with bb.plan_for(ts) as plan:
        Y = torch.from_numpy(ts.y_c64()).to(DEV)
        _compare(ts, plan, Y, 24, with_P)
        _compare(ts, plan, Y, 9, with_P)


def test_noalloc_streamed_projection_ura():
    # 256 elements: the streamed kernel's Q also lives in the scratch array
    ts = wl.config3(3).rounded()
    print("noalloc: URA 256, trials 3 then 1", flush=True)
    with bb.plan_for(ts) as plan:
        Y = torch.from_numpy(ts.y_c64()).to(DEV)
        _compare(ts, plan, Y, 3, True)
        _compare(ts, plan, Y, 1, True)


def test_noalloc_rejects_batches_beyond_the_array():
    ts = wl.config2(2).rounded()
    with bb.plan_for(ts) as plan:
        limit = 128 << 20
        B = 1
        while bb.ba_workspace_size(plan, B, ts.n_snap, False) <= limit:
            B *= 2
        Y = torch.zeros((1, ts.n_snap, ts.n_elem), dtype=torch.complex64, device=DEV)
        h = C.c_void_p(Y.data_ptr())
        L = bb.lib()
        st = L.ba_run_noalloc(plan.handle, B, ts.n_snap, h, ts.K, None, h, h, None, None)
        assert st == bb.BA_ERR_ARG
        assert b"scratch" in L.ba_last_error()

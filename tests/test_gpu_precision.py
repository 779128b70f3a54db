"""Precision variants of the projection against the FP64 oracle: FP32 on the
matrix cores (register-resident and streaming kernels), the BF16 hi/lo split
(three BF16 MFMA passes, FP32 accumulate), the one-pass BF16 ablation, and the
vector-ALU FP32 reference kernel."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bartlett as ob
from paper_2604_19723_amd import bartlett as bb
from paper_2604_19723_amd import workload as wl

from parity_util import (TOL, check_peaks_same_precision, normwise_err, peak_agreement_fp64)

pytestmark = pytest.mark.gpu
DEV = "cuda"


def oracle_P(ts):
    A = ob.steering(ts.pos_wl, ob.directions(ts.grid_kind, ts.grid))
    return np.stack([ob.spectrum(ob.covariance(ts.Y[b]), A) for b in range(ts.n_trials)])


def gpu_run(ts, prec):
    with bb.plan_for(ts, prec) as plan:
        out = bb.run_grid_search(plan, torch.from_numpy(ts.y_c64()).to(DEV), ts.K)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("prec,tol", [(bb.BA_PREC_F32, 1e-5), (bb.BA_PREC_BF16X3, 1e-3),
                                      (bb.BA_PREC_F32_VALU, 1e-5)])
def test_ura_precisions(prec, tol):
    ts = wl.config3(2).rounded()
    Pref = oracle_P(ts)
    o = gpu_run(ts, prec)
    e = normwise_err(o["P"], Pref)
    print("URA precision", prec, "normwise max", e.max())
    assert e.max() <= tol
    check_peaks_same_precision(o["P"], o["idx"], o["val"], o["refined"], ts.K, ts.grid_shape, ts.wrap0)
    _, _, bad = peak_agreement_fp64(Pref, o["idx"], ts.K, ts.grid_shape, ts.wrap0, tol)
    assert not bad, bad


# an odd trial count leaves the last workgroup of the register-resident
# kernel (two trials per workgroup) with one trial
@pytest.mark.parametrize("M,B", [(8, 12), (40, 12), (64, 12), (100, 12), (128, 12), (64, 7), (40, 1)])
def test_bf16x3_ula(M, B):
    ts = wl.make_ula_trials(B, M, 3, 64, 10.0, 1801, 99).rounded()
    Pref = oracle_P(ts)
    o = gpu_run(ts, bb.BA_PREC_BF16X3)
    e = normwise_err(o["P"], Pref)
    print("BF16x3 M=%d normwise max %.3e" % (M, e.max()))
    assert e.max() <= 1e-3
    check_peaks_same_precision(o["P"], o["idx"], o["val"], o["refined"], ts.K, ts.grid_shape, ts.wrap0)


def test_bf16_single_pass_is_an_ablation():
    """One BF16 pass drops the lo terms: its error is reported, and it must be
    visibly worse than the split (that is what the split buys)."""
    ts = wl.config2(8).rounded()
    Pref = oracle_P(ts)
    e1 = normwise_err(gpu_run(ts, bb.BA_PREC_BF16)["P"], Pref).max()
    e3 = normwise_err(gpu_run(ts, bb.BA_PREC_BF16X3)["P"], Pref).max()
    print("one-pass BF16 %.3e, BF16x3 %.3e" % (e1, e3))
    assert e3 <= 1e-3 and e1 > 4 * e3 and e1 < 0.1


def test_stage_calls_with_spectrum_workspace():
    ts = wl.config3(1).rounded()
    Pref = oracle_P(ts)
    with bb.plan_for(ts, bb.BA_PREC_BF16X3) as plan:
        Y = torch.from_numpy(ts.y_c64()).to(DEV)
        R = torch.empty((1, ts.n_elem, ts.n_elem), dtype=torch.complex64, device=DEV)
        P = torch.empty((1, plan.G), dtype=torch.float32, device=DEV)
        bb.ba_covariance(plan, 1, ts.n_snap, Y, R)
        with pytest.raises(ValueError):
            bb.ba_spectrum(plan, 1, R, P)                 # the streaming kernel needs its workspace
        bb.ba_spectrum(plan, 1, R, P, bb.spectrum_workspace_for(plan, 1))
        torch.cuda.synchronize()
        assert normwise_err(P.cpu().numpy(), Pref).max() <= 1e-3

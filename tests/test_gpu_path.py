"""GPU parity of the whole path (covariance -> spectrum -> peaks) through the
C-ABI, against the FP64 oracle on the same seeded inputs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bartlett as ob
from paper_2604_19723_amd import bartlett as bb
from paper_2604_19723_amd import workload as wl

from parity_util import (TOL, check_peaks_same_precision, normwise_err, peak_agreement_fp64)

pytestmark = pytest.mark.gpu

DEV = "cuda"


def oracle_for(ts):
    A = ob.steering(ts.pos_wl, ob.directions(ts.grid_kind, ts.grid))
    R = np.stack([ob.covariance(ts.Y[b]) for b in range(ts.n_trials)])
    P = np.stack([ob.spectrum(R[b], A) for b in range(ts.n_trials)])
    return A, R, P


def to_dev(ts):
    return torch.from_numpy(ts.y_c64()).to(DEV)


def run_and_check(ts, prec=bb.BA_PREC_F32, check_fp64_peaks=True):
    ts = ts.rounded()
    A, Rref, Pref = oracle_for(ts)
    K = ts.K
    with bb.plan_for(ts, prec) as plan:
        Y = to_dev(ts)
        out = bb.run_grid_search(plan, Y, K)
        torch.cuda.synchronize()
        P = out["P"].cpu().numpy()
        idx = out["idx"].cpu().numpy()
        val = out["val"].cpu().numpy()
        ref = out["refined"].cpu().numpy()
        R = torch.empty((ts.n_trials, ts.n_elem, ts.n_elem), dtype=torch.complex64, device=DEV)
        bb.ba_covariance(plan, ts.n_trials, ts.n_snap, Y, R)
        R = R.cpu().numpy()
    e_R = np.max(np.abs(R - Rref)) / np.max(np.abs(Rref))
    assert e_R < 1e-5, e_R
    assert np.array_equal(R, np.conj(np.transpose(R, (0, 2, 1))))      # exactly Hermitian
    e = normwise_err(P, Pref)
    tol = TOL[prec]
    assert e.max() <= tol, (e.max(), tol)
    check_peaks_same_precision(P, idx, val, ref, K, ts.grid_shape, ts.wrap0)
    if check_fp64_peaks:
        n_cmp, n_tie, bad = peak_agreement_fp64(Pref, idx, K, ts.grid_shape, ts.wrap0, tol)
        assert not bad, bad[:5]
        assert n_cmp >= 0.5 * ts.n_trials
    return dict(e=e, P=P, idx=idx, Pref=Pref)


def test_config1_all_trials():
    r = run_and_check(wl.config1(100))
    print("config1 normwise max", r["e"].max())


def test_config2_subset_ragged_grid_tail():
    # 7201 grid points: not a multiple of any tile size
    run_and_check(wl.config2(21))


def test_config3_ura_2d_wrap():
    run_and_check(wl.config3(2))


def test_snapshot_route_matches_oracle():
    ts = wl.make_ula_trials(6, 32, 3, 12, 5.0, 901, 777).rounded()   # T < M
    A, Rref, Pref = oracle_for(ts)
    with bb.plan_for(ts) as plan:
        P = torch.empty((ts.n_trials, plan.G), dtype=torch.float32, device=DEV)
        bb.ba_spectrum_snapshots(plan, ts.n_trials, ts.n_snap, to_dev(ts), P)
        P = P.cpu().numpy()
    assert normwise_err(P, Pref).max() <= 1e-5


@pytest.mark.parametrize("M,T,G,K", [(1, 1, 5, 1), (2, 1, 3, 2), (5, 3, 64, 3), (7, 33, 1000, 16),
                                     (8, 4, 17, 2), (16, 20, 4099, 3), (32, 9, 515, 3),
                                     (48, 40, 1000, 4), (64, 7, 64, 2), (65, 5, 300, 2),
                                     (128, 17, 257, 6), (256, 2, 131, 2)])
def test_edge_shapes(M, T, G, K):
    ts = wl.make_ula_trials(3, M, 1, T, 10.0, G, 4242, ang_lo=-30, ang_hi=30).rounded()
    ts.K = K
    run_and_check(ts, check_fp64_peaks=False)


def test_zero_trials_is_noop_and_bad_k_raises():
    ts = wl.config1(1)
    with bb.plan_for(ts) as plan:
        Y = to_dev(ts)
        idx = torch.empty((1, 2), dtype=torch.int32, device=DEV)
        val = torch.empty((1, 2), dtype=torch.float32, device=DEV)
        ws = bb.workspace_for(plan, 1, ts.n_snap, with_spectrum_out=False)
        bb.ba_run(plan, 0, ts.n_snap, Y, 2, None, idx, val, None, ws)
        idx17 = torch.empty((1, 17), dtype=torch.int32, device=DEV)
        val17 = torch.empty((1, 17), dtype=torch.float32, device=DEV)
        with pytest.raises(bb.BartlettError) as ei:
            bb.ba_run(plan, 1, ts.n_snap, Y, 17, None, idx17, val17, None, ws)
        assert ei.value.status == bb.BA_ERR_ARG
        with pytest.raises(ValueError):       # the binding refuses a short workspace
            bb.ba_run(plan, 1, ts.n_snap, Y, 2, None, idx, val, None, ws[:16])


def test_nan_input_gives_no_peaks_and_no_fault():
    ts = wl.config1(2)
    Y = ts.y_c64()
    Y[1, 3, 5] = np.nan
    with bb.plan_for(ts) as plan:
        out = bb.run_grid_search(plan, torch.from_numpy(Y).to(DEV), 2)
        idx = out["idx"].cpu().numpy()
        val = out["val"].cpu().numpy()
    assert np.all(idx[1] == -1) and np.all(np.isnan(val[1]))
    assert np.all(idx[0] >= 0)


def test_deterministic_replay():
    ts = wl.config2(8)
    with bb.plan_for(ts) as plan:
        Y = to_dev(ts)
        a = bb.run_grid_search(plan, Y, 4)
        b = bb.run_grid_search(plan, Y, 4)
        torch.cuda.synchronize()
        assert torch.equal(a["P"], b["P"]) and torch.equal(a["idx"], b["idx"])


def test_proposal_moments_match_oracle():
    for ts in (wl.config1(5), wl.config3(1)):
        ts = ts.rounded()
        with bb.plan_for(ts) as plan:
            out = bb.run_grid_search(plan, to_dev(ts), 1)
            d = plan.coord_dim
            mc = torch.empty((ts.n_trials, d + d * d), dtype=torch.float64, device=DEV)
            bb.ba_proposal_moments(plan, ts.n_trials, out["P"], mc)
            mc = mc.cpu().numpy()
            P = out["P"].cpu().numpy()
        for b in range(ts.n_trials):
            mu, C = ob.proposal_moments(P[b].astype(np.float64), ts.grid_kind, ts.grid,
                                        ts.grid_shape, ts.wrap0)
            np.testing.assert_array_equal(mc[b, :d], mu)
            np.testing.assert_allclose(mc[b, d:].reshape(d, d), C, rtol=1e-9, atol=1e-12)

"""Learned-proposal refinement through the C-ABI. A network whose output is a
constant (zero weights, the biases set to the sines of chosen directions)
makes the proposals known, so the window path can be checked against the
full-grid search bit for bit: window points are full-grid points computed by
the same arithmetic."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2604_19723_amd import bartlett as bb
from paper_2604_19723_amd import workload as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"
TRUE_DEG = np.array([-30.1, -10.3, 15.7, 40.2])


def fixed_trials(B, snr_db, seed=11):
    pos = wl.ula_positions(64)
    A = wl.response(pos, wl.ula_dirs(TRUE_DEG))
    Y = np.empty((B, 256, 64), np.complex64)
    for b in range(B):
        rng = wl.trial_rng(seed, b)
        Y[b] = wl._snapshots(rng, A, 256, wl.noise_variance(snr_db, 4, "per_source"))
    return Y


def constant_net(u):
    net = bb.ba_mlp_create(4096, 16, 1, 4, 256, bb.BA_PREC_BF16, 0)
    w = np.zeros(net.n_params, np.float32)
    w[-4:] = u
    bb.ba_mlp_set_weights(net, w)
    return net


def run_both(Y, u, tau, hw=50):
    B = Y.shape[0]
    grid = wl.ula_grid(7201)
    plan = bb.ba_plan_create(64, wl.ula_positions(64), bb.BA_GRID_ULA_DEG, 7201, grid, 7201, 1, 0)
    Yd = torch.from_numpy(Y).to(DEV)
    full = bb.run_grid_search(plan, Yd, 4)
    R = torch.empty((B, 64, 64), dtype=torch.complex64, device=DEV)
    bb.ba_covariance(plan, B, 256, Yd, R)
    net = constant_net(u)
    idx = torch.empty((B, 4), dtype=torch.int32, device=DEV)
    val = torch.empty((B, 4), dtype=torch.float32, device=DEV)
    ref = torch.empty((B, 4), dtype=torch.float64, device=DEV)
    fell = torch.empty(B, dtype=torch.uint8, device=DEV)
    ws = torch.empty(bb.ba_propose_workspace_size(plan, B, 4, 4), dtype=torch.uint8, device=DEV)
    nf = bb.ba_propose_refine(plan, net, B, R, 4, hw, tau, idx, val, ref, fell, ws)
    torch.cuda.synchronize()
    out = dict(idx=idx.cpu().numpy(), val=val.cpu().numpy(), ref=ref.cpu().numpy(),
               fell=fell.cpu().numpy(), nf=nf,
               fidx=full["idx"].cpu().numpy(), fval=full["val"].cpu().numpy(),
               fref=full["refined"].cpu().numpy()[..., 0])
    net.close()
    plan.close()
    return out


def test_windows_reproduce_full_grid_peaks():
    Y = fixed_trials(64, 10.0)
    u = np.sin(np.deg2rad(TRUE_DEG + np.array([0.3, -0.4, 0.2, -0.1])))
    o = run_both(Y, u.astype(np.float32), tau=0.0)
    assert o["nf"] == int(o["fell"].sum()) and o["nf"] < 8
    ok = o["fell"] == 0
    assert np.array_equal(o["idx"][ok], o["fidx"][ok])
    assert np.array_equal(o["val"][ok].view(np.int32), o["fval"][ok].view(np.int32))
    assert np.array_equal(o["ref"][ok].view(np.int64), o["fref"][ok].view(np.int64))


def test_threshold_one_sends_every_trial_to_the_full_grid():
    Y = fixed_trials(32, 0.0, seed=12)
    u = np.sin(np.deg2rad(TRUE_DEG)).astype(np.float32)
    o = run_both(Y, u, tau=1.0)
    assert o["nf"] == 32 and np.all(o["fell"] == 1)
    assert np.array_equal(o["idx"], o["fidx"])
    assert np.array_equal(o["ref"].view(np.int64), o["fref"].view(np.int64))


def test_wrong_proposal_falls_back():
    Y = fixed_trials(16, 10.0, seed=13)
    u = np.sin(np.deg2rad(np.array([-30.1, -10.3, 15.7, 75.0]))).astype(np.float32)   # no source at 75
    o = run_both(Y, u, tau=0.05, hw=20)
    assert np.all(o["fell"] == 1)
    assert np.array_equal(o["idx"], o["fidx"])


# other element counts (the 8-, 16- and 32-element register layouts take
# several 16-column blocks per steering chunk), window half widths from 1 to
# the maximum 100, and windows clipped at either end of the grid
@pytest.mark.parametrize("M,hw,deg", [(8, 50, [-20.0, 35.0]), (16, 1, [-30.1, 15.7]), (16, 100, [-88.0, 87.5]),
                                      (32, 7, [-60.0, 20.0]), (32, 100, [-89.95, 89.95, 0.0])])
def test_windows_other_sizes_and_edges(M, hw, deg):
    B, T, K = 6, 64, len(deg)
    true = np.array(deg)
    pos = wl.ula_positions(M)
    A = wl.response(pos, wl.ula_dirs(true))
    Y = np.empty((B, T, M), np.complex64)
    for b in range(B):
        Y[b] = wl._snapshots(wl.trial_rng(21 + M, b), A, T, wl.noise_variance(20.0, K, "per_source"))
    plan = bb.ba_plan_create(M, pos, bb.BA_GRID_ULA_DEG, 7201, wl.ula_grid(7201), 7201, 1, 0)
    Yd = torch.from_numpy(Y).to(DEV)
    full = bb.run_grid_search(plan, Yd, K)
    R = torch.empty((B, M, M), dtype=torch.complex64, device=DEV)
    bb.ba_covariance(plan, B, T, Yd, R)
    net = bb.ba_mlp_create(M * M, 16, 1, K, 256, bb.BA_PREC_BF16, 0)
    w = np.zeros(net.n_params, np.float32)
    w[-K:] = np.sin(np.deg2rad(true))
    bb.ba_mlp_set_weights(net, w)
    idx = torch.empty((B, K), dtype=torch.int32, device=DEV)
    val = torch.empty((B, K), dtype=torch.float32, device=DEV)
    ref = torch.empty((B, K), dtype=torch.float64, device=DEV)
    fell = torch.empty(B, dtype=torch.uint8, device=DEV)
    ws = torch.empty(bb.ba_propose_workspace_size(plan, B, K, K), dtype=torch.uint8, device=DEV)
    nf = bb.ba_propose_refine(plan, net, B, R, K, hw, 0.0, idx, val, ref, fell, ws)
    torch.cuda.synchronize()
    fell = fell.cpu().numpy()
    assert nf == int(fell.sum())
    if hw >= 50 and np.max(np.abs(true)) < 80:
        assert nf < B  # wide windows around sources away from endfire hold their peaks
    fidx, fval = full["idx"].cpu().numpy(), full["val"].cpu().numpy()
    fref = full["refined"].cpu().numpy()[..., 0]
    P = full["P"].cpu().numpy()
    idx, val, ref = idx.cpu().numpy(), val.cpu().numpy(), ref.cpu().numpy()
    # a trial that fell back carries the full grid's answer
    fb = fell == 1
    assert np.array_equal(idx[fb], fidx[fb]) and np.array_equal(ref[fb].view(np.int64), fref[fb].view(np.int64))
    # a windowed trial reports, per proposal, a point of the full spectrum: its
    # value bit for bit, a local maximum of the full grid (a grid edge counts),
    # within hw of the proposal's grid index, and the full grid's refinement
    G = P.shape[1]
    step = 180.0 / (G - 1)
    centre = np.rint((np.rad2deg(np.arcsin(np.sin(np.deg2rad(true)).astype(np.float32).astype(np.float64)))
                      + 90.0) / step).astype(int)
    for b in np.nonzero(~fb)[0]:
        assert sorted(np.abs(idx[b][:, None] - centre[None, :]).min(axis=1)) <= [hw] * K
        for g, v, r in zip(idx[b], val[b], ref[b]):
            assert v.view(np.int32) == P[b, g].view(np.int32)
            assert (g == 0 or P[b, g] > P[b, g - 1]) and (g == G - 1 or P[b, g] >= P[b, g + 1])
            d = 0.0
            if 0 < g < G - 1:
                pm, p0, pp = float(P[b, g - 1]), float(P[b, g]), float(P[b, g + 1])
                den = pm - 2.0 * p0 + pp
                d = 0.0 if den == 0.0 else min(0.5, max(-0.5, 0.5 * (pm - pp) / den))
            assert abs(r - (g + d)) <= 1e-12
        if np.max(np.abs(true)) < 80:  # away from endfire the windows hold the K largest maxima
            assert np.array_equal(idx[b], fidx[b]) and np.array_equal(val[b].view(np.int32), fval[b].view(np.int32))
    net.close()
    plan.close()

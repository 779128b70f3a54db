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

"""Learned-proposal refinement through the C-ABI.

Every result of ba_propose_refine (index, value, refinement, fallback
verdict) is compared element by element with the FP64 oracle of the window
rule (oracle/propose.py), the decision taken on the device's own FP32
spectrum of the same covariances (window points are full-grid points computed
by the same arithmetic) and the device's own network outputs. Networks: one
trained on the GPU at the learned-proposal shapes, and constant networks
(zero weights, the biases set to the sines of chosen directions) whose
proposals are known, including directions at endfire and NaN."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import propose as op
from paper_2604_19723_amd import bartlett as bb
from paper_2604_19723_amd import learned as lr
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


def device_inputs(plan, net, R, M):
    """The full FP32 spectrum of R, the FP64 sum of its FP32 trace, and the
    network outputs, all from the device path's own kernels."""
    B = R.shape[0]
    G = plan.G
    P = torch.empty((B, G), dtype=torch.float32, device=DEV)
    bb.ba_spectrum(plan, B, R, P)
    X = torch.empty((B, M * M), dtype=torch.float32, device=DEV)
    bb.ba_pack_covariance(M, B, R, X)
    U = torch.empty((B, net.dims[-1]), dtype=torch.float32, device=DEV)
    bb.ba_mlp_forward(net, B, X, U)
    torch.cuda.synchronize()
    tr = R.cpu().numpy().diagonal(axis1=1, axis2=2).real.astype(np.float64).sum(axis=1)
    return P.cpu().numpy(), tr, U.cpu().numpy()


def check_against_oracle(plan, net, R, M, K, hw, tau, grid, out, max_borderline=0.01):
    """Compare one ba_propose_refine result with the oracle's rule. Trials
    whose fallback hinges on the threshold within the FP32 rounding of the
    normalised cost (|P M / tr R - tau| <= 1e-5 tau) are counted and left out."""
    P, tr, U = device_inputs(plan, net, R, M)
    B, G = P.shape
    th0, step = float(grid[0]), float(grid[-1] - grid[0]) / (G - 1)
    n_border = 0
    for b in range(B):
        o = op.refine_trial(P[b], tr[b], M, U[b], th0, step, hw, tau, K)
        if tau > 0 and o["windows"]:
            c = [np.nanmax(P[b][lo:hi + 1]) * M / tr[b] for lo, hi in o["windows"]
                 if not np.all(np.isnan(P[b][lo:hi + 1]))]
            if any(abs(x - tau) <= 1e-5 * tau for x in c):
                n_border += 1
                continue
        assert bool(out["fell"][b]) == o["fell_back"], (b, out["fell"][b], o["fell_back"])
        assert np.array_equal(out["idx"][b], o["idx"]), (b, out["idx"][b], o["idx"])
        np.testing.assert_array_equal(out["val"][b], o["val"].astype(np.float32))
        np.testing.assert_allclose(out["ref"][b], o["refined"], rtol=0, atol=1e-12, equal_nan=True)
    assert n_border <= max_borderline * B, n_border
    assert out["nf"] == int(out["fell"].sum())
    return P


def propose(plan, net, R, K, hw, tau):
    B = R.shape[0]
    idx = torch.empty((B, K), dtype=torch.int32, device=DEV)
    val = torch.empty((B, K), dtype=torch.float32, device=DEV)
    ref = torch.empty((B, K), dtype=torch.float64, device=DEV)
    fell = torch.empty(B, dtype=torch.uint8, device=DEV)
    ws = torch.empty(bb.ba_propose_workspace_size(plan, B, net.dims[-1], K), dtype=torch.uint8, device=DEV)
    nfb = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    bb.ba_propose_refine(plan, net, B, R, K, hw, tau, idx, val, ref, fell, ws, n_fallback=nfb)
    nf = int(nfb.item())
    torch.cuda.synchronize()
    return dict(idx=idx.cpu().numpy(), val=val.cpu().numpy(), ref=ref.cpu().numpy(), fell=fell.cpu().numpy(),
                nf=nf)


def endfire_trials(B, seed, M=64, T=256, K=4):
    """Trials with one or two sources within 5 degrees of endfire."""
    pos = wl.ula_positions(M)
    Y = np.empty((B, T, M), np.complex64)
    for b in range(B):
        rng = wl.trial_rng(seed, b)
        th = np.sort(np.concatenate([rng.uniform(-89.99, -85.0, 1 + b % 2), rng.uniform(85.0, 89.99, 1),
                                     rng.uniform(-50.0, 50.0, K)]))[:K]
        Y[b] = wl._snapshots(rng, wl.response(pos, wl.ula_dirs(th)), T,
                             wl.noise_variance(rng.uniform(0.0, 20.0), K, "per_source"))
    return Y


def covariances(plan, Y):
    B, T, M = Y.shape
    Yd = torch.from_numpy(np.ascontiguousarray(Y)).to(DEV)
    R = torch.empty((B, M, M), dtype=torch.complex64, device=DEV)
    bb.ba_covariance(plan, B, T, Yd, R)
    return R


@pytest.fixture(scope="module")
def trained():
    """A network trained briefly on the GPU by the library's kernels at the
    learned-proposal shapes (64-element ULA, 4 sources, 7201-point grid)."""
    grid = wl.ula_grid(lr.G)
    plan = bb.ba_plan_create(lr.M, wl.ula_positions(lr.M), bb.BA_GRID_ULA_DEG, lr.G, grid, lr.G, 1, 0)
    net = bb.ba_mlp_create(lr.M * lr.M, 512, 3, lr.K, 4096, bb.BA_PREC_BF16, 5)
    X, U, Mk = lr.make_training_set(plan, 32768, 0xBA57_00E1, DEV)
    lr.train(net, X, U, Mk, epochs=3, batch=1024, lr=1e-3, seed=1)
    del X, U, Mk
    yield plan, net, grid
    net.close()
    plan.close()


@pytest.mark.parametrize("tau", [0.0, 0.05, 0.15, 0.3])
def test_trained_network_windows_match_the_oracle(trained, tau):
    plan, net, grid = trained
    ts = wl.config5(384, seed_offset=9)
    Y = np.concatenate([ts.y_c64(), endfire_trials(64, 0xBA57_00E2)])
    R = covariances(plan, Y)
    out = propose(plan, net, R, lr.K, 50, tau)
    check_against_oracle(plan, net, R, lr.M, lr.K, 50, tau, grid, out)
    if tau == 0.05:
        assert 0 < out["nf"] < Y.shape[0]   # both verdicts occur


@pytest.mark.parametrize("deg", [[-89.9, -88.0, 87.5, 89.95], [-90.0, -30.1, 15.7, 90.0], [-86.0, -20.0, 10.0, 86.0]])
def test_endfire_windows_match_the_oracle(trained, deg):
    plan, _, grid = trained
    net = constant_net(np.sin(np.deg2rad(deg)).astype(np.float32))
    try:
        R = covariances(plan, endfire_trials(48, 0xBA57_00E3))
        for tau in (0.0, 0.1):
            out = propose(plan, net, R, 4, 50, tau)
            check_against_oracle(plan, net, R, 64, 4, 50, tau, grid, out)
    finally:
        net.close()


def test_nan_proposal_and_nan_spectrum_fall_back_as_the_oracle_says(trained):
    plan, _, grid = trained
    Y = fixed_trials(16, 10.0, seed=14)
    R = covariances(plan, Y)
    R[5, 7, 7] = float("nan")          # trial 5: every spectrum value is NaN
    u = np.sin(np.deg2rad(TRUE_DEG)).astype(np.float32)
    net = constant_net(u)
    try:
        out = propose(plan, net, R, 4, 50, 0.0)
        check_against_oracle(plan, net, R, 64, 4, 50, 0.0, grid, out)
        assert out["fell"][5] == 1 and np.all(out["idx"][5] == -1)
    finally:
        net.close()
    u[2] = np.nan                      # a NaN network output sends every trial back
    net = constant_net(u)
    try:
        R = covariances(plan, Y)
        out = propose(plan, net, R, 4, 50, 0.0)
        assert np.all(out["fell"] == 1)
        check_against_oracle(plan, net, R, 64, 4, 50, 0.0, grid, out)
    finally:
        net.close()


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
    nfb = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    bb.ba_propose_refine(plan, net, B, R, 4, hw, tau, idx, val, ref, fell, ws, n_fallback=nfb)
    nf = int(nfb.item())
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
    nfb = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    bb.ba_propose_refine(plan, net, B, R, K, hw, 0.0, idx, val, ref, fell, ws, n_fallback=nfb)
    nf = int(nfb.item())
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
    # every result against the oracle's rule on the device's own spectrum
    _, tr, Ud = device_inputs(plan, net, R, M)
    ocl = op.refine_batch(P, tr, M, Ud, -90.0, step, hw, 0.0, K)
    assert np.array_equal(fell.astype(bool), ocl["fell_back"])
    assert np.array_equal(idx, ocl["idx"])
    np.testing.assert_array_equal(val, ocl["val"].astype(np.float32))
    np.testing.assert_allclose(ref, ocl["refined"], rtol=0, atol=1e-12)
    for b in np.nonzero(~fb)[0]:
        # each peak lies in the clipped window of one proposal of its own
        for g in idx[b]:
            assert np.any(np.abs(g - centre) <= hw)
        assert len(set(idx[b].tolist())) == K
        for g, v, r in zip(idx[b], val[b], ref[b]):
            assert v.view(np.int32) == P[b, g].view(np.int32)
            assert (g == 0 or P[b, g] > P[b, g - 1]) and (g == G - 1 or P[b, g] >= P[b, g + 1])
            d = 0.0
            if 0 < g < G - 1:
                pm, p0, pp = float(P[b, g - 1]), float(P[b, g]), float(P[b, g + 1])
                den = pm - 2.0 * p0 + pp
                d = 0.0 if den == 0.0 else min(0.5, max(-0.5, 0.5 * (pm - pp) / den))
            assert abs(r - (g + d)) <= 1e-12
        # Away from endfire the windows hold the K largest maxima. A windowed
        # trial returns local maxima of the full spectrum; they are its top K
        # only when no maximum outside the windows beats one of them, which
        # the rule does not check (the threshold guards against it).
        if np.max(np.abs(true)) < 80:
            assert np.array_equal(idx[b], fidx[b]) and np.array_equal(val[b].view(np.int32), fval[b].view(np.int32))
    net.close()
    plan.close()

"""Gaussian birth proposal through the C-ABI against the FP64 oracle: the
device's own moments and the same standard normal draws on both sides."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bartlett as ob
from oracle import proposal as op
from paper_2604_19723_amd import bartlett as bb
from paper_2604_19723_amd import workload as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"


def region_of(ts):
    """The grid's extent per coordinate; a wrapping azimuth axis is periodic."""
    if ts.grid_kind == bb.BA_GRID_ULA_DEG:
        g = np.asarray(ts.grid, float)
        return np.array([g.min()]), np.array([g.max()]), np.array([False])
    g = np.asarray(ts.grid, float).reshape(-1, 2)
    az0 = g[0, 0]
    return (np.array([az0, g[:, 1].min()]), np.array([az0 + 360.0, g[:, 1].max()]), np.array([True, False]))


def run(ts, N, seed, mu_cov_override=None):
    ts = ts.rounded()
    B = ts.n_trials
    with bb.plan_for(ts) as plan:
        d = plan.coord_dim
        out = bb.run_grid_search(plan, torch.from_numpy(ts.y_c64()).to(DEV), 1)
        mc = torch.empty((B, d + d * d), dtype=torch.float64, device=DEV)
        bb.ba_proposal_moments(plan, B, out["P"], mc)
        if mu_cov_override is not None:
            mc = torch.from_numpy(mu_cov_override).to(DEV)
        z = np.random.default_rng(seed).standard_normal((B, N, d))
        part = torch.empty((B, N, d), dtype=torch.float64, device=DEV)
        w = torch.empty((B, N), dtype=torch.float64, device=DEV)
        bb.ba_proposal_sample(plan, B, mc, N, torch.from_numpy(z).to(DEV), part, w)
        torch.cuda.synchronize()
        return mc.cpu().numpy(), z, part.cpu().numpy(), w.cpu().numpy()


def check(ts, mc, z, part, w):
    d = z.shape[2]
    lo, hi, per = region_of(ts)
    for b in range(z.shape[0]):
        mu, C = mc[b, :d], mc[b, d:].reshape(d, d)
        p_ref, w_ref = op.sample_and_weight(mu, C, z[b], lo, hi, per)
        np.testing.assert_allclose(part[b], p_ref, rtol=1e-13, atol=1e-11)
        np.testing.assert_allclose(w[b], w_ref, rtol=1e-10, atol=1e-300, equal_nan=True)


def test_ula_proposal_matches_oracle():
    ts = wl.config2(12)
    mc, z, part, w = run(ts, 3000, 1)
    check(ts.rounded(), mc, z, part, w)
    assert np.allclose(w.sum(axis=1), 1.0)


def test_ura_azimuth_wrap_matches_oracle():
    ts = wl.make_ura_trials(6, 4, 4, 1, 64, 5.0, 73, 19, wl.SEED_BASE + 70, name="ura4")
    mc, z, part, w = run(ts, 1000, 2)
    check(ts.rounded(), mc, z, part, w)
    assert np.all((part[..., 0] >= 0.0) & (part[..., 0] < 360.0))


def test_degenerate_and_empty_region():
    ts = wl.config1(3)
    # trial 0: zero covariance; trial 1: far outside the [-90, 90] region with a tiny spread;
    # trial 2: NaN moments
    mc = np.array([[10.0, 0.0], [500.0, 1e-4], [np.nan, np.nan]])
    mc_o, z, part, w = run(ts, 300, 3, mu_cov_override=mc)
    assert np.all(part[0] == 10.0) and np.allclose(w[0], 1.0 / 300)
    assert np.all(np.isnan(w[1]))
    assert np.all(np.isnan(part[2])) and np.allclose(w[2], 1.0 / 300)
    check(ts, mc, z, part, w)


def test_direction_grids_are_unsupported():
    G = 5
    dirs = ob.directions(ob.GRID_ULA_DEG, np.linspace(-30, 30, G))
    plan = bb.ba_plan_create(4, wl.ula_positions(4), bb.BA_GRID_DIRS, G, dirs, G, 1, 0)
    try:
        mc = torch.zeros((1, 12), dtype=torch.float64, device=DEV)
        z = torch.zeros((1, 2, 3), dtype=torch.float64, device=DEV)
        part = torch.empty((1, 2, 3), dtype=torch.float64, device=DEV)
        w = torch.empty((1, 2), dtype=torch.float64, device=DEV)
        with pytest.raises(bb.BartlettError):
            bb.ba_proposal_sample(plan, 1, mc, 2, z, part, w)
    finally:
        plan.close()

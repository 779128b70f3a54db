"""Coherent multi-array cost over SFV candidates through the C-ABI against the
FP64 oracle on the same seeded inputs (the oracle rebuilds every steering
vector from the geometry)."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bartlett as ob
from oracle import coherent as oc
from paper_2604_19723_amd import bartlett as bb
from paper_2604_19723_amd import workload as wl

from parity_util import normwise_err

pytestmark = pytest.mark.gpu
DEV = "cuda"


def oracle_spectra(cs, Z, cand):
    lam = oc.C_LIGHT / cs.fc
    f = oc.frequencies(cs.n_f, cs.bandwidth)
    py, pz = oc.ura_support(cs.n_y, lam), oc.ura_support(cs.n_z, lam)
    return np.stack([oc.coherent_spectrum(Z[b].astype(np.complex128), cand, cs.p_mt, cs.pa_pos, cs.pa_rot, f,
                                          py, pz, cs.fc) for b in range(Z.shape[0])])


def run(cs, Z, cand):
    B = Z.shape[0]
    with bb.ba_coherent_create(cs.pa_pos, cs.pa_rot, cs.n_y, cs.n_z, cs.n_f, cs.fc, cs.bandwidth, cs.p_mt,
                               cand) as h:
        P = torch.empty((B, len(cand)), dtype=torch.float32, device=DEV)
        ws = bb.coherent_workspace_for(h, B, DEV)
        bb.ba_coherent_spectrum(h, B, torch.from_numpy(np.ascontiguousarray(Z)).to(DEV), P, ws)
        mc = torch.empty((B, 12), dtype=torch.float64, device=DEV)
        bb.ba_coherent_moments(h, B, P, mc, ws)
        torch.cuda.synchronize()
        return P.cpu().numpy(), mc.cpu().numpy()


@pytest.mark.parametrize("B,G", [(5, 300), (1, 1), (70, 129)])
def test_coherent_spectrum_matches_oracle(B, G):
    cs = wl.coherent_config(B, G)
    P, mc = run(cs, cs.Z, cs.candidates)
    Pref = oracle_spectra(cs, cs.Z[:min(B, 6)], cs.candidates)
    e = normwise_err(P[:len(Pref)], Pref)
    assert e.max() <= 1e-5, e.max()
    # moments over the candidates from the device's own spectrum
    for b in range(min(B, 6)):
        mu, C = ob.proposal_moments(P[b].astype(np.float64), ob.GRID_DIRS, cs.candidates, (G, 1), 0)
        np.testing.assert_array_equal(mc[b, :3], mu)
        # accumulated about the maximum, as defined: FP64 rounding on the scale of C itself
        np.testing.assert_allclose(mc[b, 3:].reshape(3, 3), C, rtol=1e-9, atol=1e-13 * np.max(np.abs(C)))


def test_small_geometry_and_padding():
    # one array, one frequency, 1 x 2 elements: K = 4 real rows padded to 32
    cs = wl.coherent_config(3, 50, n_f=1)
    cs.pa_pos, cs.pa_rot = cs.pa_pos[:1], cs.pa_rot[:1]
    cs.n_y, cs.n_z = 1, 2
    rng = np.random.default_rng(5)
    Z = (rng.standard_normal((3, 1, 2)) + 1j * rng.standard_normal((3, 1, 2))).astype(np.complex64)
    P, _ = run(cs, Z, cs.candidates)
    Pref = oracle_spectra(cs, Z, cs.candidates)
    assert normwise_err(P, Pref).max() <= 1e-5


def test_noise_free_peak_at_the_true_feature():
    cs = wl.coherent_config(2, 400, snr_db=200.0)
    cand = np.concatenate([cs.candidates, cs.sfv_true[None, :]])
    P, mc = run(cs, cs.Z, cand)
    # the true SFV scores its closed-form value |rho|^2 (sum_j |psi_j|^2 / N_z)^2
    lam = oc.C_LIGHT / cs.fc
    Psi = oc.steering(cs.p_mt, cs.sfv_true, cs.pa_pos, cs.pa_rot, oc.frequencies(cs.n_f, cs.bandwidth),
                      oc.ura_support(4, lam), oc.ura_support(4, lam), cs.fc)
    want = (np.sum(np.abs(Psi) ** 2) / 160) ** 2
    assert abs(P[0, -1] - want) <= 1e-5 * want


def test_coherent_argument_errors():
    cs = wl.coherent_config(1, 4)
    bad = cs.candidates.copy()
    bad[2] = 0.0
    with pytest.raises(bb.BartlettError):
        bb.ba_coherent_create(cs.pa_pos, cs.pa_rot, 4, 4, 10, cs.fc, cs.bandwidth, cs.p_mt, bad)
    with pytest.raises(bb.BartlettError):
        bb.ba_coherent_create(cs.pa_pos, cs.pa_rot, 16, 16, 10, cs.fc, cs.bandwidth, cs.p_mt, cs.candidates)
    with pytest.raises(bb.BartlettError):
        bb.ba_coherent_create(cs.pa_pos, cs.pa_rot, 4, 4, 10, -1.0, cs.bandwidth, cs.p_mt, cs.candidates)

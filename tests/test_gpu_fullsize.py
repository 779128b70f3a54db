"""Parity at the full sizes and launch shapes the benchmark times: the
64-element ULA batch of 10 000 trials (the projection splits the grid columns
over two workgroups per trial at that batch size), the 50 000-trial uneven
batch in its persistent graph launch (autotuned as the benchmark does), and
the coherent cost over 131 072 SFV candidates for 1024 trials. The oracle
checks sampled outputs one by one: trials spread over the batch (the last
included), every size class and route, and the last tickets of the
persistent launch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bartlett as ob
from oracle import coherent as oc
from paper_2604_19723_amd import bartlett as bb
from paper_2604_19723_amd import workload as wl

from parity_util import check_peaks_same_precision, normwise_err, peak_agreement_fp64

pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_ula64_full_batch_sampled():
    B = 10000
    print("full size: ULA 64, 10 000 trials", flush=True)
    ts = wl.config2(B, dtype=np.complex64, workers=16)
    K, G = ts.K, ts.n_grid
    with bb.plan_for(ts) as plan:
        out = bb.run_grid_search(plan, torch.from_numpy(ts.Y).to(DEV), K)
        torch.cuda.synchronize()
        sel = np.unique(np.r_[np.linspace(0, B - 1, 60).astype(int), 1, 4999, 5000, B - 2, B - 1])
        st = torch.from_numpy(sel).to(DEV)
        P = out["P"][st].cpu().numpy()
        idx, val, ref = (out[k][st].cpu().numpy() for k in ("idx", "val", "refined"))
    A = ob.steering(ts.pos_wl, ob.directions(ts.grid_kind, ts.grid))
    Pref = np.stack([ob.spectrum(ob.covariance(ts.Y[b].astype(np.complex128)), A) for b in sel])
    e = normwise_err(P, Pref)
    assert e.max() <= 1e-5, (sel[np.argmax(e)], e.max())
    check_peaks_same_precision(P, idx, val, ref, K, (G, 1), 0)
    n_cmp, n_tie, bad = peak_agreement_fp64(Pref, idx, K, (G, 1), 0, 1e-5)
    assert not bad, bad[:5]
    assert n_cmp >= 0.5 * len(sel)      # low-SNR trials often tie at the K-th peak
    print("sampled %d trials: normwise max %.2e, %d ties" % (len(sel), e.max(), n_tie))


def test_ragged_full_batch_sampled(tmp_path):
    n, G, KMAX = 50000, 3601, 8
    print("full size: uneven batch, 50 000 trials", flush=True)
    Ks, Ms, Ts, off, total = wl.config4_layout(n)
    rng = np.random.default_rng(41)
    # the oracle's sample: 30 trials per size class, the 20 cheapest trials
    # (the last tickets of the longest-first order) and the 10 costliest
    cost = Ms.astype(np.float64) ** 2 * (Ts + G)
    pick = [rng.choice(np.nonzero(Ms == m)[0], 30, replace=False) for m in wl.C4_SIZES]
    order = np.argsort(cost, kind="stable")
    sel = np.unique(np.concatenate(pick + [order[:20], order[-10:], [0, n - 1]]))
    # every trial gets data of its own size; the sampled ones their true draws
    gen = torch.Generator(device=DEV)
    gen.manual_seed(7)
    pool = torch.randn(total, dtype=torch.complex64, device=DEV, generator=gen)
    ys = {}
    for i in sel:
        y = wl.config4_trial(int(i))[0].astype(np.complex64)
        ys[int(i)] = y.astype(np.complex128)          # the oracle sees the values the device holds
        pool[int(off[i]):int(off[i]) + y.size] = torch.from_numpy(y.reshape(-1)).to(DEV)
    rs = wl.RaggedSet(pool=None, y_offset=off, n_elem=Ms, n_snap=Ts, k=Ks, truth=[None] * n,
                      snr_db=np.zeros(n), grid=wl.ula_grid(G))
    plan = bb.ba_plan_create(128, wl.ula_positions(128), bb.BA_GRID_ULA_DEG, G, rs.grid, G, 1, 0)
    P = torch.empty((n, G), dtype=torch.float32, device=DEV)
    idx = torch.empty((n, KMAX), dtype=torch.int32, device=DEV)
    val = torch.empty((n, KMAX), dtype=torch.float32, device=DEV)
    ref = torch.empty((n, KMAX, 1), dtype=torch.float64, device=DEV)
    with bb.ba_ragged_create(plan, bb.ragged_descriptors(rs), KMAX, pool, P, idx, val, ref) as r:
        bb.ba_ragged_autotune(r, str(tmp_path / "tune.txt"), repeats=2, max_probe=256)
        bb.ba_ragged_launch(r)
        torch.cuda.synchronize()
        routes = bb.ba_ragged_routes(r)
    plan.close()
    st = torch.from_numpy(sel).to(DEV)
    Ph, ih, vh, rh = (t[st].cpu().numpy() for t in (P, idx, val, ref))
    assert len(set(routes[sel])) == 2, "the sample covers both routes"
    emax, bad = 0.0, []
    for j, i in enumerate(sel):
        M, K = int(Ms[i]), int(Ks[i])
        A = ob.steering(wl.ula_positions(M), ob.directions(ob.GRID_ULA_DEG, rs.grid))
        Pref = ob.spectrum(ob.covariance(ys[int(i)]), A)
        e = normwise_err(Ph[j][None], Pref[None])[0]
        emax = max(emax, e)
        assert e <= 1e-5, (i, M, int(Ts[i]), K, int(routes[i]), e)
        check_peaks_same_precision(Ph[j][None], ih[j][None, :K], vh[j][None, :K], rh[j][None, :K], K, (G, 1), 0)
        assert np.all(ih[j, K:] == -1) and np.all(np.isnan(vh[j, K:]))
        _, _, b = peak_agreement_fp64(Pref[None], ih[j][None, :K], K, (G, 1), 0, 1e-5)
        bad += [(int(i),) + tuple(x) for x in b]
    assert not bad, bad[:3]
    print("sampled %d of %d trials (routes %s): normwise max %.2e" % (
        len(sel), n, np.bincount(routes[sel]), emax))


def test_coherent_full_launch_sampled():
    B, G = 1024, 131072
    print("full size: coherent cost, 1024 trials x 131 072 candidates", flush=True)
    cs = wl.coherent_config(B, G)
    with bb.ba_coherent_create(cs.pa_pos, cs.pa_rot, cs.n_y, cs.n_z, cs.n_f, cs.fc, cs.bandwidth, cs.p_mt,
                               cs.candidates) as h:
        P = torch.empty((B, G), dtype=torch.float32, device=DEV)
        ws = bb.coherent_workspace_for(h, B, DEV)
        bb.ba_coherent_spectrum(h, B, torch.from_numpy(np.ascontiguousarray(cs.Z)).to(DEV), P, ws)
        torch.cuda.synchronize()
        trials = np.array([0, 337, 778, B - 1])
        Ph = P[torch.from_numpy(trials).to(DEV)].cpu().numpy()
    lam = oc.C_LIGHT / cs.fc
    f = oc.frequencies(cs.n_f, cs.bandwidth)
    py, pz = oc.ura_support(cs.n_y, lam), oc.ura_support(cs.n_z, lam)
    # candidates checked: 2048 spread over the set (the last included), plus
    # each sampled trial's device maximum and its index neighbours
    cand = set(np.linspace(0, G - 1, 2048).astype(int).tolist())
    for row in Ph:
        g = int(np.argmax(row))
        cand.update(range(max(0, g - 2), min(G, g + 3)))
    cand = np.array(sorted(cand))
    psi = [oc.steering(cs.p_mt, cs.candidates[g], cs.pa_pos, cs.pa_rot, f, py, pz, cs.fc) for g in cand]
    emax = 0.0
    for j, b in enumerate(trials):
        Pref = np.array([oc.coherent_cost(cs.Z[b].astype(np.complex128), s) for s in psi])
        e = np.max(np.abs(Ph[j][cand] - Pref)) / np.max(Pref)
        emax = max(emax, e)
        assert e <= 1e-5, (b, e)
        # the device maximum is the oracle's maximum over the sample (which
        # holds it), up to values tied within 4 tol of the peak
        g_dev = int(np.argmax(Ph[j]))
        assert Pref[np.searchsorted(cand, g_dev)] >= Pref.max() * (1 - 4e-5), (b, g_dev, cand[np.argmax(Pref)])
    print("sampled %d candidates x %d trials: normwise max %.2e" % (len(cand), len(trials), emax))

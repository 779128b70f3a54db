"""Learned-proposal pipeline: training data labelled by the plain grid search,
network training with the library's own kernels, threshold selection, and
the comparison against the plain FP32 full-grid search at equal RMSE.

Everything that computes runs in libbartlett's kernels (covariance, full-grid
search, packing, network forward/backward/Adam, window refinement); torch
supplies device memory, streams and, for the bulk training stream only, a
seeded on-device random generator that draws the same signal model as the
numpy workload generator (the evaluation sets come from the numpy generator).
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import bartlett as bb
from . import metrics
from . import workload as wl

M, T, K, G = 64, 256, 4, 7201


def _device_trials(n, gen, device):
    """n trials of the learned-proposal workload on the device: SNR ~ U[-10, 20]
    dB, 4 sources in [-60, 60] deg with 5 deg separation, CN(0,1) amplitudes,
    CN(0, sigma^2) noise; complex64 [n][T][M]."""
    import torch
    f32 = torch.float32
    snr = torch.rand(n, generator=gen, device=device, dtype=torch.float64) * 30.0 - 10.0
    th = torch.empty((n, K), dtype=torch.float64, device=device)
    todo = torch.arange(n, device=device)
    while todo.numel():
        cand = torch.rand((todo.numel(), K), generator=gen, device=device, dtype=torch.float64) * 120.0 - 60.0
        cand, _ = torch.sort(cand, dim=1)
        ok = (cand[:, 1:] - cand[:, :-1]).min(dim=1).values >= 5.0
        th[todo[ok]] = cand[ok]
        todo = todo[~ok]
    pos = torch.from_numpy(wl.ula_positions(M)[:, 1]).to(device)              # [M] wavelengths
    ph = pos[None, :, None] * torch.sin(torch.deg2rad(th))[:, None, :]         # [n][M][K] cycles
    ph = ph - torch.round(ph)
    Ar = torch.cos(2 * math.pi * ph).to(f32)
    Ai = torch.sin(2 * math.pi * ph).to(f32)
    Sr = torch.randn((n, T, K), generator=gen, device=device, dtype=f32) * math.sqrt(0.5)
    Si = torch.randn((n, T, K), generator=gen, device=device, dtype=f32) * math.sqrt(0.5)
    sig = torch.sqrt(0.5 * torch.pow(10.0, -snr / 10.0)).to(f32)[:, None, None]
    Nr = torch.randn((n, T, M), generator=gen, device=device, dtype=f32) * sig
    Ni = torch.randn((n, T, M), generator=gen, device=device, dtype=f32) * sig
    ArT = Ar.transpose(1, 2).contiguous()
    AiT = Ai.transpose(1, 2).contiguous()
    Yr = torch.matmul(Sr, ArT) - torch.matmul(Si, AiT) + Nr
    Yi = torch.matmul(Sr, AiT) + torch.matmul(Si, ArT) + Ni
    return torch.complex(Yr, Yi).contiguous(), snr, th


def labels_from_plain(plan, Y, device):
    """Covariance, packed network input and the plain method's own estimates
    (sines of the refined full-grid peaks, sorted; missing peaks masked)."""
    import torch
    n = Y.shape[0]
    R = torch.empty((n, M, M), dtype=torch.complex64, device=device)
    bb.ba_covariance(plan, n, T, Y, R)
    P = torch.empty((n, G), dtype=torch.float32, device=device)
    bb.ba_spectrum(plan, n, R, P)
    idx = torch.empty((n, K), dtype=torch.int32, device=device)
    val = torch.empty((n, K), dtype=torch.float32, device=device)
    ref = torch.empty((n, K, 1), dtype=torch.float64, device=device)
    bb.ba_peaks(plan, n, P, K, idx, val, ref)
    X = torch.empty((n, M * M), dtype=torch.float32, device=device)
    bb.ba_pack_covariance(M, n, R, X)
    step = 180.0 / (G - 1)
    deg = -90.0 + ref[..., 0] * step
    u = torch.sin(torch.deg2rad(deg))
    ok = idx >= 0
    u = torch.where(ok, u, torch.full_like(u, 2.0))
    u, order = torch.sort(u, dim=1)
    mask = torch.gather(ok, 1, order).to(torch.float32)
    u = torch.where(mask > 0, u, torch.zeros_like(u)).to(torch.float32)
    return X, u.contiguous(), mask.contiguous()


def make_training_set(plan, n, seed, device, chunk=8192, log=None):
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    Xs, Us, Ms = [], [], []
    for i0 in range(0, n, chunk):
        m = min(chunk, n - i0)
        Y, _, _ = _device_trials(m, gen, device)
        X, u, mk = labels_from_plain(plan, Y, device)
        Xs.append(X)
        Us.append(u)
        Ms.append(mk)
        del Y
        if log and (i0 // chunk) % 16 == 0:
            log("training set: %d / %d trials" % (i0 + m, n))
    return torch.cat(Xs), torch.cat(Us), torch.cat(Ms)


def train(net, X, U, Mk, epochs, batch, lr, seed, log=None):
    import torch
    n = X.shape[0]
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    hist = []
    steps = 0
    total = epochs * (n // batch)
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        for s in range(n // batch):
            sel = perm[s * batch:(s + 1) * batch]
            xb, ub, mb = X[sel].contiguous(), U[sel].contiguous(), Mk[sel].contiguous()
            # cosine decay
            cur = lr * 0.5 * (1.0 + math.cos(math.pi * steps / max(1, total)))
            bb.ba_mlp_train_step(net, batch, xb, ub, mb, max(cur, lr * 1e-3), loss)
            steps += 1
        hist.append(float(loss.item()))
        if log:
            log("epoch %d: last batch loss %.3e" % (ep, hist[-1]))
    return hist


def evaluate(plan, net, ts, taus, device, hw=50, steps=1, warmup=1):
    """Plain full grid vs learned proposal on a numpy-generated trial set:
    RMSE (deg) per threshold, fallback rate and timings (mean over `steps`
    timed passes after `warmup` untimed ones)."""
    import torch
    if steps < 1:
        raise ValueError("evaluate needs steps >= 1 timed passes")
    n = ts.n_trials
    Y = torch.from_numpy(ts.y_c64()).to(device)
    R = torch.empty((n, M, M), dtype=torch.complex64, device=device)
    P = torch.empty((n, G), dtype=torch.float32, device=device)
    idx = torch.empty((n, K), dtype=torch.int32, device=device)
    val = torch.empty((n, K), dtype=torch.float32, device=device)
    ref = torch.empty((n, K, 1), dtype=torch.float64, device=device)

    # the fastest plain search the plan serves: peak candidates from the
    # projection and a merge (same peaks as ba_peaks, spectrum never written)
    try:
        cand = bb.candidates_for(plan, n, K, device)
    except bb.BartlettError:
        cand = None

    def plain():
        bb.ba_covariance(plan, n, T, Y, R)
        if cand is not None:
            bb.ba_spectrum_candidates(plan, n, R, K, None, cand)
            bb.ba_peaks_merge(plan, n, K, cand, idx, val, ref)
        else:
            bb.ba_spectrum(plan, n, R, P)
            bb.ba_peaks(plan, n, P, K, idx, val, ref)

    for _ in range(max(warmup, 1)):
        plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plain()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / steps
    idx_plain = idx.cpu().numpy()
    base = _rmse(ts, idx_plain, ref.cpu().numpy()[..., 0])
    err_plain = _trial_errors(ts, idx_plain, ref.cpu().numpy()[..., 0])

    li = torch.empty((n, K), dtype=torch.int32, device=device)
    lv = torch.empty((n, K), dtype=torch.float32, device=device)
    lr_ = torch.empty((n, K), dtype=torch.float64, device=device)
    fell = torch.empty(n, dtype=torch.uint8, device=device)
    ws = torch.empty(bb.ba_propose_workspace_size(plan, n, net.dims[-1], K), dtype=torch.uint8, device=device)
    res = []
    nfb = torch.zeros(1, dtype=torch.int32, device=device)
    for tau in taus:
        def learned():
            bb.ba_covariance(plan, n, T, Y, R)
            bb.ba_propose_refine(plan, net, n, R, K, hw, tau, li, lv, lr_, fell, ws, n_fallback=nfb)
        for _ in range(max(warmup, 1)):
            learned()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            learned()
        torch.cuda.synchronize()
        t_l = (time.perf_counter() - t0) / steps
        nf = int(nfb.item())
        idx_l, ref_l = li.cpu().numpy(), lr_.cpu().numpy()
        r = _rmse(ts, idx_l, ref_l)
        cmp = metrics.compare_accuracy(_trial_errors(ts, idx_l, ref_l), err_plain)
        res.append(dict(tau=float(tau), fallback=nf / n, rmse=r, seconds=t_l, trials_per_s=n / t_l,
                        accuracy_vs_plain=cmp, index_identity_vs_plain=metrics.index_identity(idx_l, idx_plain)))
    return dict(plain=dict(rmse=base, seconds=t_plain, trials_per_s=n / t_plain), learned=res)


def _trial_errors(ts, idx, ref_grid):
    """Per trial the associated errors in degrees (sorted pairing), None
    where a peak is missing."""
    deg = -90.0 + ref_grid * (180.0 / (G - 1))
    return [None if np.any(idx[b] < 0) else metrics.associated_errors(deg[b], ts.truth[b])
            for b in range(ts.n_trials)]


def _rmse(ts, idx, ref_grid):
    """RMSE in degrees over (trial, source) pairs, sorted pairing; bootstrap SE."""
    deg = -90.0 + ref_grid * (180.0 / (G - 1))
    per = []
    fails = 0
    for b in range(ts.n_trials):
        if np.any(idx[b] < 0):
            fails += 1
            continue
        e = metrics.associated_errors(deg[b], ts.truth[b])
        per.append(np.mean(e * e))
    per = np.asarray(per)
    rng = np.random.default_rng(0)
    boots = [math.sqrt(np.mean(per[rng.integers(0, len(per), len(per))])) for _ in range(200)]
    return dict(rmse=float(math.sqrt(np.mean(per))), se=float(np.std(boots)), failed=fails)


def equal_rmse(r_l, r_p):
    """|RMSE_l - RMSE_p| <= max(1 % RMSE_p, 2 SE)."""
    return abs(r_l["rmse"] - r_p["rmse"]) <= max(0.01 * r_p["rmse"], 2.0 * max(r_l["se"], r_p["se"]))


def equal_accuracy(r, plain):
    """A learned result (one entry of evaluate()["learned"]) matches the plain
    search: equal RMSE, and equal median error, resolved fraction and RMSE over
    resolved sources in the paired comparison on the same trials."""
    return bool(equal_rmse(r["rmse"], plain["rmse"]) and r["accuracy_vs_plain"]["equal_accuracy"])


def choose_tau(ev):
    """The smallest threshold whose result matches the plain search
    (equal_accuracy), or None."""
    ok = [r for r in ev["learned"] if equal_accuracy(r, ev["plain"])]
    return min(ok, key=lambda r: r["tau"]) if ok else None

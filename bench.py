#!/usr/bin/env python3
"""Benchmark of the batched Bartlett grid search on one MI355X.

One step = the whole hot path over one batch held in HBM: sample covariance ->
Bartlett spectrum on every grid point -> top-K peaks with refinement, for the
64-element ULA workload (4 sources, 256 snapshots, 7201-point grid over
[-90, 90] deg, 10 000 trials with the SNR sweep -10..20 dB cycled over them).

Prints one JSON line on stdout (everything else goes to stderr):
  value       trials per second over the timed steps (inputs already resident)
  roofline    the projection kernel's algorithmic FLOP rate against its peak,
              timed with HIP events on the stream it is launched on
  cpu_baseline the FP64 oracle timed on a bounded sample of the same workload
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# dense peaks of the arithmetic each projection kernel runs on
SEED_PROPOSAL = 0xBA570007
PEAK = {"f32": ("mfma", 157.3), "bf16x3": ("mfma", 2500.0), "bf16": ("mfma", 2500.0),
        "f32_valu": ("alu", 157.3)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(key):
    """HBM bytes per launch of a kernel from the committed counter record
    (profiles/traffic.json: FETCH_SIZE + WRITE_SIZE, each scaled by what the
    counter reads for a copy of known size), or None when the record is
    missing or the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))[key]
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != rec["source_sha256"]:
            return None
        return rec["fetch_bytes"] + rec["write_bytes"]
    except (OSError, KeyError, ValueError):
        return None


# projection kernels that evaluate x^T Q x in its symmetric form (upper triangle of Q)
SYMMETRIC_KERNELS = {"k_proj_q", "k_proj_qc", "k_proj_qb", "k_proj_s"}


def proj_flops_per_point(M, kernel):
    """Algorithmic flops of one spectrum value of an M-element array. A kernel
    in the symmetric form computes x^T Q x as 2 x^T U x over one triangle of
    the 2M x 2M real Q, diagonal included: K (K + 1) / 2 multiply-adds with
    K = 2M, plus the epilogue's K products and K sums (the way a symmetric
    rank-k update is counted at half a GEMM). The full form Q x counts 8M^2,
    plus 8M for its epilogue."""
    if kernel in SYMMETRIC_KERNELS:
        K = 2 * M
        return float(K * (K + 1) + 2 * K)
    return 8.0 * M * M + 8.0 * M


def proj_kernel_name(precision, n_elem, candidates=False):
    """The kernel that evaluates the projection for a precision and array size
    (k_proj_qc: the FP32 register-resident kernel that also emits the peak
    candidates)."""
    if precision == "f32_valu":
        return "k_spec_cov_valu"
    if n_elem > 64:
        return "k_proj_s"
    if precision == "f32":
        return "k_proj_qc" if candidates else "k_proj_q"
    return "k_proj_qb"


def rmse_by_snr(ts, refined_deg, idx):
    """RMSE in degrees per SNR point, estimates associated to the truths
    (sorted pairing on a line, Hungarian on the sphere)."""
    from paper_2604_19723_amd import metrics
    out, fails = {}, 0
    err2 = {}
    for b in range(ts.n_trials):
        if np.any(idx[b] < 0):
            fails += 1
            continue
        e = metrics.associated_errors(refined_deg[b], ts.truth[b])
        err2.setdefault(float(ts.snr_db[b]), []).append(np.mean(e * e))
    for s in sorted(err2):
        out["%g" % s] = float(np.sqrt(np.mean(err2[s])))
    return out, fails


def cpu_baseline(ts, K, seconds):
    """The FP64 oracle on the first trials of the same workload, until the time
    budget is spent, with every BLAS thread and then with one (a third of the
    budget). Steering is built once, outside the clock (as the GPU plan)."""
    from oracle import bartlett as ob
    cores, blas, limits = None, None, None
    try:
        import threadpoolctl
        info = [i for i in threadpoolctl.threadpool_info() if i.get("user_api") == "blas"]
        cores = max([i.get("num_threads", 1) for i in info] or [1])
        blas = ", ".join("%s %s" % (i.get("internal_api"), i.get("version")) for i in info) or None
        limits = threadpoolctl.threadpool_limits
    except Exception:
        pass
    A = ob.steering(ts.pos_wl, ob.directions(ts.grid_kind, ts.grid))

    def run(budget):
        n = 0
        t0 = time.perf_counter()
        while n < ts.n_trials and time.perf_counter() - t0 < budget:
            ob.grid_search(ts.Y[n].astype(np.complex128), ts.pos_wl, ts.grid_kind, ts.grid,
                           ts.grid_shape, ts.wrap0, K, A=A)
            n += 1
        return n, time.perf_counter() - t0

    n, dt = run(seconds)
    out = {"value": n / dt, "unit": "trials/s", "cores": cores, "kind": "oracle",
           "sample": "first %d trials of the timed batch, FP64 numpy (covariance, spectrum via "
                     "zgemm, peaks, refinement), %.1f s" % (n, dt),
           "blas": blas}
    if limits is not None:
        with limits(limits=1, user_api="blas"):
            n1, dt1 = run(seconds / 3)
        out["value_1core"] = n1 / dt1
        out["sample_1core"] = "first %d trials with one BLAS thread, %.1f s" % (n1, dt1)
    return out


def trial_errors(ts, refined_deg, idx):
    """Per trial the associated errors in degrees, None where a peak is missing."""
    from paper_2604_19723_amd import metrics
    return [None if np.any(idx[b] < 0) else metrics.associated_errors(refined_deg[b], ts.truth[b])
            for b in range(ts.n_trials)]


def rmse_se_by_snr(ts, refined_deg, idx, nboot=200):
    """Per SNR point: RMSE in degrees and its bootstrap standard error over
    trials (200 resamples, fixed seed), estimates associated to the truths."""
    from paper_2604_19723_amd import metrics
    per = {}
    for b in range(ts.n_trials):
        if np.any(idx[b] < 0):
            continue
        e = metrics.associated_errors(refined_deg[b], ts.truth[b])
        per.setdefault(float(ts.snr_db[b]), []).append(np.mean(e * e))
    rng = np.random.default_rng(0)
    out = {}
    for s in sorted(per):
        v = np.asarray(per[s])
        boots = [np.sqrt(np.mean(v[rng.integers(0, len(v), len(v))])) for _ in range(nboot)]
        out["%g" % s] = {"rmse": float(np.sqrt(np.mean(v))), "se": float(np.std(boots))}
    return out


def bench_sequential(args, workers):
    """Project-out-and-rescan detection on the ULA 64 workload: one step is the
    covariance plus K passes of (residual covariance, spectrum, top-1 peak)."""
    from paper_2604_19723_amd import workload as wl
    t = time.perf_counter()
    ts = wl.config2(args.trials, dtype=np.complex64, workers=workers)
    log("generated %d trials in %.1f s" % (ts.n_trials, time.perf_counter() - t))
    import torch
    from paper_2604_19723_amd import bartlett as bb
    prec = {"f32": bb.BA_PREC_F32, "bf16x3": bb.BA_PREC_BF16X3}[args.precision]
    B, T, M, K = ts.n_trials, ts.n_snap, ts.n_elem, ts.K
    dev = torch.device("cuda:0")
    Y = torch.from_numpy(ts.Y).to(dev)
    plan = bb.plan_for(ts, prec)
    G = plan.G
    R = torch.empty((B, M, M), dtype=torch.complex64, device=dev)
    idx = torch.empty((B, K), dtype=torch.int32, device=dev)
    val = torch.empty((B, K), dtype=torch.float32, device=dev)
    ref = torch.empty((B, K, 1), dtype=torch.float64, device=dev)
    ws = bb.sequential_workspace_for(plan, B, dev)

    def step(ev=None):
        bb.ba_covariance(plan, B, T, Y, R)
        if ev is not None:
            ev[0].record()
        bb.ba_sequential_peaks(plan, B, R, K, idx, val, ref, ws)
        if ev is not None:
            ev[1].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    seq_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    log("timed %d steps: %.3f ms/step, %d passes %.3f ms" % (args.steps, dt / args.steps * 1e3, K, seq_ms))
    from paper_2604_19723_amd import metrics
    est = metrics.fractional_index_to_deg(ts.grid_kind, ts.grid, ts.grid_shape, ref.cpu().numpy())
    rmse, fails = rmse_by_snr(ts, est, idx.cpu().numpy())
    # the plain top-K search on the same trials, for the accuracy comparison
    out = bb.run_grid_search(plan, Y, K)
    torch.cuda.synchronize()
    est_p = metrics.fractional_index_to_deg(ts.grid_kind, ts.grid, ts.grid_shape, out["refined"].cpu().numpy())
    rmse_plain, fails_plain = rmse_by_snr(ts, est_p, out["idx"].cpu().numpy())
    try:
        bb.ba_candidates_size(plan, B, 1)
        cand = True   # each pass emits its peak candidates
    except bb.BartlettError:
        cand = False
    kname = proj_kernel_name(args.precision, M, cand)
    flops = float(B) * K * G * proj_flops_per_point(M, kname)
    bound, peak = PEAK[args.precision]
    achieved = flops / (seq_ms * 1e-3) / 1e12
    value = B * args.steps / dt
    line = {
        "metric": "MC trials/sec and grid-points*trials/sec at fixed RMSE; % MFMA/HBM peak",
        "value": value, "unit": "trials/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.precision,
        "data": "synthetic (seeded signal model: CN sources + CN noise on a half-wavelength ULA)",
        "config": {"workload": ts.name + "_sequential", "trials": B, "passes": K, "n_elem": M, "n_snap": T,
                   "n_grid": G, "precision": args.precision},
        "roofline": {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "%s x %d passes (residual and peak kernels inside the timed span)" % (kname, K),
                     "kernel_ms": seq_ms, "flops_per_launch": flops},
        "cpu_baseline": None,
        "grid_points_trials_per_s": value * G * K,
        "rmse_deg_by_snr": rmse, "failed_trials": fails,
        "plain_rmse_deg_by_snr": rmse_plain, "plain_failed_trials": fails_plain,
    }
    plan.close()
    return line


def bench_proposal(args, workers):
    """The birth-proposal step on the ULA 64 workload: one step is covariance,
    spectrum, proposal moments and N = 1024 Gaussian particles with importance
    weights per trial (one new feature per trial, as in the paper's proposal)."""
    from paper_2604_19723_amd import workload as wl
    t = time.perf_counter()
    ts = wl.config2(args.trials, dtype=np.complex64, workers=workers)
    log("generated %d trials in %.1f s" % (ts.n_trials, time.perf_counter() - t))
    import torch
    from paper_2604_19723_amd import bartlett as bb
    B, T, M, N = ts.n_trials, ts.n_snap, ts.n_elem, 1024
    dev = torch.device("cuda:0")
    Y = torch.from_numpy(ts.Y).to(dev)
    plan = bb.plan_for(ts, bb.BA_PREC_F32)
    G, d = plan.G, plan.coord_dim
    R = torch.empty((B, M, M), dtype=torch.complex64, device=dev)
    P = torch.empty((B, G), dtype=torch.float32, device=dev)
    mc = torch.empty((B, d + d * d), dtype=torch.float64, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(SEED_PROPOSAL)
    z = torch.randn((B, N, d), dtype=torch.float64, device=dev, generator=gen)
    part = torch.empty((B, N, d), dtype=torch.float64, device=dev)
    w = torch.empty((B, N), dtype=torch.float64, device=dev)
    ws = bb.spectrum_workspace_for(plan, B, dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]

    def step(timed=False):
        bb.ba_covariance(plan, B, T, Y, R)
        if timed:
            ev[0].record()
        bb.ba_spectrum(plan, B, R, P, ws)
        if timed:
            ev[1].record()
        bb.ba_proposal_moments(plan, B, P, mc)
        if timed:
            ev[2].record()
        bb.ba_proposal_sample(plan, B, mc, N, z, part, w)
        if timed:
            ev[3].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    proj, mom, samp = [], [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(True)
        torch.cuda.synchronize()
        proj.append(ev[0].elapsed_time(ev[1]))
        mom.append(ev[1].elapsed_time(ev[2]))
        samp.append(ev[2].elapsed_time(ev[3]))
    dt = time.perf_counter() - t0
    proj_ms, mom_ms, samp_ms = (float(np.mean(x)) for x in (proj, mom, samp))
    log("timed %d steps: %.3f ms/step; projection %.3f, moments %.3f, sampling %.3f ms" % (
        args.steps, dt / args.steps * 1e3, proj_ms, mom_ms, samp_ms))
    flops = float(B) * G * proj_flops_per_point(M, "k_proj_q")
    samp_bytes = float(B) * N * (2 * d + 1) * 8 + B * (d + d * d) * 8     # z in, particles + weights out
    mom_bytes = float(B) * G * 4 + B * (d + d * d) * 8
    wh = w.cpu().numpy()
    ph = part.cpu().numpy()
    ess = 1.0 / np.sum(wh * wh, axis=1)
    value = B * args.steps / dt
    line = {
        "metric": "MC trials/sec and grid-points*trials/sec at fixed RMSE; % MFMA/HBM peak",
        "value": value, "unit": "trials/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 spectrum, f64 proposal",
        "data": "synthetic (seeded signal model: CN sources + CN noise on a half-wavelength ULA; "
                "standard normal draws from torch's seeded device generator)",
        "config": {"workload": ts.name + "_proposal_n1024", "trials": B, "particles": N, "n_grid": G},
        "roofline": {"bound": "mfma", "achieved": flops / (proj_ms * 1e-3) / 1e12, "peak": 157.3,
                     "unit": "TFLOP/s", "frac": flops / (proj_ms * 1e-3) / 1e12 / 157.3, "traffic": None,
                     "kernel": "k_proj_q", "kernel_ms": proj_ms, "flops_per_launch": flops},
        "proposal_kernels": {
            "k_moments": {"ms": mom_ms, "bound": "hbm", "bytes": mom_bytes,
                          "achieved_gb_s": mom_bytes / (mom_ms * 1e-3) / 1e9, "peak_gb_s": 8000.0},
            "k_proposal_sample": {"ms": samp_ms, "bound": "hbm", "bytes": samp_bytes,
                                  "achieved_gb_s": samp_bytes / (samp_ms * 1e-3) / 1e9, "peak_gb_s": 8000.0}},
        "cpu_baseline": None,
        "effective_sample_size_median": float(np.median(ess)),
        "particles_finite": bool(np.all(np.isfinite(ph))),
    }
    plan.close()
    return line


def bench_coherent(args, workers):
    """The paper's own proposal cost: J = 4 URAs (4 x 4, 10 frequency bins),
    coherent over the arrays, 131 072 SFV candidates; one step is the trial
    rows, the fused GEMM + |.|^2, the proposal moments and 1024 birth
    particles per trial for 1024 trials."""
    from paper_2604_19723_amd import workload as wl
    B = args.trials if args.trials != 10000 else 1024
    t = time.perf_counter()
    cs = wl.coherent_config(B, 131072)
    log("generated %d trials in %.1f s" % (B, time.perf_counter() - t))
    import torch
    from paper_2604_19723_amd import bartlett as bb
    dev = torch.device("cuda:0")
    t = time.perf_counter()
    h = bb.ba_coherent_create(cs.pa_pos, cs.pa_rot, cs.n_y, cs.n_z, cs.n_f, cs.fc, cs.bandwidth, cs.p_mt,
                              cs.candidates)
    log("steering table of %d candidates built in %.2f s" % (h.n_cand, time.perf_counter() - t))
    G, K = h.n_cand, h.n_obs
    Z = torch.from_numpy(cs.Z).to(dev)
    P = torch.empty((B, G), dtype=torch.float32, device=dev)
    mc = torch.empty((B, 12), dtype=torch.float64, device=dev)
    ws = bb.coherent_workspace_for(h, B, dev)
    # birth particles of the new feature: 1024 per trial from N(mu, C) in the partition box
    N = 1024
    gen = torch.Generator(device=dev)
    gen.manual_seed(SEED_PROPOSAL)
    zs = torch.randn((B, N, 3), dtype=torch.float64, device=dev, generator=gen)
    part = torch.empty((B, N, 3), dtype=torch.float64, device=dev)
    wgt = torch.empty((B, N), dtype=torch.float64, device=dev)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        bb.ba_coherent_spectrum(h, B, Z, P, ws)
        if ev is not None:
            ev[1].record()
        bb.ba_coherent_moments(h, B, P, mc, ws)
        if ev is not None:
            ev[2].record()
        bb.ba_coherent_sample(h, B, mc, N, zs, part, wgt)
        if ev is not None:
            ev[3].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    mom_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    samp_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    log("timed %d steps: %.3f ms/step, spectrum %.3f ms, moments %.3f ms, sampling %.3f ms" % (
        args.steps, dt / args.steps * 1e3, k_ms, mom_ms, samp_ms))
    wh = wgt.cpu().numpy()
    ess = 1.0 / np.nansum(wh * wh, axis=1)
    flops = 8.0 * K * G * B          # complex inner products of length J N_z
    achieved = flops / (k_ms * 1e-3) / 1e12
    mu = mc[:, :3].cpu().numpy()
    err = np.linalg.norm(mu - cs.sfv_true, axis=1)
    # spot parity on two trials over the first 256 candidates
    from oracle import coherent as oc
    lam = oc.C_LIGHT / cs.fc
    f, py = oc.frequencies(cs.n_f, cs.bandwidth), oc.ura_support(cs.n_y, lam)
    Ph = P[:2, :256].cpu().numpy().astype(np.float64)
    spot = []
    for b in range(2):
        Pr = oc.coherent_spectrum(cs.Z[b].astype(np.complex128), cs.candidates[:256], cs.p_mt, cs.pa_pos,
                                  cs.pa_rot, f, py, py, cs.fc)
        spot.append(float(np.max(np.abs(Ph[b] - Pr)) / np.max(Pr)))
    value = B * args.steps / dt
    line = {
        "metric": "MC trials/sec and grid-points*trials/sec at fixed RMSE; % MFMA/HBM peak",
        "value": value, "unit": "trials/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded: 4 URAs around a room, one reflected path + noise, SNR 20 dB)",
        "config": {"workload": cs.name, "trials": B, "n_cand": G, "n_obs": K, "arrays": 4},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": 157.3, "unit": "TFLOP/s",
                     "frac": achieved / 157.3, "traffic": None, "kernel": "k_coh_rows + k_coh_gemm",
                     "kernel_ms": k_ms, "flops_per_launch": flops},
        "cpu_baseline": None,
        "grid_points_trials_per_s": value * G,
        "argmax_distance_m": {"median": float(np.median(err)), "p90": float(np.percentile(err, 90))},
        "birth_particles": {"per_trial": N, "moments_ms": mom_ms, "sampling_ms": samp_ms,
                            "sampling_gb_s": B * N * (3 * 8 * 2 + 8) / (samp_ms * 1e-3) / 1e9,
                            "effective_sample_size_median": float(np.nanmedian(ess))},
        "spot_parity_normwise_max": max(spot),
    }
    h.close()
    return line


def bench_ragged(args, workers):
    """Uneven batch: one graph replay = one step over all trials."""
    from paper_2604_19723_amd import workload as wl
    n = args.trials if args.trials != 10000 else 50000
    t = time.perf_counter()
    rs = wl.config4(n, dtype=np.complex64, workers=workers)
    log("generated %d ragged trials (%.2f GB) in %.1f s" % (n, rs.pool.nbytes / 1e9, time.perf_counter() - t))
    import torch
    from paper_2604_19723_amd import bartlett as bb
    dev = torch.device("cuda:0")
    G = len(rs.grid)
    plan = bb.ba_plan_create(128, wl.ula_positions(128), bb.BA_GRID_ULA_DEG, G, rs.grid, G, 1, 0)
    Y = torch.from_numpy(rs.pool).to(dev)
    kmax = 8
    P = torch.empty((n, G), dtype=torch.float32, device=dev)
    idx = torch.empty((n, kmax), dtype=torch.int32, device=dev)
    val = torch.empty((n, kmax), dtype=torch.float32, device=dev)
    ref = torch.empty((n, kmax, 1), dtype=torch.float64, device=dev)
    r = bb.ba_ragged_create(plan, bb.ragged_descriptors(rs), kmax, Y, P, idx, val, ref)
    if not args.no_autotune:
        t = time.perf_counter()
        bb.ba_ragged_autotune(r, None, repeats=2, max_probe=256)   # tuned afresh on every run
        log("autotuned in %.1f s: waves along rows per class %s" % (time.perf_counter() - t, bb.ba_ragged_config(r)))
    routes = bb.ba_ragged_routes(r)
    packed = bb.ba_ragged_packed(r)
    log("classes run one trial per wave: %s" % [8 << c for c in range(5) if packed[c]])
    for _ in range(args.warmup):
        bb.ba_ragged_launch(r)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record()
        bb.ba_ragged_launch(r)
        evs[k][1].record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    log("timed %d replays: %.3f ms/step, kernel %.3f ms" % (args.steps, dt / args.steps * 1e3, kms))
    M = rs.n_elem.astype(np.float64)
    T = rs.n_snap.astype(np.float64)
    snap = routes == bb.BA_ROUTE_SNAPSHOTS
    # covariance route: covariance 8M^2T, then the projection in the symmetric
    # form (K (K + 1) + 2K per grid point, K = 2M); snapshot route: |S x|^2, 8MTG
    K2 = 2 * M
    flops = np.where(snap, 8 * M * T * G, 8 * M * M * T + (K2 * (K2 + 1) + 2 * K2) * G).sum()
    achieved = flops / (kms * 1e-3) / 1e12
    from paper_2604_19723_amd import metrics
    est = metrics.fractional_index_to_deg(1, rs.grid, (G, 1), ref.cpu().numpy())
    idx_h = idx.cpu().numpy()
    err2, fails, errs = [], 0, []
    for i in range(n):
        K = int(rs.k[i])
        if np.any(idx_h[i, :K] < 0):
            fails += 1
            errs.append(None)
            continue
        e = metrics.associated_errors(est[i, :K], rs.truth[i])
        errs.append(e)
        err2.append(np.mean(e * e))
    value = n * args.steps / dt
    line = {
        "metric": "MC trials/sec and grid-points*trials/sec at fixed RMSE; % MFMA/HBM peak",
        "value": value, "unit": "trials/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded signal model, uneven ULA trials)",
        "config": {"workload": rs.name, "trials": n, "n_grid": G, "kmax": kmax,
                   "snapshot_route_trials": int(snap.sum()), "autotuned": not args.no_autotune,
                   "packed_classes": [8 << c for c in range(5) if packed[c]]},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": 157.3, "unit": "TFLOP/s",
                     "frac": achieved / 157.3, "traffic": None, "kernel": "persistent ragged kernel",
                     "kernel_ms": kms, "flops_per_launch": float(flops)},
        "cpu_baseline": None,
        "grid_points_trials_per_s": value * G,
        "rmse_deg": float(np.sqrt(np.mean(err2))), "failed_trials": fails,
        "accuracy": metrics.accuracy_summary(errs),
    }
    r.close()
    plan.close()
    return line


def bench_learned(args, workers):
    """Learned proposal vs plain FP32 grid search on the 64-element ULA: train
    on method-labelled trials, pick the fallback threshold on a validation set
    (smallest tau whose RMSE equals the plain RMSE), report the test set."""
    from paper_2604_19723_amd import workload as wl
    n_test = args.trials
    t = time.perf_counter()
    # validation and test sets share the SNR sweep of the plain-method workload
    val = wl.config5(4000, seed_offset=1, snr_db=wl.C2_SNRS, dtype=np.complex64, workers=workers)
    test = wl.config5(n_test, seed_offset=2, snr_db=wl.C2_SNRS, dtype=np.complex64, workers=workers)
    log("generated validation/test sets in %.1f s" % (time.perf_counter() - t))
    import torch
    from paper_2604_19723_amd import bartlett as bb
    from paper_2604_19723_amd import learned as L
    dev = torch.device("cuda:0")
    plan = bb.plan_for(test)
    t = time.perf_counter()
    X, U, Mk = L.make_training_set(plan, args.train_trials, 1234, dev, log=log)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t
    # maximum batch above the test set: inference runs the whole set in one pass (training uses 1024)
    net = bb.ba_mlp_create(4096, 512, 3, 4, 16384, bb.BA_PREC_BF16, 99)
    t = time.perf_counter()
    hist = L.train(net, X, U, Mk, args.epochs, 1024, 1e-3, 7, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t
    del X, U, Mk
    taus = [0.0, 0.02, 0.04, 0.06, 0.08, 0.1, 0.12, 0.14, 0.16, 0.18, 0.2, 0.22, 0.25, 0.3, 0.35, 0.4]
    ev = L.evaluate(plan, net, val, taus, dev)
    chosen = L.choose_tau(ev) or ev["learned"][-1]
    log("validation: plain %s; chosen tau %.2f (fallback %.3f, rmse %s, paired %s)" % (
        ev["plain"]["rmse"], chosen["tau"], chosen["fallback"], chosen["rmse"],
        chosen["accuracy_vs_plain"]["equal"]))
    et = L.evaluate(plan, net, test, [chosen["tau"]], dev, steps=args.steps, warmup=args.warmup)
    lt, pt = et["learned"][0], et["plain"]
    line = {
        "metric": "MC trials/sec and grid-points*trials/sec at fixed RMSE; % MFMA/HBM peak",
        "value": lt["trials_per_s"], "unit": "trials/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": lt["seconds"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 network + f32 windows",
        "data": "synthetic (seeded signal model; training stream drawn on the device)",
        "config": {"workload": test.name + "_learned", "test_trials": n_test,
                   "train_trials": args.train_trials, "epochs": args.epochs, "tau": chosen["tau"],
                   "half_window": 50},
        "roofline": None, "cpu_baseline": None,
        "plain_trials_per_s": pt["trials_per_s"], "speedup_vs_plain": lt["trials_per_s"] / pt["trials_per_s"],
        "rmse_deg": lt["rmse"], "plain_rmse_deg": pt["rmse"],
        "equal_rmse": L.equal_rmse(lt["rmse"], pt["rmse"]), "fallback_rate": lt["fallback"],
        "accuracy_vs_plain": lt["accuracy_vs_plain"], "equal_accuracy": L.equal_accuracy(lt, pt),
        "index_identity_vs_plain": lt["index_identity_vs_plain"],
        "train_seconds": t_train, "data_seconds": t_data, "final_loss": hist[-1] if hist else None,
        "validation": [{k: r[k] for k in ("tau", "fallback", "rmse", "trials_per_s", "index_identity_vs_plain")}
                       | {"equal_accuracy": L.equal_accuracy(r, ev["plain"])} for r in ev["learned"]],
        "validation_plain": ev["plain"],
    }
    net.close()
    plan.close()
    return line


def message_flops(S, P, J, nf, ny, nz):
    """Algorithmic FP64 flops of one message step: (reduction, pair kernel, PF kernel).
    A Kronecker contraction a^H X costs Kc = N_z + N_f N_y + N_f complex MACs (8 flops);
    a Gram entry <a_s, a_t> Nt = N_f + N_y + N_z; an S x S Cholesky 8 S^3 / 6, a solve 4 S^2."""
    Nz, Kc, Nt = nf * ny * nz, nf * ny * nz + nf * ny + nf, nf + ny + nz
    chol = 8.0 * S ** 3 / 6 + 4.0 * S * S
    red = 28.0 * Nz * S * J * P
    pair = J * P * (8.0 * S * Kc + 8.0 * S * S * Nt + 2 * chol)
    pf = S * J * P * (8.0 * S * Kc + 4.0 * S * S)
    return red, pair, pf


def bench_messages(args, workers):
    """Particle update messages of one BP time step (Sec. IV-C, Supplement
    S-V) at the Experiment-1 size: P = 30 000 particles, J = 4 URAs (4 x 4,
    10 bins: N_z = 160), S = 6 features (LOS + 5 surfaces). One step = one
    ba_update_messages call: particle sums, per-(feature, array) setup, MT and
    noise messages at every (particle, array), PF messages at every (feature,
    particle, array), PR messages."""
    from paper_2604_19723_amd import workload as wl
    P = args.trials if args.trials != 10000 else 30000
    t = time.perf_counter()
    ms = wl.message_config(n_part=P)
    log("generated the message workload (P = %d) in %.1f s" % (P, time.perf_counter() - t))
    import torch
    from paper_2604_19723_amd import bartlett as bb
    dev = torch.device("cuda:0")
    S, J = ms.n_feat, len(ms.pa_pos)
    h = bb.ba_msgs_create(ms.pa_pos, ms.pa_rot, ms.n_y, ms.n_z, ms.n_f, ms.fc, ms.bandwidth)
    tens = bb.message_tensors(ms, dev)
    out = dict(log_iota=torch.empty((J, P), dtype=torch.float64, device=dev),
               log_nu=torch.empty((J, P), dtype=torch.float64, device=dev),
               log_kappa=torch.empty((S, J, P), dtype=torch.float64, device=dev),
               log_kappa0=torch.empty((S, J), dtype=torch.float64, device=dev),
               log_omega=torch.empty((S, J, 2), dtype=torch.float64, device=dev))
    ws = bb.messages_workspace_for(h, S, P, dev)
    variants = {"all": out, "prep": {"log_kappa0": out["log_kappa0"]},
                "pf": {"log_kappa": out["log_kappa"]}}

    def call(which):
        bb.ba_update_messages(h, S, P, workspace=ws, **tens, **variants[which])

    def timed(which, n):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for a, b in evs:
            a.record()
            call(which)
            b.record()
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in evs]))

    for _ in range(args.warmup):
        call("all")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        call("all")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_all = timed("all", args.steps)
    ms_prep = timed("prep", args.steps)
    ms_pf = timed("pf", args.steps)
    pf_ms = ms_pf - ms_prep
    log("timed %d steps: %.3f ms/step (events %.3f ms; prep %.3f ms; PF kernel %.3f ms)" % (
        args.steps, dt / args.steps * 1e3, ms_all, ms_prep, pf_ms))
    red, pair, pf = message_flops(S, P, J, ms.n_f, ms.n_y, ms.n_z)
    achieved = pf / (pf_ms * 1e-3) / 1e12
    step_tf = (red + pair + pf) / (ms_all * 1e-3) / 1e12
    got = {k: v.cpu().numpy() for k, v in out.items()}
    # spot parity: three particles against the dense FP64 oracle
    from oracle import messages as om
    parts = [0, P // 2, P - 1]
    ref = om.mt_message(ms, parts=parts)
    spot = float(np.max(np.abs(got["log_iota"][:, parts] - ref) / np.abs(ref)))
    cpu = None
    if not args.no_cpu_baseline:
        cpu = message_cpu_baseline(ms, args.cpu_seconds)
    value = args.steps / dt
    line = {
        "metric": "MC trials/sec and grid-points*trials/sec at fixed RMSE; % MFMA/HBM peak",
        "value": value, "unit": "time steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded: 4 URAs in a room, LOS + 5 surfaces, particle clouds around the truth, "
                "SNR 20 dB)",
        "config": {"workload": ms.name, "particles": P, "features": S, "arrays": J,
                   "n_obs": ms.n_f * ms.n_y * ms.n_z},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s",
                     "frac": achieved / 78.6, "traffic": None, "kernel": "k_msg_kappa",
                     "kernel_ms": pf_ms, "flops_per_launch": pf},
        "cpu_baseline": cpu,
        "pair_messages_per_s": value * J * P,
        "step_tflops_f64": step_tf,
        "step_flops": red + pair + pf,
        "event_ms": {"all": ms_all, "prep": ms_prep, "prep_plus_pf": ms_pf},
    }
    line["spot_parity_rel_max"] = spot
    h.close()
    return line


def message_cpu_baseline(ms, seconds):
    """The FP64 oracle on a sample of particles: particle sums over the sample,
    then every message at the sample's particles; scaled to the full P (all
    parts are linear in P)."""
    import dataclasses
    from oracle import messages as om
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info if i.get("user_api") == "blas"] or [1])
    except Exception:
        cores = None
    n, dt = 0, 0.0
    for n in (2, 4, 8, 16, 32, 64, 128, 256):
        sub = dataclasses.replace(ms, mt_pos=ms.mt_pos[:n], w_beta=ms.w_beta[:n], sfv=ms.sfv[:, :n],
                                  gamma=ms.gamma[:, :n], mu=ms.mu[:, :n], w_alpha=ms.w_alpha[:, :n],
                                  eta=ms.eta[:, :n], w_xi=ms.w_xi[:, :n])
        t0 = time.perf_counter()
        avg = om.particle_averages(sub)
        om.mt_message(sub)
        om.noise_message(sub, avg=avg)
        om.pf_message(sub, avg=avg)
        om.pr_message(sub, avg=avg)
        dt = time.perf_counter() - t0
        if dt > seconds / 3:
            break
    per_step = dt * ms.n_part / n
    return {"value": 1.0 / per_step, "unit": "time steps/s", "cores": cores, "kind": "oracle",
            "sample": "%d of %d particles (all messages + particle sums over the sample, dense FP64 "
                      "numpy), %.1f s, scaled by P" % (n, ms.n_part, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--trials", type=int, default=10000)
    ap.add_argument("--precision", default="f32", choices=sorted(PEAK))
    ap.add_argument("--workload", default="ula64",
                    choices=["ula64", "ura256", "ragged", "learned", "sequential", "proposal", "coherent",
                             "messages"],
                    help="ula64: 64-element ULA, 7201-point grid (default); ura256: 16x16 URA, "
                         "361x181 az/el grid; ragged: 50 000 uneven trials (M 8..128, T 16..2048) "
                         "in one persistent launch under a HIP graph")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--staged-peaks", action="store_true",
                    help="write the spectrum and pick peaks with ba_peaks over it, instead of the "
                         "candidates the FP32 projection emits on 1-D grids")
    ap.add_argument("--train-trials", type=int, default=1000000)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, copy a buffer of this many MiB once (a plain copy kernel "
                         "of known size, to scale hardware byte counters)")
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32-reference", action="store_true",
                    help="with --precision bf16x3|bf16: skip timing the FP32 path on the same trials")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: skip the URA BF16x3, uneven-batch and learned-proposal "
                         "measurements that follow the headline")
    args = ap.parse_args()
    if args.steps < 1 or args.warmup < 0 or args.trials < 1:
        ap.error("--steps >= 1, --warmup >= 0 and --trials >= 1 required")
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the grid search shards by trials with no "
              "cross-GPU exchange in the timed path, so it measures one GPU's share at its "
              "real shape (use --gpus 1)", file=sys.stderr)
        return 2

    workers = min(16, len(os.sched_getaffinity(0)))
    modes = {"ragged": bench_ragged, "learned": bench_learned, "sequential": bench_sequential,
             "proposal": bench_proposal, "coherent": bench_coherent, "messages": bench_messages}
    line = modes.get(args.workload, bench_grid)(args, workers)
    if args.workload == "ula64" and args.precision == "f32" and not args.no_extras:
        line["extras"] = run_extras(args, workers)
    print(json.dumps(line), flush=True)
    return 0


# keys of a bench line that only the headline carries
_LINE_ONLY = ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "cpu_baseline")


def run_extras(args, workers):
    """The other workloads, each at its full size, on the same GPU after the
    headline: the URA in BF16x3 against FP32 on the same trials, the uneven
    batch in one persistent launch under a HIP graph, and the learned proposal
    against the plain FP32 search. Fewer timed steps than the headline (each
    reports its own)."""
    import torch
    steps = max(1, min(args.steps, 5))
    warm = max(1, min(args.warmup, 2))
    base = dict(vars(args))
    base.update(steps=steps, warmup=warm, no_cpu_baseline=True, calib_copy_mib=0, no_autotune=False,
                no_f32_reference=False, no_extras=True)
    jobs = [("ura256_bf16x3_vs_f32", bench_grid, dict(workload="ura256", precision="bf16x3", trials=2000)),
            ("ragged", bench_ragged, dict(workload="ragged", precision="f32", trials=50000)),
            ("learned", bench_learned, dict(workload="learned", precision="f32", trials=10000,
                                            train_trials=1000000, epochs=8))]
    out = {}
    for name, fn, kw in jobs:
        a = argparse.Namespace(**dict(base, **kw))
        t = time.perf_counter()
        try:
            r = fn(a, workers)
            out[name] = {k: v for k, v in r.items() if k not in _LINE_ONLY}
        except Exception as e:  # one failing extra must not cost the headline line
            out[name] = {"error": "%s: %s" % (type(e).__name__, e)}
        out[name]["wall_s"] = time.perf_counter() - t
        log("extra %s done in %.1f s" % (name, out[name]["wall_s"]))
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def bench_grid(args, workers):
    """The plain path (covariance, spectrum, peaks) on the ULA 64 or URA 256
    workload in the chosen precision."""
    from paper_2604_19723_amd import workload as wl
    t = time.perf_counter()
    if args.workload == "ula64":
        ts = wl.config2(args.trials, dtype=np.complex64, workers=workers)   # before the GPU is touched
    else:
        ts = wl.config3(args.trials, dtype=np.complex64, workers=workers)
    log("generated %d trials in %.1f s" % (ts.n_trials, time.perf_counter() - t))

    import torch
    from paper_2604_19723_amd import bartlett as bb
    prec = {"f32": bb.BA_PREC_F32, "bf16x3": bb.BA_PREC_BF16X3, "bf16": bb.BA_PREC_BF16,
            "f32_valu": bb.BA_PREC_F32_VALU}[args.precision]
    B, T, M, K = ts.n_trials, ts.n_snap, ts.n_elem, ts.K
    dev = torch.device("cuda:0")
    Y = torch.from_numpy(ts.Y).to(dev)
    plan = bb.plan_for(ts, prec)
    G = plan.G
    R = torch.empty((B, M, M), dtype=torch.complex64, device=dev)
    P = torch.empty((B, G), dtype=torch.float32, device=dev)
    idx = torch.empty((B, K), dtype=torch.int32, device=dev)
    val = torch.empty((B, K), dtype=torch.float32, device=dev)
    ref = torch.empty((B, K, plan.ndim), dtype=torch.float64, device=dev)
    ws = bb.spectrum_workspace_for(plan, B, dev)
    # FP32 on a 1-D grid: the projection emits the peak candidates and a
    # per-trial merge finishes the pick, so the spectrum is neither re-read
    # nor written (the step's outputs are the peaks)
    use_cand = False
    if not args.staged_peaks:
        try:
            bb.ba_candidates_size(plan, B, K)
            use_cand = True
        except bb.BartlettError:
            pass
    cand = bb.candidates_for(plan, B, K, dev) if use_cand else None
    log("peak pick: %s" % ("candidates from the projection + merge" if use_cand else "ba_peaks over P"))

    def step(ev=None):
        bb.ba_covariance(plan, B, T, Y, R)
        if ev is not None:
            ev[0].record()
        if use_cand:
            bb.ba_spectrum_candidates(plan, B, R, K, None, cand)
        else:
            bb.ba_spectrum(plan, B, R, P, ws)
        if ev is not None:
            ev[1].record()
        if use_cand:
            bb.ba_peaks_merge(plan, B, K, cand, idx, val, ref)
        else:
            bb.ba_peaks(plan, B, P, K, idx, val, ref)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
        log("step %d enqueued" % k) if k == 0 else None
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    proj_times = [a.elapsed_time(b) for a, b in evs]
    proj_ms = float(np.mean(proj_times))
    log("timed %d steps: %.3f ms/step, projection %.3f ms" % (args.steps, dt / args.steps * 1e3, proj_ms))

    kname = proj_kernel_name(args.precision, M, use_cand)
    flops_proj = float(B) * G * proj_flops_per_point(M, kname)
    bound, peak = PEAK[args.precision]
    achieved = flops_proj / (proj_ms * 1e-3) / 1e12

    from paper_2604_19723_amd import metrics
    idx_h = idx.cpu().numpy()
    est_deg = metrics.fractional_index_to_deg(ts.grid_kind, ts.grid, ts.grid_shape, ref.cpu().numpy())
    rmse, fails = rmse_by_snr(ts, est_deg, idx_h)

    # spot parity on a few trials against the oracle
    from oracle import bartlett as ob
    A = ob.steering(ts.pos_wl, ob.directions(ts.grid_kind, ts.grid))
    nspot = 8 if M <= 64 else 2
    if use_cand:
        # the timed step wrote no spectrum: evaluate it for the spot trials from
        # the resident covariances, and check the merged peaks against ba_peaks on it
        bb.ba_spectrum(plan, nspot, R, P, ws)
        i_chk = torch.empty((nspot, K), dtype=torch.int32, device=dev)
        v_chk = torch.empty((nspot, K), dtype=torch.float32, device=dev)
        bb.ba_peaks(plan, nspot, P, K, i_chk, v_chk, None)
        if not (torch.equal(i_chk, idx[:nspot]) and torch.equal(v_chk, val[:nspot])):
            raise RuntimeError("merged candidates differ from ba_peaks on the spot trials")
    P_h = P[:nspot].cpu().numpy().astype(np.float64)
    errs = []
    for b in range(nspot):
        Pr = ob.spectrum(ob.covariance(ts.Y[b].astype(np.complex128)), A)
        errs.append(np.max(np.abs(P_h[b] - Pr)) / np.max(Pr))

    vs_f32 = None
    if args.precision in ("bf16x3", "bf16") and not args.no_f32_reference:
        # the plain FP32 path on the same resident trials, same step structure
        rmse_v = rmse_se_by_snr(ts, est_deg, idx_h)
        with bb.plan_for(ts, bb.BA_PREC_F32) as plan32:
            ws32 = bb.spectrum_workspace_for(plan32, B, dev)
            # the same peak pick as the timed path: candidates + merge where served
            cand32 = None
            if use_cand:
                try:
                    cand32 = bb.candidates_for(plan32, B, K, dev)
                except bb.BartlettError:
                    pass

            def step32():
                bb.ba_covariance(plan32, B, T, Y, R)
                if cand32 is not None:
                    bb.ba_spectrum_candidates(plan32, B, R, K, None, cand32)
                    bb.ba_peaks_merge(plan32, B, K, cand32, idx, val, ref)
                else:
                    bb.ba_spectrum(plan32, B, R, P, ws32)
                    bb.ba_peaks(plan32, B, P, K, idx, val, ref)

            for _ in range(args.warmup):
                step32()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                step32()
            torch.cuda.synchronize()
            dt32 = time.perf_counter() - t0
        idx32 = idx.cpu().numpy()
        est32 = metrics.fractional_index_to_deg(ts.grid_kind, ts.grid, ts.grid_shape, ref.cpu().numpy())
        rmse_f = rmse_se_by_snr(ts, est32, idx32)
        eq = {s_: abs(rmse_v[s_]["rmse"] - rmse_f[s_]["rmse"]) <=
              max(0.01 * rmse_f[s_]["rmse"], 2.0 * max(rmse_v[s_]["se"], rmse_f[s_]["se"]))
              for s_ in rmse_f if s_ in rmse_v}
        f32_tps = B * args.steps / dt32
        acc = metrics.compare_accuracy(trial_errors(ts, est_deg, idx_h), trial_errors(ts, est32, idx32))
        vs_f32 = {"f32_trials_per_s": f32_tps, "ratio": (B * args.steps / dt) / f32_tps,
                  "f32_ms_per_step": dt32 / args.steps * 1e3,
                  "rmse_deg_by_snr": {k_: v_["rmse"] for k_, v_ in rmse_v.items()},
                  "f32_rmse_deg_by_snr": {k_: v_["rmse"] for k_, v_ in rmse_f.items()},
                  "equal_rmse_by_snr": eq, "equal_rmse": bool(eq) and all(eq.values()),
                  "rule": "|RMSE - RMSE_f32| <= max(1 % RMSE_f32, 2 bootstrap SE), per SNR point",
                  "index_identity": metrics.index_identity(idx_h, idx32),
                  "accuracy_vs_f32": acc, "equal_accuracy": acc["equal_accuracy"]}
        log("FP32 on the same trials: %.1f ms/step, ratio %.2f, equal RMSE %s, equal accuracy %s, "
            "index identity %.4f" % (dt32 / args.steps * 1e3, vs_f32["ratio"], vs_f32["equal_rmse"],
                                     acc["equal_accuracy"], vs_f32["index_identity"]))
    if args.calib_copy_mib:
        n = args.calib_copy_mib * 1024 * 256
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read + %d MiB written" % (args.calib_copy_mib, args.calib_copy_mib))
        del src, dst
    cpu = None if args.no_cpu_baseline else cpu_baseline(ts, K, args.cpu_seconds)
    value = B * args.steps / dt
    line = {
        "metric": "MC trials/sec and grid-points*trials/sec at fixed RMSE; % MFMA/HBM peak",
        "value": value,
        "unit": "trials/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f32_valu": "f32", "bf16x3": "bf16x3", "bf16": "bf16"}[args.precision],
        "data": "synthetic (seeded signal model: CN sources + CN noise on a half-wavelength ULA)",
        "config": {"workload": ts.name, "trials": B, "n_elem": M, "n_snap": T, "n_src": K,
                   "n_grid": G, "snr_db": sorted(set(float(x) for x in ts.snr_db)),
                   "precision": args.precision},
        "roofline": {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic("%s|%s|%s|b%d" % (kname, args.precision, ts.name, B)),
                     "kernel": kname, "kernel_ms": proj_ms,
                     "kernel_ms_median": float(np.median(proj_times)),
                     "flops_per_launch": flops_proj,
                     "form": ("symmetric: one triangle of the 2M x 2M real Q"
                              if kname in SYMMETRIC_KERNELS else "full Q"),
                     # the dense count 8M^2G + 8MG of the full complex product, for reference
                     "achieved_dense_count": float(B) * G * (8.0 * M * M + 8.0 * M) / (proj_ms * 1e-3) / 1e12},
        "cpu_baseline": cpu,
        "grid_points_trials_per_s": value * G,
        "rmse_deg_by_snr": rmse,
        "failed_trials": fails,
        "accuracy": metrics.accuracy_summary(trial_errors(ts, est_deg, idx_h)),
        "spot_parity_normwise_max": float(np.max(errs)),
        "peak_pick": ("candidates from the projection epilogue + per-trial merge (spectrum not written)"
                      if use_cand else "ba_peaks over the written spectrum"),
    }
    if vs_f32 is not None:
        line["vs_f32_same_trials"] = vs_f32
    plan.close()
    return line


if __name__ == "__main__":
    sys.exit(main())

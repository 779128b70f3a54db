"""Seeded synthetic workloads for the batched Bartlett grid search.

This module is the input side only. It builds array geometries, search grids
and snapshot matrices drawn from the paper's signal model, and it computes
nothing of the estimator itself (no covariance, no spectrum, no peaks). The
FP64 oracle and the HIP path both consume what it returns.

Signal model (Sec. II-B, eq. (observation-generative); amplitude and noise
laws in Sec. III-A): one snapshot is a sum of steered source amplitudes plus
circular complex white Gaussian noise, y_t = sum_k a(u_k) s_k,t + n_t, with
s_k,t ~ CN(0, 1) and n_t ~ CN(0, sigma^2 I). The spatial response is the
unit-modulus plane-wave response of eq. (spatial-response-y/z):
a_m(u) = exp(+j 2 pi p_m . u) with element positions p_m in wavelengths and
u the unit propagation direction (directional cosines, Supplement S-II).
Element supports are centred about the origin, as the paper requires of its
support vectors (Sec. II-B, after eq. (spatial-response-z)).

Randomness: every trial owns a child seed sequence
``SeedSequence(base, spawn_key=(i,))`` (the i-th child of ``SeedSequence(base)``),
so trial i is the same whatever the batch size. Draw order inside a trial:
K (if random), M (if random), T (if random), SNR (if random), source angles
(rejection sampling for the minimum separation), source amplitudes S
([T][K] complex, real and imaginary parts interleaved), noise N ([T][M]
complex, interleaved the same way).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# grid kinds, same numbering as the C-ABI enum
GRID_DIRS = 0
GRID_ULA_DEG = 1
GRID_AZEL_DEG = 2

SEED_BASE = 0xBA570000


def trial_rng(base: int, i: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(base, spawn_key=(int(i),))))


# --------------------------------------------------------------------------- geometry

def ula_positions(n_elem: int, spacing_wl: float = 0.5) -> np.ndarray:
    """Centred ULA along the y axis, [M][3] in wavelengths (the paper's horizontal
    support p_y of eq. (spatial-response-y) with the elevation at 90 degrees)."""
    p = np.zeros((n_elem, 3))
    p[:, 1] = (np.arange(n_elem) - (n_elem - 1) / 2.0) * spacing_wl
    return p


def ura_positions(nx: int, ny: int, spacing_wl: float = 0.5) -> np.ndarray:
    """Centred horizontal URA in the xy-plane, broadside at the zenith, [nx*ny][3].
    Element m = ix*ny + iy, so the response is a_x (x) a_y in Kronecker order
    (Supplement S-I template, laid horizontally by the orientation matrix)."""
    px = (np.arange(nx) - (nx - 1) / 2.0) * spacing_wl
    py = (np.arange(ny) - (ny - 1) / 2.0) * spacing_wl
    p = np.zeros((nx * ny, 3))
    p[:, 0] = np.repeat(px, ny)
    p[:, 1] = np.tile(py, nx)
    return p


def ula_dirs(theta_deg) -> np.ndarray:
    t = np.deg2rad(np.asarray(theta_deg, dtype=np.float64))
    return np.stack([np.cos(t), np.sin(t), np.zeros_like(t)], axis=-1)


def azel_dirs(az_deg, el_deg) -> np.ndarray:
    az = np.deg2rad(np.asarray(az_deg, dtype=np.float64))
    el = np.deg2rad(np.asarray(el_deg, dtype=np.float64))
    return np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], axis=-1)


def response(pos_wl: np.ndarray, dirs: np.ndarray) -> np.ndarray:
    """Source responses for data generation, [M][K] complex128."""
    ph = pos_wl @ dirs.T
    ph = ph - np.round(ph)
    return np.exp(2j * np.pi * ph)


# --------------------------------------------------------------------------- grids

def ula_grid(n_grid: int) -> np.ndarray:
    """Angles in degrees over [-90, 90], both endpoints included."""
    return np.linspace(-90.0, 90.0, n_grid)


def azel_grid(n_az: int = 361, n_el: int = 181, el_max: float = 90.0) -> np.ndarray:
    """[n_az*n_el][2] (az, el) degrees, az-major (g = i_az*n_el + i_el). Azimuth
    spans [0, 360] with the last column duplicating the first."""
    az = np.linspace(0.0, 360.0, n_az)
    el = np.linspace(0.0, el_max, n_el)
    g = np.empty((n_az * n_el, 2))
    g[:, 0] = np.repeat(az, n_el)
    g[:, 1] = np.tile(el, n_az)
    return g


# --------------------------------------------------------------------------- trials

@dataclasses.dataclass
class TrialSet:
    """A uniform batch: every trial has the same M, T and K."""
    Y: np.ndarray                 # complex128 [B][T][M], snapshot-major
    pos_wl: np.ndarray            # [M][3]
    grid_kind: int
    grid: np.ndarray              # [G] degrees, or [G][2] (az, el) degrees, or [G][3] dirs
    grid_shape: tuple             # (shape0, shape1); shape1 = 1 for 1-D grids
    wrap0: int                    # 0 none, 1 periodic, 2 periodic with duplicate last row
    K: int
    truth: np.ndarray             # [B][K] degrees (1-D) or [B][K][2] (az, el)
    snr_db: np.ndarray            # [B]
    sigma2: np.ndarray            # [B] noise variance used
    name: str = ""

    @property
    def n_trials(self):
        return self.Y.shape[0]

    @property
    def n_snap(self):
        return self.Y.shape[1]

    @property
    def n_elem(self):
        return self.Y.shape[2]

    @property
    def n_grid(self):
        return int(self.grid_shape[0] * self.grid_shape[1])

    def y_c64(self) -> np.ndarray:
        return np.ascontiguousarray(self.Y.astype(np.complex64))

    def rounded(self) -> "TrialSet":
        """The same trials with Y rounded to complex64 (what the device sees)."""
        return dataclasses.replace(self, Y=self.Y.astype(np.complex64).astype(np.complex128))


def _draw_angles_1d(rng, K, lo, hi, min_sep):
    while True:
        th = rng.uniform(lo, hi, size=K)
        if K < 2 or np.min(np.diff(np.sort(th))) >= min_sep:
            return np.sort(th)


def _great_circle_deg(u, v):
    return np.rad2deg(np.arccos(np.clip(np.sum(u * v, axis=-1), -1.0, 1.0)))


def _draw_angles_azel(rng, K, el_lo, el_hi, min_sep):
    while True:
        az = rng.uniform(0.0, 360.0, size=K)
        el = rng.uniform(el_lo, el_hi, size=K)
        d = azel_dirs(az, el)
        ok = True
        for i in range(K):
            for j in range(i + 1, K):
                if _great_circle_deg(d[i], d[j]) < min_sep:
                    ok = False
        if ok:
            return np.stack([az, el], axis=-1)


def noise_variance(snr_db: float, K: int, snr_def: str) -> float:
    """Per-source reading: sigma^2 = 10^(-SNR/10) for unit-power sources. The
    sum-channel reading follows the paper's SNR definition on the summed
    channel power per element (Sec. VI-A, system parameters): sigma^2 = K 10^(-SNR/10)."""
    base = 10.0 ** (-snr_db / 10.0)
    if snr_def == "per_source":
        return base
    if snr_def == "sum_channel":
        return K * base
    raise ValueError(snr_def)


def _snapshots(rng, A, T, sigma2):
    """Y [T][M] = S A^T + N with S [T][K] ~ CN(0, 1) and N [T][M] ~ CN(0, sigma2).
    Draws: S as T*K*2 normals (re, im interleaved, snapshot-major), then N as
    T*M*2 normals in the same order."""
    M, K = A.shape
    s = rng.standard_normal((T, K, 2)).view(np.complex128)[..., 0]
    s *= math.sqrt(0.5)
    n = rng.standard_normal((T, M, 2)).view(np.complex128)[..., 0]
    n *= math.sqrt(0.5 * sigma2)
    y = s @ A.T
    y += n
    return y


def _ula_chunk(args):
    (i0, i1, n_elem, n_src, n_snap, snrs, seed_base, ang_lo, ang_hi, min_sep, snr_def, dtype) = args
    pos = ula_positions(n_elem)
    n = i1 - i0
    Y = np.empty((n, n_snap, n_elem), dtype=dtype)
    truth = np.empty((n, n_src))
    snr = np.empty(n)
    sig = np.empty(n)
    for b in range(n):
        i = i0 + b
        rng = trial_rng(seed_base, i)
        snr[b] = snrs[i % len(snrs)]
        th = _draw_angles_1d(rng, n_src, ang_lo, ang_hi, min_sep)
        sig[b] = noise_variance(snr[b], n_src, snr_def)
        Y[b] = _snapshots(rng, response(pos, ula_dirs(th)), n_snap, sig[b])
        truth[b] = th
    return Y, truth, snr, sig


def _parallel_chunks(fn, n_trials, first_trial, rest, workers):
    bounds = np.linspace(0, n_trials, max(1, workers) * 4 + 1).astype(int)
    jobs = [(first_trial + int(a), first_trial + int(b)) + rest
            for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    if workers <= 1 or n_trials < 256:
        return [fn(j) for j in jobs]
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(fn, jobs))


def make_ula_trials(n_trials: int, n_elem: int, n_src: int, n_snap: int, snr_db, n_grid: int,
                    seed_base: int, first_trial: int = 0, ang_lo=-60.0, ang_hi=60.0,
                    min_sep=5.0, snr_def="per_source", name="", dtype=np.complex128,
                    workers: int = 1) -> TrialSet:
    """Uniform ULA batch. ``snr_db`` is a scalar or a sequence cycled over trials
    (trial i takes snr_db[i % len]). ``dtype=np.complex64`` stores Y rounded to
    what the device reads; ``workers`` > 1 generates in forked processes (call
    it before the process touches the GPU)."""
    snrs = tuple(np.atleast_1d(np.asarray(snr_db, dtype=np.float64)).tolist())
    parts = _parallel_chunks(_ula_chunk, n_trials, first_trial,
                             (n_elem, n_src, n_snap, snrs, seed_base, ang_lo, ang_hi, min_sep,
                              snr_def, dtype), workers)
    Y = np.concatenate([p[0] for p in parts]) if parts else np.empty((0, n_snap, n_elem), dtype)
    cat = lambda k, shp: np.concatenate([p[k] for p in parts]) if parts else np.empty(shp)
    return TrialSet(Y=Y, pos_wl=ula_positions(n_elem), grid_kind=GRID_ULA_DEG,
                    grid=ula_grid(n_grid), grid_shape=(n_grid, 1), wrap0=0, K=n_src,
                    truth=cat(1, (0, n_src)), snr_db=cat(2, (0,)), sigma2=cat(3, (0,)), name=name)


def _ura_chunk(args):
    (i0, i1, nx, ny, n_src, n_snap, sig, seed_base, el_lo, el_hi, min_sep, dtype) = args
    pos = ura_positions(nx, ny)
    n = i1 - i0
    Y = np.empty((n, n_snap, nx * ny), dtype=dtype)
    truth = np.empty((n, n_src, 2))
    for b in range(n):
        rng = trial_rng(seed_base, i0 + b)
        ae = _draw_angles_azel(rng, n_src, el_lo, el_hi, min_sep)
        Y[b] = _snapshots(rng, response(pos, azel_dirs(ae[:, 0], ae[:, 1])), n_snap, sig)
        truth[b] = ae
    return Y, truth


def make_ura_trials(n_trials: int, nx: int, ny: int, n_src: int, n_snap: int, snr_db: float,
                    n_az: int, n_el: int, seed_base: int, first_trial: int = 0,
                    el_lo=0.0, el_hi=80.0, min_sep=5.0, snr_def="per_source",
                    name="", dtype=np.complex128, workers: int = 1) -> TrialSet:
    sig = noise_variance(snr_db, n_src, snr_def)
    parts = _parallel_chunks(_ura_chunk, n_trials, first_trial,
                             (nx, ny, n_src, n_snap, sig, seed_base, el_lo, el_hi, min_sep, dtype),
                             workers)
    M = nx * ny
    Y = np.concatenate([p[0] for p in parts]) if parts else np.empty((0, n_snap, M), dtype)
    truth = np.concatenate([p[1] for p in parts]) if parts else np.empty((0, n_src, 2))
    return TrialSet(Y=Y, pos_wl=ura_positions(nx, ny), grid_kind=GRID_AZEL_DEG,
                    grid=azel_grid(n_az, n_el), grid_shape=(n_az, n_el), wrap0=2, K=n_src,
                    truth=truth, snr_db=np.full(n_trials, float(snr_db)),
                    sigma2=np.full(n_trials, sig), name=name)


# --------------------------------------------------------------------------- the five workloads

C2_SNRS = (-10.0, -5.0, 0.0, 5.0, 10.0, 15.0, 20.0)


def config1(n_trials: int = 100, first_trial: int = 0) -> TrialSet:
    """16-element half-wavelength ULA, 2 sources in [-60, 60] deg (sep >= 5 deg),
    64 snapshots, SNR 10 dB, 1801-point grid over [-90, 90] deg."""
    return make_ula_trials(n_trials, 16, 2, 64, 10.0, 1801, SEED_BASE + 1, first_trial,
                           name="ula16_k2_t64_g1801")


def config2(n_trials: int = 10000, first_trial: int = 0, snr_db=C2_SNRS, dtype=np.complex128,
            workers: int = 1) -> TrialSet:
    """64-element ULA, 4 sources, 256 snapshots, 7201-point grid; the SNR sweep
    -10..20 dB in 5 dB steps is cycled over the trials of one batch."""
    return make_ula_trials(n_trials, 64, 4, 256, snr_db, 7201, SEED_BASE + 2, first_trial,
                           name="ula64_k4_t256_g7201", dtype=dtype, workers=workers)


def config3(n_trials: int = 2000, first_trial: int = 0, dtype=np.complex128,
            workers: int = 1) -> TrialSet:
    """16x16 horizontal URA, 3 sources (az U[0,360), el U[0,80]), 512 snapshots,
    SNR 0 dB, 361x181 az/el grid."""
    return make_ura_trials(n_trials, 16, 16, 3, 512, 0.0, 361, 181, SEED_BASE + 3, first_trial,
                           name="ura16x16_k3_t512_g361x181", dtype=dtype, workers=workers)


# ------------------------------------------------------------------ ragged (uneven) batches

C4_SIZES = (8, 16, 32, 64, 128)


@dataclasses.dataclass
class RaggedSet:
    """Trials of different M, T and K packed into one complex pool.

    Trial i occupies pool[y_offset[i] : y_offset[i] + T_i*M_i] as a [T_i][M_i]
    snapshot-major block. Element positions of trial i are the first M_i rows of
    the centred ULA of that size; the grid is shared."""
    pool: np.ndarray              # complex128 [total]
    y_offset: np.ndarray          # int64 [B] in complex elements
    n_elem: np.ndarray            # int32 [B]
    n_snap: np.ndarray            # int32 [B]
    k: np.ndarray                 # int32 [B]
    truth: List[np.ndarray]       # per trial [K_i] degrees
    snr_db: np.ndarray
    grid: np.ndarray
    grid_kind: int = GRID_ULA_DEG
    name: str = ""

    @property
    def n_trials(self):
        return len(self.y_offset)

    def trial_y(self, i) -> np.ndarray:
        o, M, T = int(self.y_offset[i]), int(self.n_elem[i]), int(self.n_snap[i])
        return self.pool[o:o + M * T].reshape(T, M)

    def pool_c64(self) -> np.ndarray:
        if self.pool.dtype == np.complex64:
            return self.pool
        return np.ascontiguousarray(self.pool.astype(np.complex64))


def _ragged_sizes(rng, t_max):
    K = int(rng.integers(1, 7))
    M = int(C4_SIZES[int(rng.integers(0, len(C4_SIZES)))])
    T = int(np.clip(np.rint(np.exp(rng.uniform(math.log(16.0), math.log(t_max)))), 16, t_max))
    return K, M, T


def config4_layout(n_trials: int = 50000, first_trial: int = 0, t_max: int = 2048):
    """Sizes of the uneven batch without its data: K, M, T per trial (the head
    of each trial's stream) and the trials' complex offsets in the pool.
    Returns (K, M, T, offsets, pool elements)."""
    seed = SEED_BASE + 4
    Ms = np.empty(n_trials, np.int32)
    Ts = np.empty(n_trials, np.int32)
    Ks = np.empty(n_trials, np.int32)
    for b in range(n_trials):
        Ks[b], Ms[b], Ts[b] = _ragged_sizes(trial_rng(seed, first_trial + b), t_max)
    sizes = Ms.astype(np.int64) * Ts
    off = np.zeros(n_trials, np.int64)
    off[1:] = np.cumsum(sizes)[:-1]
    return Ks, Ms, Ts, off, int(sizes.sum())


def config4_trial(i: int, t_max: int = 2048):
    """Trial i of the uneven batch: (Y [T][M] complex128, truth degrees, SNR dB)."""
    rng = trial_rng(SEED_BASE + 4, i)
    K, M, T = _ragged_sizes(rng, t_max)
    s = float(rng.uniform(-10.0, 20.0))
    th = _draw_angles_1d(rng, K, -60.0, 60.0, 5.0)
    y = _snapshots(rng, response(ula_positions(M), ula_dirs(th)), T, noise_variance(s, K, "per_source"))
    return y, th, s


def config4(n_trials: int = 50000, first_trial: int = 0, n_grid: int = 3601,
            t_max: int = 2048, dtype=np.complex128, workers: int = 1) -> RaggedSet:
    """Uneven batch: M uniform over {8,16,32,64,128}, K uniform over 1..6,
    T = clip(rint(exp(U[ln 16, ln t_max])), 16, t_max), SNR ~ U[-10, 20] dB.
    Sizes are drawn first (the head of each trial's stream) to lay out the
    pool; then ``workers`` threads fill their trials in place."""
    Ks, Ms, Ts, off, total = config4_layout(n_trials, first_trial, t_max)
    pool = np.empty(total, dtype)
    snr = np.empty(n_trials)
    truth = [None] * n_trials

    def fill(lo, hi):
        for b in range(lo, hi):
            y, th, s = config4_trial(first_trial + b, t_max)
            pool[off[b]:off[b] + y.size] = y.reshape(-1)
            snr[b] = s
            truth[b] = th

    if workers <= 1 or n_trials < 64:
        fill(0, n_trials)
    else:
        import concurrent.futures as cf
        bounds = np.linspace(0, n_trials, workers * 8 + 1).astype(int)
        with cf.ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(lambda ab: fill(*ab), zip(bounds[:-1], bounds[1:])))
    return RaggedSet(pool=pool, y_offset=off, n_elem=Ms, n_snap=Ts, k=Ks, truth=truth,
                     snr_db=snr, grid=ula_grid(n_grid), name="ragged_m8-128_t16-2048_g3601")


def _c5_chunk(args):
    (i0, i1, seed, K, snr_db, dtype) = args
    pos = ula_positions(64)
    n = i1 - i0
    Y = np.empty((n, 256, 64), dtype=dtype)
    truth = np.empty((n, K))
    snr = np.empty(n)
    sig = np.empty(n)
    for b in range(n):
        i = i0 + b
        rng = trial_rng(seed, i)
        snr[b] = rng.uniform(-10.0, 20.0) if snr_db is None else snr_db[i % len(snr_db)]
        th = _draw_angles_1d(rng, K, -60.0, 60.0, 5.0)
        sig[b] = noise_variance(snr[b], K, "per_source")
        Y[b] = _snapshots(rng, response(pos, ula_dirs(th)), 256, sig[b])
        truth[b] = th
    return Y, truth, snr, sig


def config5(n_trials: int, first_trial: int = 0, seed_offset: int = 0, K: int = 4,
            snr_db: Optional[Sequence[float]] = None, dtype=np.complex128, workers: int = 1) -> TrialSet:
    """Learned-proposal workload: 64-element ULA, K sources, 256 snapshots, SNR
    ~ U[-10, 20] dB per trial (or cycled over ``snr_db``), 7201-point grid.
    ``seed_offset`` separates the training, validation and test streams."""
    seed = SEED_BASE + 5 + (seed_offset << 8)
    snrs = None if snr_db is None else tuple(float(x) for x in snr_db)
    parts = _parallel_chunks(_c5_chunk, n_trials, first_trial, (seed, K, snrs, dtype), workers)
    cat = lambda k: np.concatenate([p[k] for p in parts])
    return TrialSet(Y=cat(0), pos_wl=ula_positions(64), grid_kind=GRID_ULA_DEG, grid=ula_grid(7201),
                    grid_shape=(7201, 1), wrap0=0, K=K, truth=cat(1), snr_db=cat(2), sigma2=cat(3),
                    name="learned_ula64_k4_t256_g7201")


# ------------------------------------------------------------------ coherent multi-array (SFV candidates)
#
# The paper's own birth-proposal workload: J URAs around a room receive a
# wideband pilot from one terminal; the observation of array j is the sum of
# its paths' path-loss compensated responses plus noise (Sec. II-B,
# eq. (observation-generative)). The residual after the known paths is taken
# as exact, so a trial's observation holds the one new path (the reflection
# at the wall whose SFV is to be found) plus white noise.

C_LIGHT = 299792458.0


@dataclasses.dataclass
class CoherentSet:
    Z: np.ndarray                 # complex [B][J][N_z]
    pa_pos: np.ndarray            # [J][3] m
    pa_rot: np.ndarray            # [J][3][3] local -> global
    p_mt: np.ndarray              # [3] m
    n_y: int
    n_z: int
    n_f: int
    fc: float
    bandwidth: float
    sfv_true: np.ndarray          # [3] m
    candidates: np.ndarray        # [G][3] m
    name: str = ""

    @property
    def n_trials(self):
        return self.Z.shape[0]


def _rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _path_response(p_mt, s, p_pa, rot, f_base, p_y, p_z, fc):
    """Response of the reflected path at one array (signal model of Secs. II-A and II-B)."""
    lam = C_LIGHT / fc
    d_mt = p_mt - (p_pa - (2.0 * (p_pa @ s) / (s @ s) - 1.0) * s)   # from the virtual anchor
    w = d_mt - 2.0 * (d_mt @ s) / (s @ s) * s                        # mirrored across the surface
    r = rot.T @ w
    d = math.sqrt(r @ r)
    ph = (-2.0 * math.pi * (fc + f_base)[:, None, None] * d / C_LIGHT
          + 2.0 * math.pi / lam * (p_y[None, :, None] * r[1] / d + p_z[None, None, :] * r[2] / d))
    return (lam / (4.0 * math.pi * d)) * np.exp(1j * ph).reshape(-1)


def coherent_config(n_trials: int = 1024, n_cand: int = 131072, snr_db: float = 20.0, n_f: int = 10,
                    bandwidth: float = 100e6, seed: int = SEED_BASE + 6) -> CoherentSet:
    """J = 4 URAs of 4 x 4 elements at half a wavelength, N_f = 10 bins over
    100 MHz at 3.5 GHz (N_z = 160); arrays near the ceiling corners of a
    6 m x 5 m x 2.5 m room, each turned towards the room's centre; the new
    feature is the wall x = 7 m (SFV (14, 0, 0) m); candidates are uniform in
    the 1 m cube around it. Noise is CN(0, eta) with eta set by the sum-channel
    SNR of Sec. VI-A (mean power of the noise-free observation over the N_z J
    entries, divided by the SNR). The amplitude is common to the arrays (unit
    modulus, uniform phase per trial): the phase-coherent case the coherent
    cost is built for."""
    fc = 3.5e9
    lam = C_LIGHT / fc
    centre = np.array([4.0, 3.5])
    pa = np.array([[1.5, 1.5, 2.5], [6.5, 1.5, 2.5], [6.5, 5.5, 2.5], [1.5, 5.5, 2.5]])
    rots = np.stack([_rot_z(math.atan2(centre[1] - p[1], centre[0] - p[0])) for p in pa])
    p_mt = np.array([3.2, 2.8, 1.2])
    s_true = np.array([14.0, 0.0, 0.0])
    n_y = n_z = 4
    f_base = (np.arange(n_f) - (n_f - 1) / 2.0) * (bandwidth / (n_f - 1)) if n_f > 1 else np.zeros(1)
    p_y = (np.arange(n_y) - (n_y - 1) / 2.0) * lam / 2
    p_z = (np.arange(n_z) - (n_z - 1) / 2.0) * lam / 2
    Psi = np.stack([_path_response(p_mt, s_true, pa[j], rots[j], f_base, p_y, p_z, fc) for j in range(4)])
    J, N = Psi.shape
    crng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(0xC0,))))
    cand = s_true + crng.uniform(-0.5, 0.5, size=(n_cand, 3))
    Z = np.empty((n_trials, J, N), np.complex64)
    for b in range(n_trials):
        rng = trial_rng(seed, b)
        rho = np.exp(2j * math.pi * rng.uniform())      # one amplitude, phase-coherent across the arrays
        clean = rho * Psi
        eta = np.mean(np.abs(clean) ** 2) / 10 ** (snr_db / 10)
        noise = rng.standard_normal((J, N, 2)) @ np.array([1.0, 1j]) * math.sqrt(eta / 2)
        Z[b] = clean + noise
    return CoherentSet(Z=Z, pa_pos=pa, pa_rot=rots, p_mt=p_mt, n_y=n_y, n_z=n_z, n_f=n_f, fc=fc,
                       bandwidth=bandwidth, sfv_true=s_true, candidates=cand,
                       name="coherent_j4_ura4x4_nf%d_g%d" % (n_f, n_cand))


# --------------------------------------------------------------------------- particle update messages

@dataclasses.dataclass
class MessageSet:
    """One time step of the particle-based update messages (Sec. IV-C and
    Supplementary Sec. S-V): the observation of every array and the particle
    representations the messages are evaluated on. Feature s = 0 is the
    line-of-sight path; features s >= 1 are surfaces given by their SFVs."""
    z: np.ndarray           # complex128 [J][N_z] observation of each array
    mt_pos: np.ndarray      # [P][3] m, MT state particles (positions)
    w_beta: np.ndarray      # [P] MT particle weights (sum 1)
    sfv: np.ndarray         # [S][P][3] m, SFV particles (row 0 unused: LOS)
    gamma: np.ndarray       # [S][P] amplitude prior variance particles
    mu: np.ndarray          # complex128 [S][P] amplitude prior mean particles
    w_alpha: np.ndarray     # [S][P] PF particle weights (sum = existence probability)
    zeta: np.ndarray        # [S][J] PR existence probabilities zeta(r = 1)
    eta: np.ndarray         # [J][P] noise variance particles
    w_xi: np.ndarray        # [J][P] noise particle weights (sum 1 per array)
    pa_pos: np.ndarray      # [J][3] m
    pa_rot: np.ndarray      # [J][3][3] local -> global
    n_y: int
    n_z: int
    n_f: int
    fc: float
    bandwidth: float
    name: str = ""

    @property
    def n_feat(self):
        return self.gamma.shape[0]

    @property
    def n_part(self):
        return self.mt_pos.shape[0]


def _los_response(p_mt, p_pa, rot, f_base, p_y, p_z, fc):
    """Response of the direct path at one array (signal model of Secs. II-A and II-B)."""
    lam = C_LIGHT / fc
    r = rot.T @ (p_mt - p_pa)
    d = math.sqrt(r @ r)
    ph = (-2.0 * math.pi * (fc + f_base)[:, None, None] * d / C_LIGHT
          + 2.0 * math.pi / lam * (p_y[None, :, None] * r[1] / d + p_z[None, None, :] * r[2] / d))
    return (lam / (4.0 * math.pi * d)) * np.exp(1j * ph).reshape(-1)


# walls x = 1, x = 7, y = 1, y = 6 and the ceiling z = 2.5 of the room: SFV = the
# origin mirrored across each surface
MSG_SFVS = np.array([[2.0, 0.0, 0.0], [14.0, 0.0, 0.0], [0.0, 2.0, 0.0], [0.0, 12.0, 0.0], [0.0, 0.0, 5.0]])


def message_config(n_part: int = 30000, n_feat: int = 6, snr_db: float = 20.0, n_f: int = 10,
                   bandwidth: float = 100e6, spread: float = 0.05, seed: int = SEED_BASE + 7,
                   n_y: int = 4, n_z: int = 4) -> MessageSet:
    """Experiment-1 sized message workload: J = 4 URAs of 4 x 4 elements at half
    a wavelength, N_f = 10 bins over 100 MHz at 3.5 GHz (N_z = 160), P = 30 000
    particles, S = 6 features (LOS plus the four walls and the ceiling of a
    6 m x 5 m x 2.5 m room). Arrays hang 0.3 m below the ceiling near its
    corners, turned towards the room's centre.

    Observation: per array, the sum over features of the path response times
    an amplitude drawn from CN(mu_s, gamma_s) (mu_s common to the arrays:
    |mu| = 1 for LOS, 0.6 for surfaces, uniform phase; gamma_s = 0.01 |mu_s|^2),
    plus CN(0, eta) noise, eta set by the SNR over the mean power of the
    noise-free observation. Particles: MT positions N(p_mt, spread^2 I); SFV
    positions N(s_true, spread^2 I); gamma particles gamma_s U(0.5, 1.5); mu
    particles mu_s + CN(0, (0.05 |mu_s|)^2); MT weights (1 + 0.2 U(-1, 1))
    normalised; PF weights (existence e_s = 0.99, 0.9, 0.8, 0.7, 0.6, 0.5, ...)
    e_s (1 + 0.2 U(-1, 1)) / sum; zeta U(0.5, 1); noise particles
    eta U(0.5, 2), weights 1/P. With n_feat above 6, the extra features reuse
    the surfaces in order with SFVs moved by 0.25 m. n_y x n_z sets the URA
    (4 x 4 in the paper's experiments)."""
    if not 1 <= n_feat <= 16:
        raise ValueError("n_feat must be in [1, 16]")
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(0x3E55,))))
    fc = 3.5e9
    lam = C_LIGHT / fc
    centre = np.array([4.0, 3.5])
    pa = np.array([[1.5, 1.5, 2.2], [6.5, 1.5, 2.2], [6.5, 5.5, 2.2], [1.5, 5.5, 2.2]])
    rots = np.stack([_rot_z(math.atan2(centre[1] - p[1], centre[0] - p[0])) for p in pa])
    p_mt = np.array([3.2, 2.8, 1.2])
    J = len(pa)
    f_base = (np.arange(n_f) - (n_f - 1) / 2.0) * (bandwidth / (n_f - 1)) if n_f > 1 else np.zeros(1)
    p_y = (np.arange(n_y) - (n_y - 1) / 2.0) * lam / 2
    p_z = (np.arange(n_z) - (n_z - 1) / 2.0) * lam / 2
    S, P = n_feat, n_part
    sfv_true = np.zeros((S, 3))
    for s in range(1, S):
        base = MSG_SFVS[(s - 1) % len(MSG_SFVS)]
        sfv_true[s] = base + 0.25 * ((s - 1) // len(MSG_SFVS)) * base / np.linalg.norm(base)
    mu_true = np.exp(2j * math.pi * rng.uniform(size=S)) * np.where(np.arange(S) == 0, 1.0, 0.6)
    gamma_true = 0.01 * np.abs(mu_true) ** 2
    N = n_f * n_y * n_z
    clean = np.zeros((J, N), np.complex128)
    for j in range(J):
        for s in range(S):
            amp = mu_true[s] + math.sqrt(gamma_true[s] / 2) * (rng.standard_normal() + 1j * rng.standard_normal())
            if s == 0:
                psi = _los_response(p_mt, pa[j], rots[j], f_base, p_y, p_z, fc)
            else:
                psi = _path_response(p_mt, sfv_true[s], pa[j], rots[j], f_base, p_y, p_z, fc)
            clean[j] += amp * psi
    eta_true = np.mean(np.abs(clean) ** 2) / 10 ** (snr_db / 10)
    z = clean + math.sqrt(eta_true / 2) * (rng.standard_normal((J, N)) + 1j * rng.standard_normal((J, N)))
    mt_pos = p_mt + spread * rng.standard_normal((P, 3))
    w_beta = 1.0 + 0.2 * rng.uniform(-1, 1, size=P)
    w_beta /= w_beta.sum()
    sfv = np.zeros((S, P, 3))
    sfv[1:] = sfv_true[1:, None, :] + spread * rng.standard_normal((S - 1, P, 3))
    gamma = gamma_true[:, None] * rng.uniform(0.5, 1.5, size=(S, P))
    mu = mu_true[:, None] + 0.05 * np.abs(mu_true)[:, None] * (
        rng.standard_normal((S, P)) + 1j * rng.standard_normal((S, P))) / math.sqrt(2)
    exist = np.array([0.99, 0.9, 0.8, 0.7, 0.6, 0.5] + [0.5] * 10)[:S]
    w_alpha = 1.0 + 0.2 * rng.uniform(-1, 1, size=(S, P))
    w_alpha *= (exist / w_alpha.sum(axis=1))[:, None]
    zeta = rng.uniform(0.5, 1.0, size=(S, J))
    eta = eta_true * rng.uniform(0.5, 2.0, size=(J, P))
    w_xi = np.full((J, P), 1.0 / P)
    return MessageSet(z=z, mt_pos=mt_pos, w_beta=w_beta, sfv=sfv, gamma=gamma, mu=mu, w_alpha=w_alpha,
                      zeta=zeta, eta=eta, w_xi=w_xi, pa_pos=pa, pa_rot=rots, n_y=n_y, n_z=n_z, n_f=n_f,
                      fc=fc, bandwidth=bandwidth,
                      name="messages_j4_ura%dx%d_nf%d_s%d_p%d" % (n_y, n_z, n_f, S, P))

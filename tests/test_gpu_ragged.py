"""Uneven batches in one persistent launch under a HIP graph: every trial
against the FP64 oracle on its own centred array, both routes, graph replay
determinism, and the autotuner."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bartlett as ob
from paper_2604_19723_amd import bartlett as bb
from paper_2604_19723_amd import workload as wl

from parity_util import check_peaks_same_precision, normwise_err, peak_agreement_fp64

pytestmark = pytest.mark.gpu
DEV = "cuda"
KMAX = 8


def ragged_plan(G=3601, M=128):
    return bb.ba_plan_create(M, wl.ula_positions(M), bb.BA_GRID_ULA_DEG, G, wl.ula_grid(G), G, 1, 0)


def run(rs, route=bb.BA_ROUTE_AUTO, autotune=None, replays=1, plan=None):
    B, G = rs.n_trials, len(rs.grid)
    own_plan = plan is None
    plan = ragged_plan(G) if own_plan else plan
    Y = torch.from_numpy(rs.pool_c64()).to(DEV)
    P = torch.full((B, G), -1.0, dtype=torch.float32, device=DEV)
    idx = torch.empty((B, KMAX), dtype=torch.int32, device=DEV)
    val = torch.empty((B, KMAX), dtype=torch.float32, device=DEV)
    ref = torch.empty((B, KMAX, plan.ndim), dtype=torch.float64, device=DEV)
    desc = bb.ragged_descriptors(rs, route)
    with bb.ba_ragged_create(plan, desc, KMAX, Y, P, idx, val, ref) as r:
        if autotune is not None:
            bb.ba_ragged_autotune(r, autotune, repeats=1, max_probe=64)
        outs = []
        for _ in range(replays):
            bb.ba_ragged_launch(r)
            torch.cuda.synchronize()
            outs.append((P.clone(), idx.clone(), val.clone(), ref.clone()))
            # eager work on the same stream between replays
            x = torch.randn(512, 512, device=DEV)
            (x @ x).sum().item()
        routes = bb.ba_ragged_routes(r)
        cfg = bb.ba_ragged_config(r)
        packed = bb.ba_ragged_packed(r)
    if own_plan:
        plan.close()
    P, idx, val, ref = [t.cpu().numpy() for t in outs[0]]
    return dict(P=P, idx=idx, val=val, ref=ref, routes=routes, cfg=cfg, packed=packed, outs=outs)


def check(rs, o, fp64_peaks=True, positions=None, grid_kind=ob.GRID_ULA_DEG, wrap0=0, shape=None):
    """Every trial against the oracle on the plan's first M elements
    (positions: the plan's [M_plan][3] geometry; default the ULA; shape: the
    grid's (rows, columns), default one column)."""
    pool = rs.pool_c64().astype(np.complex128)
    bad, ncmp = [], 0
    emax = 0.0
    for i in range(rs.n_trials):
        M, T, K = int(rs.n_elem[i]), int(rs.n_snap[i]), int(rs.k[i])
        Yi = pool[rs.y_offset[i]:rs.y_offset[i] + M * T].reshape(T, M)
        pos = wl.ula_positions(M) if positions is None else positions[:M]
        A = ob.steering(pos, ob.directions(grid_kind, rs.grid))
        Pref = ob.spectrum(ob.covariance(Yi), A)
        e = normwise_err(o["P"][i][None], Pref[None])[0]
        emax = max(emax, e)
        assert e <= 1e-5, (i, M, T, K, e, o["routes"][i])
        G = len(rs.grid)
        shp = (G, 1) if shape is None else shape
        check_peaks_same_precision(o["P"][i][None], o["idx"][i][None, :K], o["val"][i][None, :K],
                                   o["ref"][i][None, :K], K, shp, wrap0)
        assert np.all(o["idx"][i, K:] == -1) and np.all(np.isnan(o["val"][i, K:]))
        if fp64_peaks:
            n, _, b = peak_agreement_fp64(Pref[None], o["idx"][i][None, :K], K, shp, wrap0, 1e-5)
            ncmp += n
            bad += b
    assert not bad, bad[:3]
    return emax


def test_config4_subset_auto_routes():
    rs = wl.config4(400)
    o = run(rs)
    assert 0 < np.sum(o["routes"] == bb.BA_ROUTE_SNAPSHOTS) < rs.n_trials
    print("ragged normwise max", check(rs, o))


@pytest.mark.parametrize("route", [bb.BA_ROUTE_COV, bb.BA_ROUTE_SNAPSHOTS])
def test_forced_routes(route):
    rs = wl.config4(150, first_trial=1000)
    if route == bb.BA_ROUTE_SNAPSHOTS:
        keep = [i for i in range(rs.n_trials)
                if ((int(rs.n_snap[i]) + 7) & ~7) <= (8 << [8, 16, 32, 64, 128].index(
                    next(c for c in (8, 16, 32, 64, 128) if rs.n_elem[i] <= c)))]
        rs = _subset(rs, keep)
    o = run(rs, route=route)
    assert np.all(o["routes"] == route)
    check(rs, o)


def _subset(rs, keep):
    blocks = [rs.trial_y(i).reshape(-1) for i in keep]
    sizes = np.array([b.size for b in blocks], np.int64)
    off = np.zeros(len(keep), np.int64)
    off[1:] = np.cumsum(sizes)[:-1]
    return wl.RaggedSet(pool=np.concatenate(blocks), y_offset=off, n_elem=rs.n_elem[keep],
                        n_snap=rs.n_snap[keep], k=rs.k[keep], truth=[rs.truth[i] for i in keep],
                        snr_db=rs.snr_db[keep], grid=rs.grid)


def test_edge_trials():
    rng = np.random.default_rng(5)
    Ms = [1, 3, 8, 9, 17, 33, 100, 128, 128, 64]
    Ts = [1, 2, 7, 300, 1, 5, 40, 24, 200, 64]
    Ks = [1, 8, 2, 8, 3, 1, 6, 4, 8, 5]
    blocks = [(rng.standard_normal((T, M)) + 1j * rng.standard_normal((T, M))).reshape(-1)
              for M, T in zip(Ms, Ts)]
    sizes = np.array([b.size for b in blocks], np.int64)
    off = np.zeros(len(Ms), np.int64)
    off[1:] = np.cumsum(sizes)[:-1]
    rs = wl.RaggedSet(pool=np.concatenate(blocks), y_offset=off, n_elem=np.array(Ms, np.int32),
                      n_snap=np.array(Ts, np.int32), k=np.array(Ks, np.int32), truth=[None] * len(Ms),
                      snr_db=np.zeros(len(Ms)), grid=wl.ula_grid(1001))
    o = run(rs)
    check(rs, o, fp64_peaks=False)


def test_graph_replays_are_bitwise_identical():
    rs = wl.config4(120, first_trial=5000)
    o = run(rs, replays=3)
    ibits = {4: torch.int32, 8: torch.int64}
    for later in o["outs"][1:]:
        for a, b in zip(o["outs"][0], later):
            # bitwise: NaN slots (fewer peaks than kmax) must match too
            assert torch.equal(a.view(ibits[a.element_size()]), b.view(ibits[b.element_size()]))


def test_autotune_keeps_parity_and_uses_cache(tmp_path):
    rs = wl.config4(200, first_trial=9000)
    cache = str(tmp_path / "tune.txt")
    o = run(rs, autotune=cache)
    check(rs, o)
    text = open(cache).read()
    assert "|wr|" in text
    o2 = run(rs, autotune=cache)          # second run reads the cache
    assert np.array_equal(o["cfg"], o2["cfg"])


def test_rebinding_buffers_retargets_the_graph():
    rs = wl.config4(160, first_trial=7000)
    B, G = rs.n_trials, len(rs.grid)
    plan = ragged_plan(G)
    YA = torch.from_numpy(rs.pool_c64()).to(DEV)
    gen = torch.Generator(device=DEV)
    gen.manual_seed(3)
    YB = torch.randn(YA.numel(), dtype=torch.complex64, device=DEV, generator=gen)

    def outs():
        return (torch.full((B, G), -1.0, dtype=torch.float32, device=DEV),
                torch.empty((B, KMAX), dtype=torch.int32, device=DEV),
                torch.empty((B, KMAX), dtype=torch.float32, device=DEV),
                torch.empty((B, KMAX, 1), dtype=torch.float64, device=DEV))

    desc = bb.ragged_descriptors(rs)
    oa, ob_ = outs(), outs()
    with bb.ba_ragged_create(plan, desc, KMAX, YA, *oa) as r:
        bb.ba_ragged_launch(r)
        bb.ba_ragged_bind(r, YB, *ob_)
        bb.ba_ragged_launch(r)
        torch.cuda.synchronize()
        ra = [t.clone() for t in oa]
        routes = bb.ba_ragged_routes(r)
        with pytest.raises(bb.BartlettError):
            bb.ba_ragged_bind(r, YA[:10], *outs())     # a pool that misses the trials' blocks
    # the reference: a handle created on the second set of buffers
    oref = outs()
    with bb.ba_ragged_create(plan, desc, KMAX, YB, *oref) as r2:
        bb.ba_ragged_launch(r2)
        torch.cuda.synchronize()
    plan.close()
    ibits = {4: torch.int32, 8: torch.int64}
    for a, b in zip(ob_, oref):
        assert torch.equal(a.view(ibits[a.element_size()]), b.view(ibits[b.element_size()]))
    # the first set holds the first launch's results: the oracle on pool A
    o = dict(P=ra[0].cpu().numpy(), idx=ra[1].cpu().numpy(), val=ra[2].cpu().numpy(), ref=ra[3].cpu().numpy(),
             routes=routes)
    check(rs, o)


def _with_pack(cache, value):
    """Rewrite the packing choices in an autotune cache file to `value`."""
    lines = []
    for line in open(cache).read().splitlines():
        key, v = line.rsplit(" ", 1)
        lines.append("%s %d" % (key, value) if "|pack|" in key else line)
    open(cache, "w").write("\n".join(lines) + "\n")


def test_packed_and_whole_workgroup_small_trials_agree(tmp_path):
    """The 8-, 16- and 32-element classes run packed (one trial per wave) or
    one per workgroup, as the autotune cache says: both against the oracle,
    and spectra within the sum of the two parity gates."""
    rs = wl.config4(500, first_trial=20000)
    keep = [i for i in range(rs.n_trials) if rs.n_elem[i] <= 32]
    rs = _subset(rs, keep)
    print("small trials:", rs.n_trials, flush=True)
    cache = str(tmp_path / "tune.txt")
    o_tuned = run(rs, autotune=cache)
    assert "|pack|" in open(cache).read()
    runs = {}
    for value in (0, 1):
        _with_pack(cache, value)
        o = run(rs, autotune=cache)
        assert list(o["packed"][:3]) == [value] * 3, o["packed"]
        check(rs, o)
        runs[value] = o
    d = np.abs(runs[0]["P"].astype(np.float64) - runs[1]["P"]).max(axis=1) / runs[0]["P"].max(axis=1)
    assert d.max() <= 2e-5, d.max()  # each within 1e-5 of the oracle
    del o_tuned


@pytest.mark.parametrize("wrap0", [0, 1, 2])
def test_packed_trials_on_a_wrapping_direction_grid(wrap0):
    """Packed trials on a 1-D azimuth circle (wrap of the row, and a
    duplicated last direction with wrap0 = 2): the end columns of the row
    are maxima or not by the wrapped rule."""
    G, Mp = 721, 32
    az = np.linspace(0.0, 2 * np.pi, G, endpoint=(wrap0 == 2))
    dirs = np.stack([np.cos(az), np.sin(az), np.zeros_like(az)], axis=1)
    rng = np.random.default_rng(41 + wrap0)
    pos = np.zeros((Mp, 3))
    pos[:, 0] = 0.5 * np.arange(Mp)
    pos[:, 1] = 0.25 * rng.standard_normal(Mp)   # not symmetric about the x axis
    Ms = [1, 2, 5, 8, 9, 12, 16, 16, 3, 16, 7, 14, 17, 32, 25, 32]
    Ts = [40, 3, 300, 20, 64, 1000, 17, 2048, 100, 33, 9, 128, 50, 700, 2, 31]
    Ks = [1, 2, 3, 8, 4, 5, 6, 2, 1, 8, 3, 7, 4, 8, 2, 5]
    blocks = [(rng.standard_normal((T, M)) + 1j * rng.standard_normal((T, M))).reshape(-1)
              for M, T in zip(Ms, Ts)]
    sizes = np.array([b.size for b in blocks], np.int64)
    off = np.zeros(len(Ms), np.int64)
    off[1:] = np.cumsum(sizes)[:-1]
    rs = wl.RaggedSet(pool=np.concatenate(blocks), y_offset=off, n_elem=np.array(Ms, np.int32),
                      n_snap=np.array(Ts, np.int32), k=np.array(Ks, np.int32), truth=[None] * len(Ms),
                      snr_db=np.zeros(len(Ms)), grid=dirs)
    with bb.ba_plan_create(Mp, pos, bb.BA_GRID_DIRS, G, dirs, G, 1, wrap0) as plan:
        o = run(rs, route=bb.BA_ROUTE_COV, plan=plan)
    assert list(o["packed"][:3]) == [1, 1, 1]
    check(rs, o, fp64_peaks=False, positions=pos, grid_kind=ob.GRID_DIRS, wrap0=wrap0)


@pytest.mark.parametrize("wrap0", [0, 1])
def test_whole_workgroup_trials_on_an_azimuth_elevation_grid(wrap0):
    """A 2-D az/el grid (rows = azimuths, columns = elevations; wrap0 = 1
    closes the azimuth circle): the whole-workgroup peak pick over a 2-D
    spectrum row (eight neighbours, the earlier ones strictly below), every
    size class, refinement in both dimensions, against the oracle's spectrum
    and its 2-D peak rule on the same FP32 values."""
    az = np.arange(0.0, 360.0, 6.0) if wrap0 else np.arange(-60.0, 61.0, 4.0)
    el = np.arange(0.0, 41.0, 5.0)
    grid = np.array([(a, e) for a in az for e in el])
    rows, s1 = len(az), len(el)
    Mp = 128
    rng = np.random.default_rng(97 + wrap0)
    pos = np.zeros((Mp, 3))
    pos[:, 0] = 0.5 * (np.arange(Mp) % 16)
    pos[:, 1] = 0.5 * (np.arange(Mp) // 16)
    pos[:, 2] = 0.1 * rng.standard_normal(Mp)   # not a symmetric planar array
    Ms = [128, 100, 64, 40, 33, 32, 24, 16, 9, 8, 5, 3, 128, 64]
    Ts = [300, 50, 1000, 64, 7, 200, 3, 90, 2048, 16, 40, 5, 20, 33]
    Ks = [4, 8, 1, 3, 2, 6, 5, 7, 2, 8, 3, 1, 6, 5]
    blocks = [(rng.standard_normal((T, M)) + 1j * rng.standard_normal((T, M))).reshape(-1)
              for M, T in zip(Ms, Ts)]
    sizes = np.array([b.size for b in blocks], np.int64)
    off = np.zeros(len(Ms), np.int64)
    off[1:] = np.cumsum(sizes)[:-1]
    rs = wl.RaggedSet(pool=np.concatenate(blocks), y_offset=off, n_elem=np.array(Ms, np.int32),
                      n_snap=np.array(Ts, np.int32), k=np.array(Ks, np.int32), truth=[None] * len(Ms),
                      snr_db=np.zeros(len(Ms)), grid=grid)
    with bb.ba_plan_create(Mp, pos, bb.BA_GRID_AZEL_DEG, len(grid), grid, rows, s1, wrap0) as plan:
        assert plan.ndim == 2
        o = run(rs, plan=plan)
    assert o["ref"].shape[-1] == 2
    check(rs, o, fp64_peaks=False, positions=pos, grid_kind=ob.GRID_AZEL_DEG, wrap0=wrap0, shape=(rows, s1))

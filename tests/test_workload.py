"""Seeded workload generator: shapes, per-trial reproducibility, and the
statistics the signal model fixes (per-element power = K + sigma^2 for
unit-power sources and unit-modulus responses)."""
import numpy as np

from paper_2604_19723_amd import workload as wl


def test_trial_independent_of_batch_size():
    a = wl.config1(5)
    b = wl.config1(2, first_trial=3)
    np.testing.assert_array_equal(a.Y[3:], b.Y)
    np.testing.assert_array_equal(a.truth[3:], b.truth)


def test_config1_shapes_and_angles():
    ts = wl.config1(20)
    assert ts.Y.shape == (20, 64, 16) and ts.n_grid == 1801
    assert np.all(np.abs(ts.truth) <= 60) and np.all(np.diff(ts.truth, axis=1) >= 5)
    assert ts.grid[0] == -90 and ts.grid[-1] == 90 and abs(ts.grid[1] - ts.grid[0] - 0.1) < 1e-12


def test_per_element_power():
    ts = wl.make_ula_trials(200, 8, 3, 64, 0.0, 181, 12345)
    p = np.mean(np.abs(ts.Y) ** 2)
    assert abs(p - (3 + 1.0)) < 0.1


def test_sum_channel_snr_reading():
    assert wl.noise_variance(10.0, 4, "sum_channel") == 4 * wl.noise_variance(10.0, 4, "per_source")


def test_config2_snr_cycle():
    ts = wl.config2(14)
    assert list(ts.snr_db[:7]) == list(wl.C2_SNRS) and list(ts.snr_db[7:]) == list(wl.C2_SNRS)


def test_config3_geometry():
    ts = wl.config3(2)
    assert ts.Y.shape == (2, 512, 256) and ts.grid_shape == (361, 181) and ts.wrap0 == 2
    assert np.all(ts.truth[..., 1] <= 80) and np.all(ts.truth[..., 0] < 360)
    # centred aperture, Kronecker order x-major
    assert np.allclose(ts.pos_wl.mean(0), 0) and ts.pos_wl[1, 0] == ts.pos_wl[0, 0]


def test_config4_ragged_pool():
    rs = wl.config4(300)
    assert set(np.unique(rs.n_elem)) <= set(wl.C4_SIZES)
    assert rs.n_snap.min() >= 16 and rs.n_snap.max() <= 2048
    assert rs.k.min() >= 1 and rs.k.max() <= 6
    for i in (0, 17, 299):
        assert rs.trial_y(i).shape == (rs.n_snap[i], rs.n_elem[i])
    assert rs.pool.size == int(np.sum(rs.n_elem.astype(np.int64) * rs.n_snap))

"""Pins for the coherent multi-array oracle: mirror geometry against an
independent plane construction, the reflected path length through the
reflection point, array-response structure and closed forms, and the cost of
a noise-free single path."""
import cmath
import math

import numpy as np

from oracle import coherent as oc

FC = 3.5e9
LAM = oc.C_LIGHT / FC


def plane_of(s):
    """The surface whose mirror image of the origin is s: unit normal n, offset c (n.x = c)."""
    n = s / np.linalg.norm(s)
    return n, np.linalg.norm(s) / 2.0


def mirror(x, s):
    n, c = plane_of(s)
    return x - 2.0 * (n @ x - c) * n


def rot_z(a):
    return np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0], [0.0, 0.0, 1.0]])


def test_sfv_is_the_mirror_of_the_origin_and_the_anchor_the_mirror_of_the_array():
    rng = np.random.default_rng(0)
    for _ in range(20):
        s = rng.uniform(-10, 10, 3)
        p = rng.uniform(-4, 4, 3)
        np.testing.assert_allclose(mirror(np.zeros(3), s), s, atol=1e-12)
        np.testing.assert_allclose(oc.virtual_anchor(p, s), mirror(p, s), atol=1e-12)


def test_householder_properties():
    s = np.array([1.0, -2.0, 0.5])
    H = oc.householder(s)
    np.testing.assert_allclose(H @ H.T, np.eye(3), atol=1e-15)
    np.testing.assert_allclose(H @ s, -s, atol=1e-15)
    x = np.cross(s, [0.3, 0.1, 0.7])
    np.testing.assert_allclose(H @ x, x, atol=1e-15)
    assert abs(np.linalg.det(H) + 1.0) < 1e-14


def test_local_vector_points_at_the_virtual_mobile():
    rng = np.random.default_rng(1)
    for _ in range(20):
        s = rng.uniform(-10, 10, 3)
        p_pa, p_mt = rng.uniform(-4, 4, 3), rng.uniform(-4, 4, 3)
        rot = rot_z(rng.uniform(0, 2 * math.pi))
        r = oc.local_vector(p_mt, s, p_pa, rot)
        np.testing.assert_allclose(rot @ r, mirror(p_mt, s) - p_pa, atol=1e-12)
    r = oc.local_vector(np.array([1.0, 2.0, 3.0]), None, np.array([0.5, 0.0, 0.0]), rot_z(0.3))
    np.testing.assert_allclose(rot_z(0.3) @ r, [0.5, 2.0, 3.0], atol=1e-15)


def test_reflected_path_length_through_the_reflection_point():
    # array and terminal on the same side of a wall x = 5 (SFV at (10, 0, 0))
    s = np.array([10.0, 0.0, 0.0])
    p_pa, p_mt = np.array([1.0, 2.0, 1.0]), np.array([3.0, -1.0, 2.0])
    n, c = plane_of(s)
    vm = mirror(p_mt, s)
    t = (c - n @ p_pa) / (n @ (vm - p_pa))          # where the segment array -> virtual mobile crosses the wall
    q = p_pa + t * (vm - p_pa)
    assert abs(n @ q - c) < 1e-12 and 0 < t < 1
    d = np.linalg.norm(oc.local_vector(p_mt, s, p_pa, np.eye(3)))
    assert abs(d - (np.linalg.norm(p_mt - q) + np.linalg.norm(q - p_pa))) < 1e-12


def test_array_response_structure_and_closed_forms():
    f = oc.frequencies(10, 100e6)
    assert np.allclose(f, -f[::-1])
    py, pz = oc.ura_support(4, LAM), oc.ura_support(4, LAM)
    r = np.array([3.0, 1.2, -0.7])
    d = np.linalg.norm(r)
    psi = oc.array_response(r, f, py, pz, FC)
    assert psi.shape == (160,)
    np.testing.assert_allclose(np.abs(psi), LAM / (4 * math.pi * d), rtol=1e-13)
    # Kronecker order: frequency slowest, then y, then z
    P = psi.reshape(10, 4, 4)
    np.testing.assert_allclose(P[1] / P[0], np.exp(-2j * math.pi * (f[1] - f[0]) * d / oc.C_LIGHT), rtol=1e-12)
    # horizontal response: direction cosine u = r_y / d, element phase pi (i - 1.5) u
    u = r[1] / d
    np.testing.assert_allclose(P[0, 1, 0] / P[0, 0, 0], cmath.exp(1j * math.pi * u), rtol=1e-12)
    w = r[2] / d
    np.testing.assert_allclose(P[0, 0, 1] / P[0, 0, 0], cmath.exp(1j * math.pi * w), rtol=1e-12)
    # broadside, zero delay offset at the centre frequency: carrier phase only
    psi_b = oc.array_response(np.array([2.0, 0.0, 0.0]), np.zeros(1), np.zeros(1), np.zeros(1), FC,
                              unit_modulus=True)
    np.testing.assert_allclose(psi_b, [cmath.exp(-2j * math.pi * 2.0 / LAM)], rtol=1e-12)


def test_hand_single_element():
    # J = 1, N_f = 1, one antenna: psi = lambda / (4 pi d) exp(-j 2 pi d / lambda); cost = |conj(z) psi|^2
    d = 2.5
    z = np.array([[0.3 - 0.4j]])
    psi = oc.steering(np.array([d, 0.0, 0.0]), None, [np.zeros(3)], [np.eye(3)], np.zeros(1), np.zeros(1),
                      np.zeros(1), FC)
    want = abs(np.conj(z[0, 0]) * LAM / (4 * math.pi * d) * cmath.exp(-2j * math.pi * d / LAM)) ** 2
    assert abs(oc.coherent_cost(z, psi) - want) < 1e-18


def test_noise_free_path_cost():
    rng = np.random.default_rng(2)
    pas = [np.array([0.0, 0.0, 1.0]), np.array([6.0, 0.0, 1.0]), np.array([6.0, 5.0, 1.0]), np.array([0.0, 5.0, 1.0])]
    rots = [rot_z(a) for a in (0.25 * math.pi, 0.75 * math.pi, -0.75 * math.pi, -0.25 * math.pi)]
    f, py, pz = oc.frequencies(10, 100e6), oc.ura_support(4, LAM), oc.ura_support(4, LAM)
    p_mt = np.array([2.0, 2.5, 1.2])
    s_true = np.array([14.0, 0.0, 0.0])
    rho = 0.8 + 0.6j
    Psi = oc.steering(p_mt, s_true, pas, rots, f, py, pz, FC)
    Z = rho * Psi
    want = abs(rho) ** 2 * (np.sum(np.abs(Psi) ** 2) / 160) ** 2
    assert abs(oc.coherent_cost(Z, Psi) - want) < 1e-12 * want
    # a candidate elsewhere scores lower than the true one here
    other = oc.coherent_cost(Z, oc.steering(p_mt, s_true + np.array([0.3, 0.2, 0.0]), pas, rots, f, py, pz, FC))
    assert other < want

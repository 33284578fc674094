"""Pins of the oracle's pure shear, Eq. (17): F = [[1, a], [b, 1]] on (x, y)
(CPU only).  The box sequence H_k = F^k diag(L) and the map of the positions
are checked against what the mathematics fixes: the simple-shear limit
b = 0, repeated products, the eigen-decomposition (eigenvalues 1 +- sqrt(ab)),
the determinant (1 - ab)^k, unchanged fractional coordinates, the explicit
image sum in the deformed box, and the stress as the energy's derivative
along the pure-shear path."""
import math

import numpy as np
import pytest

import oracle as O
from gpu_common import load_glass

POT = O.kob_andersen()


def naive_power(a, b, k):
    F = np.array([[1.0, a], [b, 1.0]])
    R = np.eye(2)
    for _ in range(k):
        R = R @ F
    return R


def test_power_reduces_to_simple_shear():
    a = 1e-4
    for k in (0, 1, 2, 3, 17, 200, 1000):
        M = np.array(O.deformation_power(a, 0.0, k))
        assert M[0, 0] == 1.0 and M[1, 1] == 1.0 and M[1, 0] == 0.0
        assert M[0, 1] == pytest.approx(k * a, rel=1e-13, abs=0.0)
    # and the box of a pure shear with b = 0 is the simple-shear box bit for bit
    assert np.array_equal(O.strain_box(2, 10.0, 37, a, 0.0), O.strain_box(2, 10.0, 37, a))


@pytest.mark.parametrize("a,b", [(1e-3, 2e-3), (5e-3, -3e-3), (-2e-3, 1e-3)])
def test_power_matches_repeated_products(a, b):
    for k in (1, 2, 7, 64, 200):
        np.testing.assert_allclose(np.array(O.deformation_power(a, b, k)), naive_power(a, b, k),
                                   rtol=1e-13, atol=1e-15)


def test_power_closed_form():
    # ab > 0: F = V diag(1 + s, 1 - s) V^-1, s = sqrt(ab), V = [[sqrt a, sqrt a], [sqrt b, -sqrt b]]
    a, b, k = 4e-3, 1e-3, 200
    s = math.sqrt(a * b)
    V = np.array([[math.sqrt(a), math.sqrt(a)], [math.sqrt(b), -math.sqrt(b)]])
    want = V @ np.diag([(1 + s) ** k, (1 - s) ** k]) @ np.linalg.inv(V)
    np.testing.assert_allclose(np.array(O.deformation_power(a, b, k)), want, rtol=1e-12)
    # the transposed map has the transposed power (a and b enter asymmetrically)
    np.testing.assert_allclose(np.array(O.deformation_power(b, a, k)), want.T, rtol=1e-12)


@pytest.mark.parametrize("a,b", [(1e-3, 2e-3), (5e-3, -3e-3)])
def test_power_determinant(a, b):
    for k in (1, 10, 300):
        M = np.array(O.deformation_power(a, b, k))
        assert np.linalg.det(M) == pytest.approx((1.0 - a * b) ** k, rel=1e-12)


def test_negative_index_refused():
    with pytest.raises(ValueError):
        O.deformation_power(1e-3, 1e-3, -1)


def test_map_keeps_fractional_coordinates_and_composes():
    pos, types, L, dim = load_glass("glass2d_256")
    a, b = 2e-3, -1e-3
    H0 = O.strain_box(dim, L, 0, a, b)
    assert np.array_equal(H0, np.diag([L, L]))
    for k in (1, 5, 40):
        rk = O.affine(pos, a, b, steps=k)
        Hk = O.strain_box(dim, L, k, a, b)
        s0 = np.linalg.solve(H0, pos.T).T
        sk = np.linalg.solve(Hk, rk.T).T
        np.testing.assert_allclose(sk, s0, atol=1e-12)
    np.testing.assert_allclose(O.affine(O.affine(pos, a, b, steps=3), a, b, steps=5),
                               O.affine(pos, a, b, steps=8), atol=1e-12)
    # one increment is exactly x + a y, b x + y
    r1 = O.affine(pos, a, b)
    assert np.array_equal(r1[:, 0], pos[:, 0] + a * pos[:, 1])
    assert np.array_equal(r1[:, 1], b * pos[:, 0] + pos[:, 1])


@pytest.mark.parametrize("dim,name", [(2, "glass2d_256"), (3, "glass3d_1500")])
def test_minimum_image_equals_image_sum_in_a_pure_sheared_box(dim, name):
    pos, types, L, d = load_glass(name)
    a, b = 3e-3, 2e-3
    k = 60
    r = O.affine(pos, a, b, steps=k)
    H = O.strain_box(d, L, k, a, b)
    assert H[1, 0] != 0.0
    E0, F0, S0, _ = O.energy_forces(r, types, H, POT)
    E1, F1, S1, _ = O.energy_forces(r, types, H, POT, image_sum=True, image_range=2)
    assert E0 == pytest.approx(E1, rel=1e-12)
    np.testing.assert_allclose(F0, F1, atol=1e-10)
    np.testing.assert_allclose(S0, S1, atol=1e-12)
    # and the energy is that of the undeformed lattice of images: wrapping
    # every atom by a box vector changes nothing
    shift = H @ np.array([1.0, -1.0] + ([0.0] if d == 3 else []))
    E2 = O.energy_forces(r + shift, types, H, POT)[0]
    assert E2 == pytest.approx(E0, rel=1e-12)


def test_stress_is_the_energy_derivative_along_the_pure_shear():
    # dE/de of r(e) = F(e) r, H(e) = F(e) diag(L), F(e) = [[1, e a], [e b, 1]]:
    # V (a sigma_xy + b sigma_yx) at e = 0
    pos, types, L, dim = load_glass("glass2d_256")
    a, b = 1.0, 0.6
    H0 = np.diag([L, L])
    E0, F0, S0, _ = O.energy_forces(pos, types, H0, POT)

    def energy(e):
        M = np.array([[1.0, e * a], [e * b, 1.0]])
        return O.energy_forces(pos @ M.T, types, M @ H0, POT)[0]

    h = 1e-6
    dE = (energy(h) - energy(-h)) / (2 * h)
    V = L * L
    assert dE == pytest.approx(V * (a * S0[0, 1] + b * S0[1, 0]), rel=1e-6)


def test_one_pure_shear_step_minimises_to_an_inherent_structure():
    pos, types, L, dim = load_glass("glass2d_256")
    a, b = 1e-3, 5e-4
    H1 = O.strain_box(dim, L, 1, a, b)
    res = O.fire(O.affine(pos, a, b), types, H1, POT)
    assert res.status == 0
    assert O.max_force(res.pos, types, H1, POT) < 1e-10
    assert res.E <= O.energy_forces(O.affine(pos, a, b), types, H1, POT)[0]

"""Pins of the oracle's pair potential, energies, forces, stress and images
against closed forms, lattice sums by shell enumeration, finite differences
and the explicit image sum (CPU only)."""
import math
import os

import numpy as np
import pytest

import aqs_synth as S
import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, *v = line.split()
        out[k] = v
    return out


POT = O.kob_andersen()


def test_dimer_closed_forms():
    g = golden("lj_closed_forms.txt")
    rstar = float(g["r_star_over_sigma"][0])
    assert abs(rstar - 2 ** (1 / 6)) < 1e-15
    for (a, b) in [(0, 0), (0, 1), (1, 1)]:
        sig, eps = POT.sigma[a][b], POT.eps[a][b]
        u, gr, inside = O.pair(POT, a, b, rstar * sig)
        assert inside
        assert abs(gr) < 1e-13 * eps / sig ** 2
        assert u == pytest.approx(float(g["u_min_over_eps"][0]) * eps, rel=1e-12)
        # curvature by central differences of U'(r) = r g(r)
        h = 1e-5 * sig
        up = O.pair(POT, a, b, rstar * sig + h)[1] * (rstar * sig + h)
        um = O.pair(POT, a, b, rstar * sig - h)[1] * (rstar * sig - h)
        k = (up - um) / (2 * h)
        assert k == pytest.approx(float(g["k_min_sigma2_over_eps"][0]) * eps / sig ** 2, rel=1e-7)


def test_cutoff_shift_and_continuity():
    for (a, b) in [(0, 0), (0, 1), (1, 1)]:
        rc = 2.5 * POT.sigma[a][b]
        u_in, _, inside = O.pair(POT, a, b, rc * (1 - 1e-12))
        assert inside and abs(u_in) < 1e-12
        u_out, g_out, inside = O.pair(POT, a, b, rc)
        assert not inside and u_out == 0.0 and g_out == 0.0


def test_pair_derivative_matches_energy_differences():
    for r in [0.8, 0.95, 1.1, 1.5, 2.2]:
        u0, g, _ = O.pair(POT, 0, 1, r)
        h = 1e-6
        du = (O.pair(POT, 0, 1, r + h)[0] - O.pair(POT, 0, 1, r - h)[0]) / (2 * h)
        assert g * r == pytest.approx(du, rel=1e-7, abs=1e-9)


def test_paper_binary_parameters():
    g = golden("paper_values.txt")
    p = O.paper_binary()
    assert p.sigma[0][0] == pytest.approx(2 * math.sin(math.pi / 10))
    assert p.sigma[1][1] == pytest.approx(2 * math.sin(math.pi / 5))
    assert p.sigma[0][1] == pytest.approx(float(g["sigma_SL"][0]))
    assert p.eps[0][0] == float(g["eps_SS"][0]) and p.eps[1][1] == float(g["eps_LL"][0])
    assert p.eps[0][1] == float(g["eps_SL"][0])


# --- lattice sums by shell enumeration (independent of the pair loop) -------

def tri_lattice(nx, ny, a):
    pos = [((i + 0.5 * (j % 2)) * a, j * a * math.sqrt(3) / 2) for j in range(ny) for i in range(nx)]
    return np.array(pos), nx * a, ny * a * math.sqrt(3) / 2


def tri_shell_energy(a, rc=2.5):
    """E/N = 1/2 sum over lattice vectors R != 0 with |R| < rc of U(|R|)."""
    e = 0.0
    m = int(rc / a) + 3
    uc = 4 * (2.5 ** -12 - 2.5 ** -6)
    for i in range(-m, m + 1):
        for j in range(-m, m + 1):
            if i == 0 and j == 0:
                continue
            x = i * a + j * a / 2
            y = j * a * math.sqrt(3) / 2
            r = math.hypot(x, y)
            if r < rc:
                e += 0.5 * (4 * (r ** -12 - r ** -6) - uc)
    return e


def fcc_lattice(m, a):
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    cells = np.stack(np.meshgrid(range(m), range(m), range(m), indexing="ij"), -1).reshape(-1, 3)
    return ((cells[:, None, :] + basis[None]) * a).reshape(-1, 3), m * a


def fcc_shell_energy(a, rc=2.5):
    prim = np.array([[0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]]) * a
    m = int(2 * rc / a) + 3
    e = 0.0
    uc = 4 * (2.5 ** -12 - 2.5 ** -6)
    rng = range(-m, m + 1)
    for i in rng:
        for j in rng:
            for k in rng:
                if i == j == k == 0:
                    continue
                R = i * prim[0] + j * prim[1] + k * prim[2]
                r = float(np.sqrt(R @ R))
                if r < rc:
                    e += 0.5 * (4 * (r ** -12 - r ** -6) - uc)
    return e


@pytest.mark.parametrize("a", [1.05, 1.12, 1.2])
def test_triangular_lattice_energy_forces_pressure(a):
    pos, Lx, Ly = tri_lattice(8, 10, a)
    n = len(pos)
    types = np.zeros(n, dtype=np.uint8)
    H = O.box_matrix(2, [Lx, Ly], 0.0)
    E, F, Sg, _ = O.energy_forces(pos, types, H, POT)
    assert E / n == pytest.approx(tri_shell_energy(a), rel=1e-12, abs=1e-13)
    assert np.abs(F).max() < 1e-11
    # virial trace: (sigma_xx + sigma_yy) V = a dE/da (every pair scales with a)
    h = 1e-6
    dEda = n * (tri_shell_energy(a + h) - tri_shell_energy(a - h)) / (2 * h)
    assert (Sg[0, 0] + Sg[1, 1]) * Lx * Ly == pytest.approx(a * dEda, rel=1e-6, abs=1e-8)
    assert abs(Sg[0, 1] - Sg[1, 0]) < 1e-12


@pytest.mark.parametrize("a", [1.45, 1.55])
def test_fcc_lattice_energy(a):
    pos, L = fcc_lattice(4, a)
    n = len(pos)
    types = np.zeros(n, dtype=np.uint8)
    H = O.box_matrix(3, L, 0.0)
    E, F, Sg, _ = O.energy_forces(pos, types, H, POT)
    assert E / n == pytest.approx(fcc_shell_energy(a), rel=1e-12)
    assert np.abs(F).max() < 1e-11
    h = 1e-6
    dEda = n * (fcc_shell_energy(a + h) - fcc_shell_energy(a - h)) / (2 * h)
    assert np.trace(Sg) * L ** 3 == pytest.approx(a * dEda, rel=1e-6)


# --- forces, stress, images on disordered configurations --------------------

def jittered(dim, m, seed, gamma):
    s = S.jittered_lattice_start(dim, m, 77, seed, jitter=0.15)
    H = O.box_matrix(dim, s.L, gamma)
    pos = s.pos.copy()
    pos[:, 0] += gamma * pos[:, 1]
    return pos, s.types, H


@pytest.mark.parametrize("dim,m,gamma", [(2, 7, 0.0), (2, 7, 0.3), (3, 6, -0.2)])
def test_forces_match_finite_differences(dim, m, gamma):
    pos, types, H = jittered(dim, m, 1, gamma)
    E, F, _, _ = O.energy_forces(pos, types, H, POT)
    rng = np.random.default_rng(3)
    h = 1e-6
    for i in rng.choice(len(pos), 6, replace=False):
        for a in range(dim):
            p = pos.copy()
            p[i, a] += h
            ep = O.energy_forces(p, types, H, POT)[0]
            p[i, a] -= 2 * h
            em = O.energy_forces(p, types, H, POT)[0]
            fd = -(ep - em) / (2 * h)
            assert F[i, a] == pytest.approx(fd, rel=1e-5, abs=1e-7)


@pytest.mark.parametrize("dim,m,gamma", [(2, 8, 0.1), (3, 6, 0.25)])
def test_net_force_vanishes(dim, m, gamma):
    pos, types, H = jittered(dim, m, 2, gamma)
    _, F, _, _ = O.energy_forces(pos, types, H, POT)
    scale = np.abs(F).sum()
    assert np.abs(F.sum(axis=0)).max() < 1e-13 * scale * 10


@pytest.mark.parametrize("dim,m,gamma", [(2, 8, 0.0), (2, 8, 0.1), (3, 6, 0.05)])
def test_shear_stress_is_energy_derivative(dim, m, gamma):
    """sigma_xy V = dE/dgamma under the affine map of positions and box
    (Lagrangian energy, Eq. 5)."""
    pos, types, H = jittered(dim, m, 4, gamma)
    _, _, Sg, _ = O.energy_forces(pos, types, H, POT)
    L = H[1, 1]
    vol = abs(np.linalg.det(H))
    h = 1e-6
    ep = O.energy_forces(O.affine(pos, h), types, O.box_matrix(dim, np.diag(H), gamma + h), POT)[0]
    em = O.energy_forces(O.affine(pos, -h), types, O.box_matrix(dim, np.diag(H), gamma - h), POT)[0]
    assert Sg[0, 1] * vol == pytest.approx((ep - em) / (2 * h), rel=1e-6, abs=1e-8)
    del L


@pytest.mark.parametrize("dim,m,gamma", [(2, 7, -0.45), (2, 7, 0.33), (3, 6, 0.45)])
def test_minimum_image_equals_explicit_image_sum(dim, m, gamma):
    pos, types, H = jittered(dim, m, 5, gamma)
    E0, F0, S0, _ = O.energy_forces(pos, types, H, POT)
    E1, F1, S1, _ = O.energy_forces(pos, types, H, POT, image_sum=True, image_range=2)
    assert E0 == pytest.approx(E1, rel=1e-12)
    assert np.allclose(F0, F1, rtol=1e-10, atol=1e-10)
    assert np.allclose(S0, S1, rtol=1e-10, atol=1e-12)


def test_energy_invariant_under_full_period_shear():
    """Shearing the box by a full period (gamma -> gamma + 1 with Lx = Ly)
    maps the lattice onto itself: the energy of unchanged positions is the
    same (explicit image sum, valid for any tilt)."""
    pos, types, H = jittered(2, 7, 6, 0.2)
    L = H[0, 0]
    E0 = O.energy_forces(pos, types, O.box_matrix(2, L, 0.2), POT, image_sum=True, image_range=3)[0]
    E1 = O.energy_forces(pos, types, O.box_matrix(2, L, 1.2), POT, image_sum=True, image_range=3)[0]
    assert E0 == pytest.approx(E1, rel=1e-12)


def test_affine_composition():
    """F(a) F(b) = F(a + b) for simple shear (Eq. 16)."""
    pos, _, _ = jittered(2, 7, 7, 0.0)
    x1 = O.affine(O.affine(pos, 0.013), 0.021)
    x2 = O.affine(pos, 0.034)
    assert np.allclose(x1, x2, rtol=0, atol=4 * np.finfo(float).eps * np.abs(pos).max())
    assert np.array_equal(x1[:, 1], pos[:, 1])


def test_forces_on_subset_match_full():
    pos, types, H = jittered(3, 6, 8, 0.1)
    _, F, _, _ = O.energy_forces(pos, types, H, POT)
    idx = np.array([0, 7, 42, 124])
    assert np.array_equal(O.forces_on(pos, types, H, POT, idx), F[idx])


def test_min_image_guard():
    pos, types, _ = jittered(2, 4, 9, 0.0)
    H = O.box_matrix(2, 4.0, 0.0)   # too small for rc = 2.5
    assert not O.min_image_valid(H, POT)
    with pytest.raises(ValueError):
        O.energy_forces(pos, types, H, POT)

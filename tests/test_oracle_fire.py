"""Pins of the oracle's minimiser (Eq. 10 realised by FIRE 2.0) and of the
configuration distance of the equality test (Eq. 20), CPU only."""
import math

import numpy as np
import pytest

import aqs_synth as S
import oracle as O

POT = O.kob_andersen()
TUNED = O.FireParams(dt0=0.005, dt_max=0.03, f_dec=0.9, alpha0=0.2, f_alpha=0.95, n_delay=5, f_inc=1.2)


@pytest.fixture(scope="module")
def glass():
    s = S.uniform_glass_start(2, 256, 1, 0)
    H = O.box_matrix(2, s.L, 0.0)
    r = O.fire(s.pos, s.types, H, POT, TUNED)
    assert r.status == O.CONVERGED
    return r.pos, s.types, s.L


@pytest.mark.parametrize("params", [O.FireParams(), TUNED])
@pytest.mark.parametrize("r0", [1.3, 1.0, 2.0])
def test_dimer_reaches_the_analytic_minimum(params, r0):
    L = 12.0
    pos = np.array([[3.0, 4.0], [3.0 + r0, 4.0]])
    types = np.zeros(2, dtype=np.uint8)
    r = O.fire(pos, types, O.box_matrix(2, L, 0.0), POT, params)
    assert r.status == O.CONVERGED
    d = np.linalg.norm(r.pos[1] - r.pos[0])
    assert abs(d - 2 ** (1 / 6)) < 1e-11
    assert r.E == pytest.approx(-0.983683108864, abs=1e-12)
    # the centre of mass does not move (equal and opposite forces, FIRE mixing)
    assert np.allclose(r.pos.mean(axis=0), pos.mean(axis=0), atol=1e-13)


def test_inherent_structure_takes_zero_iterations(glass):
    """F(r_star) = r_star for the i = 0 anchor (Sec. 3.2): the convergence
    test comes before any update."""
    pos, types, L = glass
    r = O.fire(pos, types, O.box_matrix(2, L, 0.0), POT, TUNED)
    assert r.iters == 0 and r.status == O.CONVERGED
    assert np.array_equal(r.pos, pos)


def test_perfect_lattice_takes_zero_iterations():
    """A perfect lattice has zero force on every atom by inversion symmetry."""
    a = 1.08
    nx, ny = 8, 10
    pos = np.array([((i + 0.5 * (j % 2)) * a, j * a * math.sqrt(3) / 2) for j in range(ny) for i in range(nx)])
    H = O.box_matrix(2, [nx * a, ny * a * math.sqrt(3) / 2], 0.0)
    r = O.fire(pos, np.zeros(len(pos), np.uint8), H, POT, TUNED)
    assert r.iters == 0 and r.status == O.CONVERGED


def test_aqs_step_descends_and_is_certified(glass):
    pos, types, L = glass
    dg = 1e-3
    H = O.strain_box(2, L, 1, dg)
    x = O.affine(pos, dg)
    E0 = O.energy_forces(x, types, H, POT)[0]
    r = O.fire(x, types, H, POT, TUNED, trace_cap=100000)
    assert r.status == O.CONVERGED and r.iters > 0
    assert r.E < E0
    assert r.trace[0] == pytest.approx(E0, rel=1e-15)
    assert r.E <= r.trace.min() + 1e-12 * abs(r.E)
    # independent evaluation of the end state
    E1, F, _, _ = O.energy_forces(r.pos, types, H, POT)
    assert E1 == r.E
    assert np.sqrt((F * F).sum(1)).max() == r.fmax < 1e-10


def test_maxiter_status_and_determinism(glass):
    pos, types, L = glass
    H = O.strain_box(2, L, 1, 1e-2)
    x = O.affine(pos, 1e-2)
    p = O.FireParams(**{**TUNED.__dict__, "max_iter": 9})
    a = O.fire(x, types, H, POT, p)
    b = O.fire(x, types, H, POT, p)
    assert a.status == O.MAXITER and a.iters == 9
    assert np.array_equal(a.pos, b.pos)


def test_nonfinite_input_is_reported():
    pos = np.array([[1.0, 1.0], [np.nan, 2.0], [5.0, 5.0]])
    r = O.fire(pos, np.zeros(3, np.uint8), O.box_matrix(2, 12.0, 0.0), POT, TUNED)
    assert r.status == O.NONFINITE


def test_distance_of_the_equality_test(glass):
    pos, types, L = glass
    H = O.strain_box(2, L, 3, 1e-3)
    assert O.compare(pos, pos, H)[0] == 0.0
    # an atom moved by a lattice vector is the same configuration
    q = pos.copy()
    q[5] += H[:, 1]
    q[9] -= H[:, 0]
    assert O.compare(pos, q, H)[0] < 1e-12
    # a rigid translation t gives max = |t| and mean = t
    t = np.array([0.003, -0.004])
    d, mean = O.compare(pos + t, pos, H)
    assert d == pytest.approx(0.005, rel=1e-9)
    assert np.allclose(mean, t, atol=1e-12)


def test_perturbed_inherent_structure_relaxes_back(glass):
    """An IS perturbed by 1e-4 sigma noise (mean removed) and re-minimised is
    equal (same basin, Eq. 20).  A 1e-3 sigma kick lands this small glass in
    a distinct nearby minimum (higher energy, max displacement 3.5e-4 sigma,
    above the threshold 1e-4): the test tells them apart.  A different glass
    is not equal."""
    pos, types, L = glass
    H = O.box_matrix(2, L, 0.0)
    E0 = O.energy_forces(pos, types, H, POT)[0]
    for amp, same in [(1e-4, True), (1e-3, False)]:
        rng = S.rng_for(42)
        noise = rng.uniform(-amp, amp, pos.shape)
        noise -= noise.mean(axis=0)
        r = O.fire(pos + noise, types, H, POT, TUNED)
        assert r.status == O.CONVERGED
        d, mean = O.compare(r.pos, pos, H)
        assert np.abs(mean).max() < 1e-13
        assert O.equal_configs(r.pos, pos, H) == same
        if same:
            assert d < 1e-9
        else:
            assert 1e-4 < d < 1e-3 and r.E > E0 + 1e-7
    other = S.uniform_glass_start(2, 256, 1, 1)
    assert not O.equal_configs(other.pos, pos, H)

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


# Curvature of the shifted pair energy at its minimum (closed form, also in
# tests/golden/lj_closed_forms.txt): U''(r*) = 36 * 2^(2/3) for eps = sigma = 1.
K_DIMER = 36.0 * 2.0 ** (2.0 / 3.0)


@pytest.mark.parametrize("n_neg_max", [0, 1, 5, 40])
def test_stalled_after_n_neg_max_overshooting_steps(n_neg_max):
    """STALLED counts consecutive evaluations with P = F.v <= 0.  A dimer near
    its minimum is a harmonic oscillator of the bond u = r - r* with
    u'' = -2 k u.  With a constant time step (f_inc = f_dec = 1) and
    c = 2 k dt^2 in (1, 4/3), every step overshoots: after the restart of
    step 5 the bond follows u_(n+1) = (1 - c) u_n + (c / 2) u_(n-1) (u_(-1) = 0:
    the first step starts from rest), whose dominant root is negative with
    modulus below one, so u changes sign at every step, P < 0 at every
    evaluation after the first (where v = 0, P = 0), and the amplitude decays
    too slowly to converge before the stall.  Hence n_neg = it + 1 at
    evaluation it, and the minimiser stops at evaluation it = n_neg_max with
    STALLED, before that evaluation's update."""
    c = 1.15
    dt = math.sqrt(c / (2.0 * K_DIMER))
    rstar = 2.0 ** (1.0 / 6.0)
    u0 = 1e-3
    pos = np.array([[3.0, 4.0], [3.0 + rstar + u0, 4.0]])
    types = np.zeros(2, dtype=np.uint8)
    p = O.FireParams(dt0=dt, dt_max=dt, dt_min=1e-6, f_inc=1.0, f_dec=1.0, alpha0=0.1, f_alpha=0.99,
                     dmax=1.0, n_delay=5, n_neg_max=n_neg_max)
    r = O.fire(pos, types, O.box_matrix(2, 12.0, 0.0), POT, p)
    assert r.status == O.STALLED and r.iters == n_neg_max
    # the bond alternates in sign and decays with the predicted root
    lam = ((1 - c) - math.sqrt(1 + c * c)) / 2
    assert -1.0 < lam < 0.0
    # the same run with max_iter = n_neg_max stops at the same positions
    # (the stall exits before moving)
    if n_neg_max > 0:
        q = O.fire(pos, types, O.box_matrix(2, 12.0, 0.0), POT,
                   O.FireParams(**{**p.__dict__, "n_neg_max": 10 ** 6, "max_iter": n_neg_max}))
        assert q.status == O.MAXITER and np.array_equal(q.pos, r.pos)
    else:
        assert np.array_equal(r.pos, pos)
    # with a step inside the stable range (c < 1) the same start converges
    ok = O.fire(pos, types, O.box_matrix(2, 12.0, 0.0), POT,
                O.FireParams(**{**p.__dict__, "dt0": 0.5 * dt, "dt_max": 0.5 * dt, "n_neg_max": 2000}))
    assert ok.status == O.CONVERGED


def test_consecutive_count_resets_after_positive_power(glass):
    """Relaxing a glass from a small perturbation of its inherent structure
    has short runs of P <= 0 and many of them.  A bound of 1 stalls at the
    first run of two (iteration i1), a bound of 2 at the first run of three
    (i2 > i1 + 1, so a different run).  Counting the first evaluation (v = 0,
    P = 0), at least 1 + 2 + 3 = 6 evaluations had P <= 0 by i2, so a
    count that was not reset at P > 0 would pass a bound of 5 there; with
    the reset, a bound of 5 changes nothing."""
    pos, types, L = glass
    H = O.box_matrix(2, L, 0.0)
    x = pos + S.rng_for(2507, 20802, 91).normal(0.0, 0.02, size=pos.shape)
    ref = O.fire(x, types, H, POT, TUNED)
    run = {m: O.fire(x, types, H, POT, O.FireParams(**{**TUNED.__dict__, "n_neg_max": m})) for m in (1, 2, 5)}
    assert ref.status == O.CONVERGED
    assert run[1].status == O.STALLED and run[2].status == O.STALLED
    i1, i2 = run[1].iters, run[2].iters
    assert i2 > i1 + 1 and i2 < ref.iters
    assert run[5].status == O.CONVERGED
    assert run[5].iters == ref.iters and np.array_equal(run[5].pos, ref.pos)

"""Pins of the oracle's conjugate-gradient minimiser (Eq. 10 by the paper's
own method, Sec. 2.1: Polak-Ribiere+ with a line search on the directional
derivative), CPU only.

On a quadratic the directional derivative is linear in the step, so every
secant step of the line search lands exactly on the minimum along the line,
and conjugate gradients with exact line searches end after as many search
directions as the Hessian has distinct eigenvalues.  Those two facts pin the
line search (extrapolation, interpolation) and the direction update (beta).
On the Lennard-Jones system: the dimer minimum at 2^(1/6) sigma, zero
iterations at an inherent structure and at a perfect lattice, descent,
certification by the independent force evaluation, the displacement cap,
and the same inherent structure as FIRE (Eq. 20) -- two independent
minimisers agreeing."""
import math

import numpy as np
import pytest

import aqs_synth as S
import oracle as O

POT = O.kob_andersen()
FIRE = O.FireParams(dt0=0.005, dt_max=0.03, f_dec=0.9, alpha0=0.2, f_alpha=0.95, n_delay=5, f_inc=1.2)
# no displacement cap; sigma so small that a search ends only at the exact
# minimum along the line (to rounding), as finite termination requires
EXACT = O.CgParams(dmax=1e9, sigma=1e-9)


def _quadratic(m: int, n: int = 60, seed: int = 0):
    rng = np.random.default_rng(seed)
    vals = np.geomspace(1.0, 30.0, m)
    kk = vals[rng.permutation(np.arange(n) % m)]
    return rng.normal(size=(n, 1)), kk[:, None]


@pytest.mark.parametrize("m", [1, 2, 3, 5])
@pytest.mark.parametrize("seed", [0, 1])
def test_quadratic_ends_after_one_direction_per_distinct_stiffness(m, seed):
    x0, kk = _quadratic(m, seed=seed)
    r = O.cg_quadratic(x0, kk, EXACT)
    assert r.status == O.CONVERGED
    assert r.dirs == m
    # a search takes at most three evaluations, plus up to three extrapolations
    # of the first one from a_init = 0.01 towards steps of order 1 / k
    assert r.iters <= 3 * m + 3
    assert np.abs(kk * r.pos).max() < EXACT.ftol


@pytest.mark.parametrize("a_init,iters", [
    (0.05, 2),    # short first trial: the secant extrapolation from (0, p0) lands on 1/k
    (0.15, 2),    # first trial past the minimum: the secant root of the bracket is 1/k
    (0.01, 3),    # 1/k = 10 a_init: clamped to grow a_init, then the secant lands on 1/k
])
def test_line_search_is_exact_on_one_stiffness(a_init, iters):
    """E = k |x|^2 / 2 with k = 10: the minimum along d = F is at a = 1/k."""
    x0 = np.random.default_rng(3).normal(size=(20, 2))
    kk = np.full_like(x0, 10.0)
    r = O.cg_quadratic(x0, kk, O.CgParams(dmax=1e9, a_init=a_init, grow=4.0))
    assert r.status == O.CONVERGED and r.dirs == 1 and r.iters == iters
    assert np.abs(r.pos).max() < 1e-14


def test_second_direction_is_polak_ribiere():
    """With a loose line search (sigma = 0.9) the first trial x1 = x0 + a F0
    is accepted while F1.F0 != 0, so Polak-Ribiere and Fletcher-Reeves
    differ.  On E = sum k x^2 / 2 everything is known in closed form
    (F = -k x): the second update must be x2 = x1 + a1 d2 with the textbook
    d2 = F1 + beta F0, beta = (|F1|^2 - F1.F0) / |F0|^2 (Polak and Ribiere,
    1969), and a1 = a (F0.F0) / (F1.d2)."""
    rng = np.random.default_rng(7)
    x0 = rng.normal(size=(30, 1))
    kk = rng.uniform(1.0, 10.0, size=(30, 1))
    a = 0.05
    r = O.cg_quadratic(x0, kk, O.CgParams(dmax=1e9, sigma=0.9, a_init=a, max_iter=2))
    assert r.status == O.MAXITER and r.iters == 2 and r.dirs == 2
    F0 = -kk * x0
    x1 = x0 + a * F0
    F1 = -kk * x1
    f00, f10, f11 = (F0 * F0).sum(), (F1 * F0).sum(), (F1 * F1).sum()
    assert abs(f10) <= 0.9 * f00 and abs(f10) > 0.1 * f00   # accepted, and PR != FR
    beta = max(0.0, (f11 - f10) / f00)
    d2 = F1 + beta * F0
    x2 = x1 + a * f00 / (F1 * d2).sum() * d2
    assert np.allclose(r.pos, x2, rtol=1e-12, atol=1e-14)
    d_fr = F1 + f11 / f00 * F0
    x2_fr = x1 + a * f00 / (F1 * d_fr).sum() * d_fr
    assert np.abs(x2_fr - x2).max() > 1e-3


@pytest.fixture(scope="module")
def glass():
    s = S.uniform_glass_start(2, 256, 1, 0)
    H = O.box_matrix(2, s.L, 0.0)
    r = O.fire(s.pos, s.types, H, POT, FIRE)
    assert r.status == O.CONVERGED
    return r.pos, s.types, s.L


@pytest.mark.parametrize("r0", [1.3, 1.0, 2.0])
def test_dimer_reaches_the_analytic_minimum(r0):
    pos = np.array([[3.0, 4.0], [3.0 + r0, 4.0]])
    r = O.cg(pos, np.zeros(2, np.uint8), O.box_matrix(2, 12.0, 0.0), POT)
    assert r.status == O.CONVERGED
    assert abs(np.linalg.norm(r.pos[1] - r.pos[0]) - 2 ** (1 / 6)) < 1e-11
    assert r.E == pytest.approx(-0.983683108864, abs=1e-12)
    assert np.allclose(r.pos.mean(axis=0), pos.mean(axis=0), atol=1e-13)


def test_inherent_structure_and_lattice_take_zero_iterations(glass):
    pos, types, L = glass
    r = O.cg(pos, types, O.box_matrix(2, L, 0.0), POT)
    assert r.iters == 0 and r.status == O.CONVERGED and np.array_equal(r.pos, pos)
    a, nx, ny = 1.08, 8, 10
    lat = np.array([((i + 0.5 * (j % 2)) * a, j * a * math.sqrt(3) / 2) for j in range(ny) for i in range(nx)])
    H = O.box_matrix(2, [nx * a, ny * a * math.sqrt(3) / 2], 0.0)
    r = O.cg(lat, np.zeros(len(lat), np.uint8), H, POT)
    assert r.iters == 0 and r.status == O.CONVERGED


@pytest.mark.parametrize("dg", [1e-4, 1e-3])
def test_aqs_step_descends_is_certified_and_equals_fire(glass, dg):
    pos, types, L = glass
    H = O.strain_box(2, L, 1, dg)
    x = O.affine(pos, dg)
    E0, _, _, _ = O.energy_forces(x, types, H, POT)
    c = O.cg(x, types, H, POT)
    assert c.status == O.CONVERGED and c.E < E0
    E1, F1, _, _ = O.energy_forces(c.pos, types, H, POT)
    assert np.sqrt((F1 * F1).sum(1)).max() < 1e-10 and E1 == c.E
    f = O.fire(x, types, H, POT, FIRE)
    d, mean = O.compare(c.pos, f.pos, H)
    assert d < 1e-8 and np.abs(mean).max() < 1e-9
    assert abs(c.E - f.E) <= 1e-12 * abs(f.E)


def test_same_inherent_structure_as_fire_in_3d():
    s = S.uniform_glass_start(3, 400, 1, 0)
    H0 = O.box_matrix(3, s.L, 0.0)
    q = O.fire(s.pos, s.types, H0, POT, FIRE)
    assert q.status == O.CONVERGED
    dg = 5e-5
    H = O.strain_box(3, s.L, 1, dg)
    x = O.affine(q.pos, dg)
    c = O.cg(x, s.types, H, POT)
    f = O.fire(x, s.types, H, POT, FIRE)
    assert c.status == O.CONVERGED and f.status == O.CONVERGED
    assert O.compare(c.pos, f.pos, H)[0] < 1e-8


def test_first_step_respects_the_displacement_cap(glass):
    """After one update no atom has moved more than dmax (a1 <= dmax / max|F_i|)."""
    pos, types, L = glass
    dg = 2e-2
    H = O.strain_box(2, L, 1, dg)
    x = O.affine(pos, dg)
    _, F, _, _ = O.energy_forces(x, types, H, POT)
    p = O.CgParams(dmax=0.01, a_init=1.0, max_iter=1)
    assert 1.0 * np.sqrt((F * F).sum(1)).max() > p.dmax   # the cap is active
    r = O.cg(x, types, H, POT, p)
    assert r.status == O.MAXITER and r.iters == 1
    step = np.sqrt(((r.pos - x) ** 2).sum(1))
    assert step.max() <= p.dmax * (1 + 1e-12) and step.max() >= p.dmax * (1 - 1e-12)


def test_maxiter_and_determinism(glass):
    pos, types, L = glass
    dg = 1e-3
    H = O.strain_box(2, L, 1, dg)
    x = O.affine(pos, dg)
    a = O.cg(x, types, H, POT, O.CgParams(max_iter=9))
    b = O.cg(x, types, H, POT, O.CgParams(max_iter=9))
    assert a.status == O.MAXITER and a.iters == 9
    assert np.array_equal(a.pos, b.pos) and a.E == b.E


def test_nonfinite_input_is_reported():
    pos = np.array([[1.0, 1.0], [1.0, 1.0], [3.0, 3.0]])
    r = O.cg(pos, np.zeros(3, np.uint8), O.box_matrix(2, 12.0, 0.0), POT)
    assert r.status == O.NONFINITE and r.iters == 0


@pytest.mark.parametrize("n_fail_max", [0, 1, 3])
def test_stalled_after_n_fail_max_failed_line_searches(n_fail_max):
    """On E = sum x^2 / 2 (stiffness 1) a line search along d = F from x
    with trial step a has phi'(a) / phi'(0) = 1 - a, so the first trial
    a_init = 0.01 leaves |phi'| = 0.99 |phi'(0)| > sigma |phi'(0)|.  With
    ls_max = 0 every search fails at its first trial, restarts along the
    new F with a_init (same ratio), and the (n_fail_max + 1)-th failure in a
    row stops the minimiser: STALLED after n_fail_max + 1 iterations, each
    a trial step x <- 0.99 x."""
    x0 = np.array([[0.3, -0.2], [0.1, 0.25]])
    kk = np.ones_like(x0)
    p = O.CgParams(a_init=0.01, sigma=0.1, ls_max=0, n_fail_max=n_fail_max, dmax=10.0)
    r = O.cg_quadratic(x0, kk, p)
    assert r.status == O.STALLED and r.iters == n_fail_max + 1
    np.testing.assert_allclose(r.pos, x0 * 0.99 ** (n_fail_max + 1), rtol=1e-14)

"""Pins of the oracle's linear-response start (Eqs. 7-8 as one Newton step
from the affine start, conjugate gradients on probe Hessian-vector
products), CPU only."""
import numpy as np
import pytest

import aqs_synth as S
import oracle as O
from oracle import linear_response as LR

POT = O.kob_andersen()
FIRE = O.FireParams(dt0=0.01, dt_max=0.03, dt_min=2e-4, f_inc=1.2, f_dec=0.9, alpha0=0.2, f_alpha=0.95,
                    n_delay=5)


def _lj_derivs(r):
    """U'(r), U''(r) of 4 (r^-12 - r^-6) (epsilon = sigma = 1)."""
    return 4.0 * (-12.0 * r ** -13 + 6.0 * r ** -7), 4.0 * (156.0 * r ** -14 - 42.0 * r ** -8)


@pytest.mark.parametrize("r,dim", [(1.2, 2), (1.05, 3), (1.5, 2)])
def test_probe_hessian_vector_product_of_the_dimer(r, dim):
    """Analytic dimer Hessian: blocks +-K, K = U'' r^r^T + U'/r (I - r^r^T)."""
    L = 12.0
    x = np.full((2, dim), 4.0)
    d = np.zeros(dim)
    d[0], d[1] = 0.6, 0.8
    x[1] = x[0] + r * d
    H = O.box_matrix(dim, L, 0.0)
    u1, u2 = _lj_derivs(r)
    K = u2 * np.outer(d, d) + (u1 / r) * (np.eye(dim) - np.outer(d, d))
    Hfull = np.block([[K, -K], [-K, K]])
    v = S.rng_for(201, dim).normal(size=(2, dim))
    hv = LR.hessian_vector(x, np.zeros(2, np.uint8), H, POT, v)
    want = (Hfull @ v.ravel()).reshape(2, dim)
    assert np.abs(hv - want).max() <= 1e-6 * np.abs(want).max()


@pytest.mark.parametrize("r", [1.05, 1.15])
def test_dimer_start_is_the_newton_step(r):
    """The bond is an eigenvector (eigenvalue 2 U''): one CG iteration gives
    the separation r - U'(r) / U''(r)."""
    x = np.array([[3.0, 4.0], [3.0 + r, 4.0]])
    H = O.box_matrix(2, 12.0, 0.0)
    start, iters, ok, u = LR.linear_response_start(x, np.zeros(2, np.uint8), H, POT)
    u1, u2 = _lj_derivs(r)
    assert iters == 1 and ok
    assert abs((start[1, 0] - start[0, 0]) - (r - u1 / u2)) < 1e-8
    assert np.allclose(start.mean(0), x.mean(0), atol=1e-14)


@pytest.mark.parametrize("dim,n,dg", [(2, 256, 1e-4), (3, 400, 1e-5)])
def test_glass_start_is_closer_and_reaches_the_same_inherent_structure(dim, n, dg):
    s = S.uniform_glass_start(dim, n, 1, 0)
    q = O.fire(s.pos, s.types, O.box_matrix(dim, s.L, 0.0), POT, FIRE)
    assert q.status == O.CONVERGED
    H = O.strain_box(dim, s.L, 1, dg)
    x0 = O.affine(q.pos, dg)
    start, iters, ok, u = LR.linear_response_start(x0, s.types, H, POT)
    assert ok and iters >= 1
    E0 = O.energy_forces(x0, s.types, H, POT)[0]
    E1 = O.energy_forces(start, s.types, H, POT)[0]
    assert E1 < E0
    plain = O.fire(x0, s.types, H, POT, FIRE)
    lr = O.fire(start, s.types, H, POT, FIRE)
    assert plain.status == lr.status == O.CONVERGED
    assert O.compare(plain.pos, lr.pos, H)[0] < 1e-8
    assert lr.iters < plain.iters


def test_a_step_beyond_the_move_limit_keeps_the_affine_start():
    """At r = 1.2 the Newton step moves each atom 0.116 sigma > 0.1 sigma."""
    r = 1.2
    x = np.array([[3.0, 4.0], [3.0 + r, 4.0]])
    start, iters, ok, u = LR.linear_response_start(x, np.zeros(2, np.uint8), O.box_matrix(2, 12.0, 0.0), POT)
    u1, u2 = _lj_derivs(r)
    assert iters == 1 and not ok and np.array_equal(start, x)
    assert abs(abs(u[1, 0] - u[0, 0]) - u1 / u2) < 1e-8 and 0.5 * u1 / u2 > 0.1


def test_non_positive_curvature_stops_the_solve():
    """A dimer beyond the inflection point (U'' < 0 along the bond) stops at
    once and keeps the affine start."""
    r = 1.6
    x = np.array([[3.0, 4.0], [3.0 + r, 4.0]])
    start, iters, ok, u = LR.linear_response_start(x, np.zeros(2, np.uint8), O.box_matrix(2, 12.0, 0.0), POT)
    assert _lj_derivs(r)[1] < 0
    assert iters == 0 and np.array_equal(start, x)

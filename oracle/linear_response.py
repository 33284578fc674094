"""Linear-response start of an AQS step -- TEST INFRASTRUCTURE ONLY.

The paper's equation of equilibrium (Sec. 2.1, Eqs. 7-8): an inherent
structure strained by d gamma stays in equilibrium if its non-affine
displacement dr/d gamma solves  H dr/d gamma = F~, F~ the force the affine
deformation induces.  After an affine step from an inherent structure, the
force there is f(x0) = F~ d gamma to first order, so the non-affine
displacement of the step is u = H^-1 f(x0): one Newton step from the affine
start x0.  Here H = H(x0), and H v comes from central differences of the
forces, H v ~ (f(x0 - h v^) - f(x0 + h v^)) / (2 h) * max_i |v_i| with
v^ = v / max_i |v_i| (probe h in the max norm).

Steps, in order (the GPU's AQS_START_LINEAR takes the same ones):
  1  b = f(x0); r = b; p = r; u = 0; rr = |r|^2; bb = rr
  2  repeat at most max_cg times:
       pmax = max_i |p_i|; Hp from the probes x0 -/+ (h / pmax) p
       pHp = p . Hp; if pHp <= 0: stop (non-positive curvature)
       alpha = rr / pHp; u += alpha p; r -= alpha Hp; iters += 1
       rr' = |r|^2; if rr' <= tol^2 bb: stop
       beta = rr' / rr; rr = rr'; p = r + beta p
  3  accepted if max_i |u_i| <= max_move and E and max_i |F_i| at x0 + u
     do not exceed their values at x0; the start is x0 + u if accepted,
     else x0.
Sums over atoms and components are taken in atom order.  Pinned by: the
probe Hessian-vector product against the analytic Hessian of the dimer;
the dimer's start equal to the Newton step r - U'(r) / U''(r) along the
bond; and, on a glass, a start closer to the inherent structure than the
affine one that leads to the same inherent structure (Eq. 20).
"""
from __future__ import annotations

import numpy as np

from . import energy_forces


def _forces(x, types, H, pot):
    return energy_forces(x, types, H, pot)[1]


def hessian_vector(x0, types, H, pot, v, probe: float = 1e-5) -> np.ndarray:
    """H(x0) v by central differences of the forces (probe h in max norm)."""
    vmax = float(np.sqrt((v * v).sum(1)).max())
    s = probe / vmax
    fp = _forces(x0 + s * v, types, H, pot)
    fm = _forces(x0 - s * v, types, H, pot)
    return (fm - fp) / (2.0 * probe) * vmax


def linear_response_start(x0, types, H, pot, max_cg: int = 50, tol: float = 1e-3,
                          probe: float = 1e-5, max_move: float = 0.1):
    """(start, cg iterations, accepted, u) for an affine start x0."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    b = _forces(x0, types, H, pot)
    r = b.copy()
    p = r.copy()
    u = np.zeros_like(x0)
    rr = float((r * r).sum())
    bb = rr
    iters = 0
    for _ in range(max_cg):
        hp = hessian_vector(x0, types, H, pot, p, probe)
        php = float((p * hp).sum())
        if not php > 0.0:
            break
        alpha = rr / php
        u += alpha * p
        r -= alpha * hp
        iters += 1
        rr_new = float((r * r).sum())
        if rr_new <= tol * tol * bb:
            break
        beta = rr_new / rr
        rr = rr_new
        p = r + beta * p
    ok = bool(np.all(np.isfinite(u))) and float(np.sqrt((u * u).sum(1)).max()) <= max_move
    if ok:
        E0, F0, _, _ = energy_forces(x0, types, H, pot)
        E1, F1, _, _ = energy_forces(x0 + u, types, H, pot)
        ok = E1 <= E0 and np.sqrt((F1 * F1).sum(1)).max() <= np.sqrt((F0 * F0).sum(1)).max()
    return (x0 + u if ok else x0.copy()), iters, ok, u

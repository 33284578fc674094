"""CPU FP64 oracle of the AQS hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU path: the arithmetic is
in ``oracle.c`` (compiled with gcc, FP64, no FMA contraction) plus the plain
Python/NumPy modules next to it; this file only marshals arguments.

Method: Reihn, Bamer, Stamm, "Parallel athermal quasistatic deformation
stepping of molecular systems" (arXiv 2507.20802).

Parity status of each function is recorded next to it ("pinned by" = the
independent check in ``tests/test_oracle_*.py`` that would fail on a plausible
mistake).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

CONVERGED, MAXITER, STALLED, NONFINITE = 0, 1, 2, 3


class _Pot(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("eps", (ctypes.c_double * 2) * 2), ("sigma", (ctypes.c_double * 2) * 2),
                ("rc_factor", ctypes.c_double)]


class _Fire(ctypes.Structure):
    _fields_ = [("dt0", ctypes.c_double), ("dt_max", ctypes.c_double), ("dt_min", ctypes.c_double),
                ("f_inc", ctypes.c_double), ("f_dec", ctypes.c_double), ("alpha0", ctypes.c_double),
                ("f_alpha", ctypes.c_double), ("dmax", ctypes.c_double), ("ftol", ctypes.c_double),
                ("n_delay", ctypes.c_int32), ("n_neg_max", ctypes.c_int32),
                ("initial_delay", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("max_iter", ctypes.c_int64)]


class _Cg(ctypes.Structure):
    _fields_ = [("a_init", ctypes.c_double), ("sigma", ctypes.c_double), ("grow", ctypes.c_double),
                ("dmax", ctypes.c_double), ("ftol", ctypes.c_double),
                ("ls_max", ctypes.c_int32), ("n_fail_max", ctypes.c_int32), ("max_iter", ctypes.c_int64)]


@dataclass
class Potential:
    """Binary truncated-and-shifted LJ, Eq. (13); cutoff rc_ab = rc_factor sigma_ab."""
    eps: tuple = ((1.0, 1.5), (1.5, 0.5))
    sigma: tuple = ((1.0, 0.8), (0.8, 0.88))
    rc_factor: float = 2.5

    def c(self, dim: int) -> _Pot:
        p = _Pot()
        p.dim = dim
        for a in range(2):
            for b in range(2):
                p.eps[a][b] = self.eps[a][b]
                p.sigma[a][b] = self.sigma[a][b]
        p.rc_factor = self.rc_factor
        return p


def kob_andersen() -> Potential:
    """A = type 0, B = type 1: eps_AA = sigma_AA = 1, eps_AB = 1.5,
    sigma_AB = 0.8, eps_BB = 0.5, sigma_BB = 0.88, rc = 2.5 sigma_ab."""
    return Potential()


def paper_binary() -> Potential:
    """The paper's own binary glass, Eqs. (14)-(15): type 0 = small (S),
    type 1 = large (L)."""
    import math
    s_ss, s_ll = 2.0 * math.sin(math.pi / 10.0), 2.0 * math.sin(math.pi / 5.0)
    return Potential(eps=((0.5, 0.5), (0.5, 1.0)), sigma=((s_ss, 1.0), (1.0, s_ll)))


@dataclass
class FireParams:
    dt0: float = 0.005
    dt_max: float = 0.05
    dt_min: float = 1e-4
    f_inc: float = 1.1
    f_dec: float = 0.5
    alpha0: float = 0.25
    f_alpha: float = 0.99
    dmax: float = 0.1
    ftol: float = 1e-10
    n_delay: int = 20
    n_neg_max: int = 2000
    initial_delay: int = 1
    max_iter: int = 1_000_000

    def c(self) -> _Fire:
        f = _Fire()
        for k in ("dt0", "dt_max", "dt_min", "f_inc", "f_dec", "alpha0", "f_alpha", "dmax", "ftol",
                  "n_delay", "n_neg_max", "initial_delay", "max_iter"):
            setattr(f, k, getattr(self, k))
        return f


@dataclass
class CgParams:
    """Nonlinear conjugate gradients (see orc_cg in oracle.c): first trial
    step, curvature constant of the line search, largest extrapolation
    factor, largest displacement of an atom per line search, force
    tolerance, evaluations per line search, consecutive failed searches
    before STALLED, iteration limit."""
    a_init: float = 0.01
    sigma: float = 0.1
    grow: float = 4.0
    dmax: float = 0.1
    ftol: float = 1e-10
    ls_max: int = 20
    n_fail_max: int = 5
    max_iter: int = 1_000_000

    def c(self) -> _Cg:
        g = _Cg()
        for k in ("a_init", "sigma", "grow", "dmax", "ftol", "ls_max", "n_fail_max", "max_iter"):
            setattr(g, k, getattr(self, k))
        return g


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_eval.restype = ctypes.c_int
        L.orc_fire.restype = ctypes.c_int
        L.orc_cg.restype = ctypes.c_int
        L.orc_cg_quadratic.restype = ctypes.c_int
        L.orc_compare.restype = ctypes.c_int
        L.orc_forces_on.restype = ctypes.c_int
        L.orc_min_image_valid.restype = ctypes.c_int
        L.orc_pair.restype = ctypes.c_int
        L.orc_get_threads.restype = ctypes.c_int
        _LIB = L
        del dp
    return _LIB


def _d(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def box_matrix(dim: int, L, gamma: float) -> np.ndarray:
    """Bravais tensor H^(gamma) = F^(gamma) diag(L) for simple shear, Eq. (1)
    and Eq. (16): columns h_1 = (Lx, 0[, 0]), h_2 = (gamma Ly, Ly[, 0]),
    h_3 = (0, 0, Lz).  L is a scalar (square/cube) or a per-axis sequence."""
    Ls = np.broadcast_to(np.asarray(L, dtype=np.float64), (dim,))
    H = np.diag(Ls).astype(np.float64)
    H[0, 1] = gamma * Ls[1]
    return H


def strain_box(dim: int, L, k: int, dgamma: float, dgamma_y: float = 0.0) -> np.ndarray:
    """Box at strain index k.  Simple shear (dgamma_y = 0): gamma = k * dgamma,
    computed in one product so that equal indices give bit-identical boxes.
    Pure shear (Eq. 17, dgamma_y != 0): H_k = F^k diag(L) with
    F = [[1, dgamma], [dgamma_y, 1]] acting on (x, y) and z unchanged, F^k by
    deformation_power."""
    Ls = np.broadcast_to(np.asarray(L, dtype=np.float64), (dim,))
    H = np.diag(Ls).astype(np.float64)
    if dgamma_y == 0.0:
        H[0, 1] = (float(k) * dgamma) * Ls[1]
        return H
    M = deformation_power(dgamma, dgamma_y, k)
    H[0, 0] = M[0][0] * Ls[0]
    H[0, 1] = M[0][1] * Ls[1]
    H[1, 0] = M[1][0] * Ls[0]
    H[1, 1] = M[1][1] * Ls[1]
    return H


def deformation_power(a: float, b: float, k: int):
    """F^k for the 2x2 map F = [[1, a], [b, 1]] of Eq. (17), k >= 0, as nested
    lists of Python floats (FP64, no fused operations).  Square and multiply
    over the bits of k from the lowest: R <- R B when the bit is set, then
    B <- B B; each entry of a product is X[i][0] Y[0][j] + X[i][1] Y[1][j].
    Pinned by repeated multiplication, the eigenvalues 1 +- sqrt(ab), the
    determinant (1 - ab)^k and the simple-shear case b = 0 (F^k = [[1, ka], [0, 1]])."""
    if k < 0:
        raise ValueError("the strain index of a pure shear must be >= 0")

    def mul(X, Y):
        return [[X[0][0] * Y[0][0] + X[0][1] * Y[1][0], X[0][0] * Y[0][1] + X[0][1] * Y[1][1]],
                [X[1][0] * Y[0][0] + X[1][1] * Y[1][0], X[1][0] * Y[0][1] + X[1][1] * Y[1][1]]]

    R = [[1.0, 0.0], [0.0, 1.0]]
    B = [[1.0, float(a)], [float(b), 1.0]]
    while k:
        if k & 1:
            R = mul(R, B)
        B = mul(B, B)
        k >>= 1
    return R


def pair(pot: Potential, ti: int, tj: int, r: float):
    """(U(r) - U(rc), U'(r)/r, inside) for one pair.  Pinned by the dimer
    closed form and finite differences."""
    u = ctypes.c_double()
    g = ctypes.c_double()
    inside = lib().orc_pair(ctypes.byref(pot.c(2)), int(ti), int(tj), ctypes.c_double(r * r),
                            ctypes.byref(u), ctypes.byref(g))
    return u.value, g.value, bool(inside)


def energy_forces(pos: np.ndarray, types: np.ndarray, H: np.ndarray, pot: Potential,
                  image_sum: bool = False, image_range: int = 2):
    """(E, F[n, dim], stress[dim, dim], e_atom[n]) -- plain O(N^2) pair sums.
    Pinned by: finite differences, zero net force, lattice sums computed by
    shell enumeration, explicit image sum vs minimum image."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n, dim = pos.shape
    types = np.ascontiguousarray(types, dtype=np.uint8)
    Hc = np.ascontiguousarray(H, dtype=np.float64)
    E = ctypes.c_double()
    F = np.zeros((n, dim))
    S = np.zeros((dim, dim))
    ea = np.zeros(n)
    rc = lib().orc_eval(dim, n, _d(pos), types.ctypes.data_as(ctypes.c_void_p), _d(Hc),
                        ctypes.byref(pot.c(dim)), 1 if image_sum else 0, int(image_range),
                        ctypes.byref(E), _d(F), _d(S), _d(ea))
    if rc != 0:
        raise ValueError(f"orc_eval failed ({rc}): box with a z coupling or too small for the cutoff")
    return E.value, F, S, ea


def forces_on(pos: np.ndarray, types: np.ndarray, H: np.ndarray, pot: Potential, idx) -> np.ndarray:
    """Forces on the atoms idx only, each an O(N) minimum-image sum."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n, dim = pos.shape
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros((idx.size, dim))
    rc = lib().orc_forces_on(dim, n, _d(pos), np.ascontiguousarray(types, dtype=np.uint8).ctypes.data_as(ctypes.c_void_p),
                             _d(np.ascontiguousarray(H, dtype=np.float64)), ctypes.byref(pot.c(dim)),
                             int(idx.size), idx.ctypes.data_as(ctypes.c_void_p), _d(out))
    if rc != 0:
        raise ValueError(f"orc_forces_on failed ({rc})")
    return out


def min_image_valid(H: np.ndarray, pot: Potential) -> bool:
    dim = H.shape[0]
    return bool(lib().orc_min_image_valid(dim, _d(np.ascontiguousarray(H, dtype=np.float64)), ctypes.byref(pot.c(dim))))


def affine(pos: np.ndarray, dgamma: float, dgamma_y: float = 0.0, steps: int = 1) -> np.ndarray:
    """The affine map of `steps` increments.  Simple shear (dgamma_y = 0):
    x_i <- x_i + (steps dgamma) y_i (Eqs. 2-3, 16).  Pure shear (Eq. 17):
    (x_i, y_i) <- F^steps (x_i, y_i), z unchanged.  Returns a new array.
    Pinned by the composition law F(a) F(b) = F(a + b), the energy invariance
    under a shear by a full box period and, for the pure shear, the box
    sequence (fractional coordinates unchanged)."""
    out = np.ascontiguousarray(pos, dtype=np.float64).copy()
    n, dim = out.shape
    if dgamma_y == 0.0:
        lib().orc_affine(dim, n, _d(out), ctypes.c_double(float(steps) * dgamma if steps != 1 else dgamma))
        return out
    M = deformation_power(dgamma, dgamma_y, steps)
    Mc = np.ascontiguousarray([M[0][0], M[0][1], M[1][0], M[1][1]], dtype=np.float64)
    lib().orc_linear_xy(dim, n, _d(out), _d(Mc))
    return out


@dataclass
class FireResult:
    pos: np.ndarray
    iters: int
    E: float
    fmax: float
    status: int
    trace: np.ndarray


def fire(pos: np.ndarray, types: np.ndarray, H: np.ndarray, pot: Potential,
         params: FireParams | None = None, trace_cap: int = 0) -> FireResult:
    """The minimisation operator of Eq. (10) as FIRE 2.0 (see oracle.c).
    Pinned by: the dimer reaching 2^(1/6) sigma, zero iterations at an
    inherent structure and at a perfect lattice, E_end <= E_start, and
    certification of the end state by the independent force evaluation."""
    params = params or FireParams()
    x = np.ascontiguousarray(pos, dtype=np.float64).copy()
    n, dim = x.shape
    it = ctypes.c_int64()
    E = ctypes.c_double()
    fm = ctypes.c_double()
    st = ctypes.c_int32()
    tr = np.zeros(max(trace_cap, 1))
    rc = lib().orc_fire(dim, n, _d(x), np.ascontiguousarray(types, dtype=np.uint8).ctypes.data_as(ctypes.c_void_p),
                        _d(np.ascontiguousarray(H, dtype=np.float64)), ctypes.byref(pot.c(dim)),
                        ctypes.byref(params.c()), ctypes.byref(it), ctypes.byref(E), ctypes.byref(fm),
                        ctypes.byref(st), _d(tr), ctypes.c_int64(trace_cap))
    if rc != 0:
        raise ValueError(f"orc_fire failed ({rc})")
    ntr = min(int(it.value) + 1, trace_cap)
    return FireResult(x, int(it.value), E.value, fm.value, int(st.value), tr[:ntr].copy())


@dataclass
class CgResult:
    pos: np.ndarray
    iters: int
    dirs: int
    E: float
    fmax: float
    status: int


def cg(pos: np.ndarray, types: np.ndarray, H: np.ndarray, pot: Potential,
       params: CgParams | None = None) -> CgResult:
    """The minimisation operator of Eq. (10) by nonlinear conjugate gradients
    (Polak-Ribiere+, force-only line search; see oracle.c).  Pinned by: finite
    termination on quadratics (at most one search direction per distinct
    stiffness, two evaluations per search), the dimer reaching
    2^(1/6) sigma, zero iterations at an inherent structure, E_end <=
    E_start, the end state certified by the independent force evaluation,
    and the same inherent structure as FIRE (Eq. 20)."""
    params = params or CgParams()
    x = np.ascontiguousarray(pos, dtype=np.float64).copy()
    n, dim = x.shape
    it, nd, E, fm, st = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    rc = lib().orc_cg(dim, n, _d(x), np.ascontiguousarray(types, dtype=np.uint8).ctypes.data_as(ctypes.c_void_p),
                      _d(np.ascontiguousarray(H, dtype=np.float64)), ctypes.byref(pot.c(dim)),
                      ctypes.byref(params.c()), ctypes.byref(it), ctypes.byref(nd), ctypes.byref(E),
                      ctypes.byref(fm), ctypes.byref(st))
    if rc != 0:
        raise ValueError(f"orc_cg failed ({rc})")
    return CgResult(x, int(it.value), int(nd.value), E.value, fm.value, int(st.value))


def cg_quadratic(x0: np.ndarray, kk: np.ndarray, params: CgParams | None = None) -> CgResult:
    """The same conjugate-gradient core on E = sum k x^2 / 2 (x0, kk: [n, dim])."""
    params = params or CgParams()
    x = np.ascontiguousarray(x0, dtype=np.float64).copy()
    n, dim = x.shape
    kk = np.ascontiguousarray(kk, dtype=np.float64)
    it, nd, E, fm, st = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    lib().orc_cg_quadratic(dim, n, _d(x), _d(kk), ctypes.byref(params.c()), ctypes.byref(it), ctypes.byref(nd),
                           ctypes.byref(E), ctypes.byref(fm), ctypes.byref(st))
    return CgResult(x, int(it.value), int(nd.value), E.value, fm.value, int(st.value))


def compare(pos_a: np.ndarray, pos_b: np.ndarray, H: np.ndarray):
    """(max_i |minimg(a_i - b_i)|, mean displacement vector).  The distance
    used by the equality test of Eq. (20)."""
    a = np.ascontiguousarray(pos_a, dtype=np.float64)
    b = np.ascontiguousarray(pos_b, dtype=np.float64)
    n, dim = a.shape
    m = ctypes.c_double()
    mean = np.zeros(dim)
    rc = lib().orc_compare(dim, n, _d(a), _d(b), _d(np.ascontiguousarray(H, dtype=np.float64)), ctypes.byref(m), _d(mean))
    if rc != 0:
        raise ValueError("orc_compare failed")
    return m.value, mean


def max_force(pos, types, H, pot) -> float:
    _, F, _, _ = energy_forces(pos, types, H, pot)
    return float(np.sqrt((F * F).sum(axis=1)).max())


def equal_configs(pos_a, pos_b, H, delta_eq: float = 1e-4) -> bool:
    """a ~= b (Eq. 20) read as: max minimum-image displacement < delta_eq."""
    return compare(pos_a, pos_b, H)[0] < delta_eq

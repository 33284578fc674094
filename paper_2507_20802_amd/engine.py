"""Python face of the batched AQS engine (include/aqs.h).

PyTorch supplies the device workspace and the stream; the library does the
rest.  A context holds a batch of replica slots; the operators of the paper
(affine shear Eqs. 2-3/16, the minimisation operator Eq. 10 as FIRE 2.0, the
chained AQS steps Eqs. 12/19, the equality test Eq. 20, the stress of Fig. 2)
act on any subset of slots at once.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field

import numpy as np

from . import _lib
from ._lib import (AQS_START_LEARNED, AQS_START_PLAIN, aqs_check, aqs_fire_params, aqs_potential,
                   aqs_step_record, aqs_tuning, check)

STATUS_NAMES = {0: "converged", 1: "maxiter", 2: "stalled", 3: "nonfinite", 4: "cancelled"}


@dataclass
class LJParams:
    """Binary truncated-and-shifted Lennard-Jones, Eq. (13).  Default: the
    Kob-Andersen-type parameter set of the synthetic glasses (A = 0, B = 1)."""
    eps: tuple = ((1.0, 1.5), (1.5, 0.5))
    sigma: tuple = ((1.0, 0.8), (0.8, 0.88))
    rc_factor: float = 2.5

    def to_c(self, dim: int) -> aqs_potential:
        p = aqs_potential()
        p.dim = dim
        for a in range(2):
            for b in range(2):
                p.eps[a][b] = float(self.eps[a][b])
                p.sigma[a][b] = float(self.sigma[a][b])
        p.rc_factor = float(self.rc_factor)
        return p

    @property
    def rc_max(self) -> float:
        return self.rc_factor * max(max(r) for r in self.sigma)


@dataclass
class Fire:
    """FIRE 2.0 constants.  The defaults were chosen by an iteration-count
    search on synthetic glasses at max|F| < 1e-10."""
    dt0: float = 0.01
    dt_max: float = 0.03
    dt_min: float = 2e-4
    f_inc: float = 1.2
    f_dec: float = 0.9
    alpha0: float = 0.2
    f_alpha: float = 0.95
    dmax: float = 0.1
    ftol: float = 1e-10
    n_delay: int = 5
    n_neg_max: int = 2000
    initial_delay: int = 1
    max_iter: int = 1_000_000

    def to_c(self) -> aqs_fire_params:
        f = aqs_fire_params()
        for k in ("dt0", "dt_max", "dt_min", "f_inc", "f_dec", "alpha0", "f_alpha", "dmax", "ftol",
                  "n_delay", "n_neg_max", "initial_delay", "max_iter"):
            setattr(f, k, getattr(self, k))
        return f


@dataclass
class Cg:
    """Nonlinear conjugate gradients (aqs_set_minimizer): first trial step,
    curvature constant of the line search, largest extrapolation factor,
    largest displacement of an atom per line search, force tolerance,
    evaluations per line search, consecutive failed searches before
    STALLED, iteration limit."""
    a_init: float = 0.01
    sigma: float = 0.1
    grow: float = 4.0
    dmax: float = 0.1
    ftol: float = 1e-10
    ls_max: int = 20
    n_fail_max: int = 5
    max_iter: int = 1_000_000

    def to_c(self) -> "_lib.aqs_cg_params":
        g = _lib.aqs_cg_params()
        for k in ("a_init", "sigma", "grow", "dmax", "ftol", "ls_max", "n_fail_max", "max_iter"):
            setattr(g, k, getattr(self, k))
        return g


@dataclass
class Tuning:
    skin: float = 0.3
    max_neighbors: int = 0
    block_iters: int = 32
    use_graph: int = 0
    max_chain_steps: int = 1024
    threads_per_atom: int = 0
    live_batch_blocks: int = 0   # live rounds: batch force blocks per CU (0: 3; < 0: no limit)
    live_xcds: int = 0           # live rounds: XCDs reserved for the critical chain (0: none)
    tile_fill: float = 0.0       # force-tile atoms per block's atom lanes (0: 0.9)
    force_waves: int = 0         # force kernel occupancy target, waves per SIMD: 4 or 5 (0: 5)

    def to_c(self) -> aqs_tuning:
        t = aqs_tuning()
        t.skin = self.skin
        t.max_neighbors = self.max_neighbors
        t.block_iters = self.block_iters
        t.use_graph = self.use_graph
        t.max_chain_steps = self.max_chain_steps
        t.threads_per_atom = self.threads_per_atom
        t.live_batch_blocks = self.live_batch_blocks
        t.live_xcds = self.live_xcds
        t.tile_fill = self.tile_fill
        t.force_waves = self.force_waves
        return t


def _records(recs, n: int, width: int) -> np.ndarray:
    out = np.zeros((n, width), dtype=[("iters", np.int64), ("energy", np.float64),
                                      ("max_f", np.float64), ("sigma_xy", np.float64),
                                      ("status", np.int32), ("start", np.int32)])
    for i in range(n):
        for s in range(width):
            x = recs[i * width + s]
            out[i, s] = (x.iters, x.energy, x.max_f, x.sigma_xy, x.status, x.start)
    return out


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int64)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


class Engine:
    """A batch of replica slots on one GPU."""

    def __init__(self, dim: int, n_atoms, box_len, dgamma, pot: LJParams | None = None,
                 fire: Fire | None = None, tuning: "Tuning | str | None" = None, device: str = "cuda"):
        """tuning: knobs, None (defaults), "auto" (the autotuner's cached
        knobs for this shape, else the defaults) or "autotune" (run the
        autotuner when the shape is not cached)."""
        import torch
        self._lib = _lib.load()
        self.dim = int(dim)
        self.n_atoms = _i32(np.atleast_1d(n_atoms))
        self.n_rep = int(self.n_atoms.size)
        bl = np.asarray(box_len, dtype=np.float64)
        if bl.ndim == 0:
            bl = np.full((self.n_rep, self.dim), float(bl))
        elif bl.ndim == 1:
            bl = np.repeat(bl[:, None], self.dim, axis=1) if bl.size == self.n_rep else np.tile(bl, (self.n_rep, 1))
        self.box_len = _f64(bl.reshape(self.n_rep, self.dim))
        dg = np.asarray(dgamma, dtype=np.float64)
        self.dgamma = np.array(np.broadcast_to(dg, (self.n_rep,)), dtype=np.float64)   # own, writable copy
        self.pot = pot or LJParams()
        self.fire = fire or Fire()
        self.minimizer, self.cg = "fire", None
        if isinstance(tuning, str):   # "auto": the autotuner's cached knobs for this shape
            from . import autotune
            tuning = autotune.tuned(self.dim, self.n_atoms, self.n_rep,
                                    run_if_missing=(tuning == "autotune"))
        self.tuning = tuning or Tuning()
        self._cpot = self.pot.to_c(self.dim)
        self._cfire = self.fire.to_c()
        self._ctune = self.tuning.to_c()
        nbytes = self._lib.aqs_workspace_bytes(ctypes.byref(self._cpot), ctypes.byref(self._ctune),
                                               self.n_rep, _p(self.n_atoms, ctypes.c_int32),
                                               _p(self.box_len, ctypes.c_double))
        if nbytes == 0:
            raise _lib.AQSError(-1, "aqs_workspace_bytes", self._lib.aqs_last_error().decode())
        self.device = torch.device(device)
        self.workspace = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        # a captured iteration block needs a stream of its own (the default
        # stream cannot be captured); default priority
        self._stream = torch.cuda.Stream(self.device) if self.tuning.use_graph \
            else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        check(self._lib.aqs_create(ctypes.byref(self._cpot), ctypes.byref(self._cfire), ctypes.byref(self._ctune),
                                   self.n_rep, _p(self.n_atoms, ctypes.c_int32), _p(self.box_len, ctypes.c_double),
                                   _p(self.dgamma, ctypes.c_double), ctypes.c_void_p(aligned),
                                   ctypes.c_size_t(int(nbytes)), ctypes.c_void_p(self._stream.cuda_stream),
                                   ctypes.byref(ctx)), "aqs_create")
        self._ctx = ctx
        self.workspace_bytes = int(nbytes)

    # -- lifetime ---------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_ctx", None):
            self._lib.aqs_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- slots --------------------------------------------------------------
    def set_replica(self, rep: int, types, pos, strain_index: int = 0) -> None:
        t = np.ascontiguousarray(types, dtype=np.uint8)
        x = _f64(pos).reshape(-1)
        if t.size != self.n_atoms[rep] or x.size != self.n_atoms[rep] * self.dim:
            raise ValueError("types/positions do not match the slot's atom count")
        check(self._lib.aqs_set_replica(self._ctx, int(rep), t.ctypes.data_as(ctypes.c_void_p),
                                        _p(x, ctypes.c_double), int(strain_index)), "aqs_set_replica")

    def set_positions(self, rep: int, pos) -> None:
        x = _f64(pos).reshape(-1)
        if x.size != self.n_atoms[rep] * self.dim:
            raise ValueError("positions do not match the slot's atom count")
        check(self._lib.aqs_set_positions(self._ctx, int(rep), _p(x, ctypes.c_double)), "aqs_set_positions")

    def positions(self, rep: int) -> np.ndarray:
        out = np.zeros((int(self.n_atoms[rep]), self.dim))
        check(self._lib.aqs_get_positions(self._ctx, int(rep), _p(out, ctypes.c_double)), "aqs_get_positions")
        return out

    def strain_index(self, rep: int) -> int:
        k = ctypes.c_int64()
        check(self._lib.aqs_get_strain_index(self._ctx, int(rep), ctypes.byref(k)), "aqs_get_strain_index")
        return int(k.value)

    def box(self, rep: int) -> np.ndarray:
        """Bravais tensor of slot rep at its current strain index (Eq. 1), from
        the library (simple or pure shear)."""
        H = np.zeros((self.dim, self.dim), dtype=np.float64)
        check(self._lib.aqs_get_box(self._ctx, int(rep), H.ctypes.data_as(_lib.c_double_p)), "aqs_get_box")
        return H

    def copy_replica(self, src: int, dst: int) -> None:
        check(self._lib.aqs_copy_replica(self._ctx, int(src), int(dst)), "aqs_copy_replica")

    # -- operators ----------------------------------------------------------
    def affine_shear(self, reps, dk) -> None:
        r = _i32(np.atleast_1d(reps))
        d = _i64(np.broadcast_to(np.atleast_1d(dk), r.shape))
        check(self._lib.aqs_affine_shear(self._ctx, int(r.size), _p(r, ctypes.c_int32), _p(d, ctypes.c_int64)),
              "aqs_affine_shear")

    def minimize(self, reps, n_steps=None, snap_dst=None, start: int = AQS_START_PLAIN) -> np.ndarray:
        """Minimise the slots, then run n_steps fine AQS steps on the device.
        Returns a (len(reps), max(n_steps)+1) structured array of records."""
        r = _i32(np.atleast_1d(reps))
        ns = None if n_steps is None else _i32(np.broadcast_to(np.atleast_1d(n_steps), r.shape))
        sd = None if snap_dst is None else _i32(np.broadcast_to(np.atleast_1d(snap_dst), r.shape))
        width = 1 + (int(ns.max()) if ns is not None and ns.size else 0)
        recs = (aqs_step_record * (r.size * width))()
        for x in recs:
            x.status = -1
        check(self._lib.aqs_minimize_batch(self._ctx, int(r.size), _p(r, ctypes.c_int32), int(start),
                                           None if ns is None else _p(ns, ctypes.c_int32),
                                           None if sd is None else _p(sd, ctypes.c_int32), recs),
              "aqs_minimize_batch")
        return _records(recs, r.size, width)

    def run_round(self, chains, snaps, n_steps, start: int = AQS_START_PLAIN, delta_eq: float = 1e-4,
                  live: bool = False, abandon: bool = False):
        """Level II and the checks of one round of Algorithm 1 (aqs_run_round):
        chain i (already at its level-I start) is minimised, then runs
        n_steps[i] fine steps; check i compares the end of chain i-1 with the
        first inherent structure of chain i, copied into snaps[i].  With live,
        checks are taken as soon as possible and chains after a failed check
        stop; with abandon also, a stress drop in the critical chain stops the
        chains after it before its check (decided = 2).  Returns (records (P,
        max n_steps + 1), checks) where checks[i] = (decided, equal, max_disp,
        dE/N) for i >= 1."""
        c = _i32(np.atleast_1d(chains))
        P = int(c.size)
        sn = _i32(np.broadcast_to(np.atleast_1d(snaps), c.shape))
        ns = _i32(np.broadcast_to(np.atleast_1d(n_steps), c.shape))
        width = 1 + int(ns.max())
        recs = (aqs_step_record * (P * width))()
        for x in recs:
            x.status = -1
        chk = (aqs_check * P)()
        check(self._lib.aqs_run_round(self._ctx, P, _p(c, ctypes.c_int32), _p(sn, ctypes.c_int32),
                                      _p(ns, ctypes.c_int32), int(start), float(delta_eq),
                                      (2 if abandon else 1) if live else 0, recs, chk), "aqs_run_round")
        checks = [(int(x.decided), bool(x.equal), x.max_disp, x.de_per_atom) for x in chk]
        return _records(recs, P, width), checks

    def compare(self, a: int, b: int, delta_eq: float = 1e-4):
        """(equal, max_disp, dE/N) of the equality test, Eq. (20)."""
        eq = ctypes.c_int32()
        md = ctypes.c_double()
        de = ctypes.c_double()
        check(self._lib.aqs_compare_configs(self._ctx, int(a), int(b), float(delta_eq), ctypes.byref(eq),
                                            ctypes.byref(md), ctypes.byref(de)), "aqs_compare_configs")
        return bool(eq.value), md.value, de.value

    def stress(self, rep: int):
        s = np.zeros((self.dim, self.dim))
        e = ctypes.c_double()
        check(self._lib.aqs_stress(self._ctx, int(rep), _p(s, ctypes.c_double), ctypes.byref(e)), "aqs_stress")
        return s, e.value

    def energy_forces(self, rep: int):
        f = np.zeros((int(self.n_atoms[rep]), self.dim))
        e = ctypes.c_double()
        check(self._lib.aqs_energy_forces(self._ctx, int(rep), ctypes.byref(e), _p(f, ctypes.c_double)),
              "aqs_energy_forces")
        return e.value, f

    # -- measurement ------------------------------------------------------
    def set_minimizer(self, kind: str = "fire", cg: "Cg | None" = None) -> None:
        """Minimiser of the later minimisations: "fire" (FIRE 2.0) or "cg"
        (nonlinear conjugate gradients with the constants cg)."""
        if kind == "fire":
            check(self._lib.aqs_set_minimizer(self._ctx, _lib.AQS_MIN_FIRE, None), "aqs_set_minimizer")
        elif kind == "cg":
            self.cg = cg or Cg()
            check(self._lib.aqs_set_minimizer(self._ctx, _lib.AQS_MIN_CG, ctypes.byref(self.cg.to_c())),
                  "aqs_set_minimizer")
        else:
            raise ValueError(f"unknown minimiser {kind!r}")
        self.minimizer = kind

    def set_live_batch_blocks(self, blocks: int) -> None:
        """Batch force blocks per CU beside the critical chain of later live
        rounds (0: the default, 3; < 0: no limit); changes no result."""
        check(self._lib.aqs_set_live_batch_blocks(self._ctx, int(blocks)), "aqs_set_live_batch_blocks")

    def set_live_xcds(self, xcds: int) -> None:
        """XCDs of the 8 reserved for the critical chain of later live rounds
        (0: no partition); changes no result."""
        check(self._lib.aqs_set_live_xcds(self._ctx, int(xcds)), "aqs_set_live_xcds")

    def set_dgamma(self, slots, dgamma) -> None:
        """New fine strain increments of the slots, their strains kept exactly
        (the strain index converts; dynamic step sizing)."""
        sel = _i32(slots)
        dg = np.ascontiguousarray(np.broadcast_to(np.asarray(dgamma, dtype=np.float64), sel.shape))
        check(self._lib.aqs_set_dgamma(self._ctx, int(sel.size), sel.ctypes.data_as(_lib.c_int32_p),
                                       dg.ctypes.data_as(_lib.c_double_p)), "aqs_set_dgamma")
        self.dgamma[sel] = dg

    def set_linear_start(self, max_cg: int = 50, tol: float = 1e-3, probe: float = 1e-5) -> None:
        """Parameters of the linear-response start (AQS_START_LINEAR): at most
        max_cg conjugate-gradient updates, stop at |r| <= tol |f(x0)|, probe
        length of the Hessian-vector products."""
        check(self._lib.aqs_set_linear_start(self._ctx, int(max_cg), float(tol), float(probe)),
              "aqs_set_linear_start")

    def set_live_duty(self, duty: int) -> None:
        """Later live rounds: the batch of speculative chains runs one block of
        iterations in `duty` while a critical chain runs (1: always); changes no
        result."""
        check(self._lib.aqs_set_live_duty(self._ctx, int(duty)), "aqs_set_live_duty")

    def set_pure_shear(self, slots, dgamma_y) -> None:
        """Deformation of the slots: dgamma_y = 0 simple shear (Eq. 16), else
        the pure shear of Eq. (17), F = [[1, dgamma], [dgamma_y, 1]] on (x, y).
        Slots must be idle; set it before loading positions."""
        sel = _i32(slots)
        dy = np.ascontiguousarray(np.broadcast_to(np.asarray(dgamma_y, dtype=np.float64), sel.shape))
        check(self._lib.aqs_set_pure_shear(self._ctx, int(sel.size), sel.ctypes.data_as(_lib.c_int32_p),
                                           dy.ctypes.data_as(_lib.c_double_p)), "aqs_set_pure_shear")

    def set_profiling(self, every_nth_block: int) -> None:
        check(self._lib.aqs_set_profiling(self._ctx, int(every_nth_block)), "aqs_set_profiling")

    def counters(self, reset: bool = False) -> dict:
        c = _lib.aqs_counters()
        check(self._lib.aqs_get_counters(self._ctx, ctypes.byref(c), int(reset)), "aqs_get_counters")
        return {k: getattr(c, k) for k, _ in c._fields_}

    # -- learned start ----------------------------------------------------
    def _dev_f32(self, rows: int, cols: int, out=None):
        import torch
        if out is None:
            out = torch.empty((rows, cols), dtype=torch.float32, device=self.device)
        if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() < rows * cols \
                or not out.is_cuda:
            raise ValueError("output must be a contiguous float32 tensor on the engine's device")
        return out

    def learned_features(self, rep: int, out=None):
        """Descriptors of slot rep (n x 64 float32 tensor on the device,
        atom-id order)."""
        n = int(self.n_atoms[rep])
        out = self._dev_f32(n, 64, out)
        check(self._lib.aqs_learned_features(self._ctx, int(rep), ctypes.c_void_p(out.data_ptr())),
              "aqs_learned_features")
        return out

    def learned_targets(self, rep_prev: int, rep_next: int, out=None):
        """Non-affine displacement per unit strain from slot rep_prev to
        slot rep_next (n x dim float32 tensor on the device, atom-id order)."""
        n = int(self.n_atoms[rep_next])
        out = self._dev_f32(n, self.dim, out)
        check(self._lib.aqs_learned_targets(self._ctx, int(rep_prev), int(rep_next),
                                            ctypes.c_void_p(out.data_ptr())), "aqs_learned_targets")
        return out

    def learned_load(self, model: "_lib.aqs_mlp") -> None:
        check(self._lib.aqs_learned_load(self._ctx, ctypes.byref(model)), "aqs_learned_load")

    def learned_predict(self, rep: int, out=None):
        n = int(self.n_atoms[rep])
        out = self._dev_f32(n, self.dim, out)
        check(self._lib.aqs_learned_predict(self._ctx, int(rep), ctypes.c_void_p(out.data_ptr())),
              "aqs_learned_predict")
        return out

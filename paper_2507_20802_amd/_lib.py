"""ctypes binding of libaqs.so (the C ABI in include/aqs.h).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaqs.so")

AQS_OK, AQS_EINVAL, AQS_EHIP, AQS_ENOMEM, AQS_ECAPACITY, AQS_ESTATE = 0, -1, -2, -3, -4, -5
AQS_CONVERGED, AQS_MAXITER, AQS_STALLED, AQS_NONFINITE, AQS_CANCELLED = 0, 1, 2, 3, 4
AQS_START_PLAIN, AQS_START_LEARNED, AQS_START_FALLBACK, AQS_START_EXTRAPOLATED, AQS_START_LINEAR = 0, 1, 2, 3, 4
AQS_MIN_FIRE, AQS_MIN_CG = 0, 1

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int32_p = ctypes.POINTER(ctypes.c_int32)
c_int64_p = ctypes.POINTER(ctypes.c_int64)


class aqs_potential(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("eps", (ctypes.c_double * 2) * 2), ("sigma", (ctypes.c_double * 2) * 2),
                ("rc_factor", ctypes.c_double)]


class aqs_fire_params(ctypes.Structure):
    _fields_ = [("dt0", ctypes.c_double), ("dt_max", ctypes.c_double), ("dt_min", ctypes.c_double),
                ("f_inc", ctypes.c_double), ("f_dec", ctypes.c_double), ("alpha0", ctypes.c_double),
                ("f_alpha", ctypes.c_double), ("dmax", ctypes.c_double), ("ftol", ctypes.c_double),
                ("n_delay", ctypes.c_int32), ("n_neg_max", ctypes.c_int32),
                ("initial_delay", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("max_iter", ctypes.c_int64)]


class aqs_cg_params(ctypes.Structure):
    _fields_ = [("a_init", ctypes.c_double), ("sigma", ctypes.c_double), ("grow", ctypes.c_double),
                ("dmax", ctypes.c_double), ("ftol", ctypes.c_double), ("ls_max", ctypes.c_int32),
                ("n_fail_max", ctypes.c_int32), ("max_iter", ctypes.c_int64)]


class aqs_tuning(ctypes.Structure):
    _fields_ = [("skin", ctypes.c_double), ("max_neighbors", ctypes.c_int32),
                ("block_iters", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("max_chain_steps", ctypes.c_int32), ("threads_per_atom", ctypes.c_int32),
                ("live_batch_blocks", ctypes.c_int32), ("live_xcds", ctypes.c_int32),
                ("force_waves", ctypes.c_int32), ("tile_fill", ctypes.c_double)]


class aqs_step_record(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("energy", ctypes.c_double), ("max_f", ctypes.c_double),
                ("sigma_xy", ctypes.c_double), ("status", ctypes.c_int32), ("start", ctypes.c_int32)]


class aqs_check(ctypes.Structure):
    _fields_ = [("decided", ctypes.c_int32), ("equal", ctypes.c_int32), ("max_disp", ctypes.c_double),
                ("de_per_atom", ctypes.c_double)]


class aqs_counters(ctypes.Structure):
    _fields_ = [("force_ms", ctypes.c_double), ("force_timed", ctypes.c_int64),
                ("update_ms", ctypes.c_double), ("update_timed", ctypes.c_int64),
                ("force_launches", ctypes.c_int64), ("rebuilds", ctypes.c_int64),
                ("host_polls", ctypes.c_int64), ("atom_evals", ctypes.c_int64),
                ("timed_atom_evals", ctypes.c_int64)]


class aqs_mlp(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("w1", ctypes.c_float * (64 * 128)), ("b1", ctypes.c_float * 128),
                ("w2", ctypes.c_float * (128 * 128)), ("b2", ctypes.c_float * 128),
                ("w3", ctypes.c_float * (128 * 3)), ("b3", ctypes.c_float * 3),
                ("feat_mean", ctypes.c_float * 64), ("feat_std", ctypes.c_float * 64),
                ("tgt_mean", ctypes.c_float * 3), ("tgt_std", ctypes.c_float * 3)]


class aqs_train_params(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("huber_delta", ctypes.c_float), ("batch", ctypes.c_int32),
                ("epochs", ctypes.c_int32), ("pad_", ctypes.c_int32)]


c_float_p = ctypes.POINTER(ctypes.c_float)

# name -> (restype, argtypes); every symbol declared in include/aqs.h
SIGNATURES = {
    "aqs_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(aqs_potential), ctypes.POINTER(aqs_tuning),
                                              ctypes.c_int32, c_int32_p, c_double_p]),
    "aqs_create": (ctypes.c_int32, [ctypes.POINTER(aqs_potential), ctypes.POINTER(aqs_fire_params),
                                    ctypes.POINTER(aqs_tuning), ctypes.c_int32, c_int32_p, c_double_p,
                                    c_double_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_void_p)]),
    "aqs_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "aqs_set_replica": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, c_double_p,
                                         ctypes.c_int64]),
    "aqs_set_positions": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, c_double_p]),
    "aqs_get_positions": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, c_double_p]),
    "aqs_get_strain_index": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, c_int64_p]),
    "aqs_get_box": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, c_double_p]),
    "aqs_copy_replica": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "aqs_affine_shear": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, c_int32_p, c_int64_p]),
    "aqs_minimize_batch": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, c_int32_p, ctypes.c_int32,
                                            c_int32_p, c_int32_p, ctypes.POINTER(aqs_step_record)]),
    "aqs_run_round": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, c_int32_p, c_int32_p, c_int32_p,
                                       ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                       ctypes.POINTER(aqs_step_record), ctypes.POINTER(aqs_check)]),
    "aqs_compare_configs": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_double, c_int32_p, c_double_p, c_double_p]),
    "aqs_stress": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, c_double_p, c_double_p]),
    "aqs_energy_forces": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, c_double_p, c_double_p]),
    "aqs_set_profiling": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "aqs_set_live_batch_blocks": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "aqs_set_live_xcds": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "aqs_set_pure_shear": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, c_int32_p, c_double_p]),
    "aqs_set_live_duty": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "aqs_set_dgamma": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, c_int32_p, c_double_p]),
    "aqs_set_linear_start": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_double]),
    "aqs_set_minimizer": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(aqs_cg_params)]),
    "aqs_get_counters": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(aqs_counters), ctypes.c_int32]),
    "aqs_learned_load": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(aqs_mlp)]),
    "aqs_learned_features": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "aqs_learned_predict": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "aqs_learned_targets": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_void_p]),
    "aqs_mlp_train": (ctypes.c_int32, [ctypes.POINTER(aqs_train_params), ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(aqs_mlp),
                                       c_float_p, ctypes.c_void_p]),
    "aqs_mlp_train_static": (ctypes.c_int32, [ctypes.POINTER(aqs_train_params), ctypes.c_int64, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(aqs_mlp),
                                              c_float_p, ctypes.c_void_p]),
    "aqs_mlp_gradients": (ctypes.c_int32, [ctypes.POINTER(aqs_mlp), ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_float, ctypes.POINTER(aqs_mlp),
                                           c_float_p, ctypes.c_void_p]),
    "aqs_last_error": (ctypes.c_char_p, []),
}

_LIB = None


class AQSError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} returned {code}: {msg}")
        self.code = code


def load() -> ctypes.CDLL:
    """Load libaqs.so; raise if it is missing (there is no fallback path)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              f"`python -c 'import __graft_entry__ as g; g.build()'`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def check(code: int, where: str) -> None:
    if code != AQS_OK:
        msg = load().aqs_last_error().decode(errors="replace")
        raise AQSError(code, where, msg)

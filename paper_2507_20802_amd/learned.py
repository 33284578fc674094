"""The per-atom network of the learned start: host-side containers and the
GPU training call (aqs_mlp_train / aqs_mlp_gradients of include/aqs.h).

Training, inference and descriptors run in the HIP kernels of libaqs.so;
this module only moves arrays between NumPy, torch device tensors and the
C structures.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import aqs_mlp, aqs_train_params, check

PARAMS = ("w1", "b1", "w2", "b2", "w3", "b3")
SHAPES = {"w1": (64, 128), "b1": (128,), "w2": (128, 128), "b2": (128,), "w3": (128, 3), "b3": (3,)}


@dataclass
class TrainParams:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    huber_delta: float = 1.0
    batch: int = 4096
    epochs: int = 50

    def to_c(self) -> aqs_train_params:
        p = aqs_train_params()
        p.lr, p.beta1, p.beta2, p.eps = self.lr, self.beta1, self.beta2, self.eps
        p.huber_delta, p.batch, p.epochs = self.huber_delta, self.batch, self.epochs
        return p


def _view(m: aqs_mlp, name: str) -> np.ndarray:
    return np.ctypeslib.as_array(getattr(m, name))


def make_mlp(dim: int, params: dict, feat_mean=None, feat_std=None, tgt_mean=None, tgt_std=None) -> aqs_mlp:
    """aqs_mlp from [in, out] weight arrays (w3 may have dim columns)."""
    m = aqs_mlp()
    m.dim = int(dim)
    for k in PARAMS:
        a = np.asarray(params[k], dtype=np.float32)
        full = np.zeros(SHAPES[k], dtype=np.float32)
        if k == "w3":
            full[:, :a.shape[1]] = a
        elif k == "b3":
            full[:a.shape[0]] = a
        else:
            full[...] = a
        _view(m, k)[:] = full.reshape(-1)
    _view(m, "feat_mean")[:] = 0.0 if feat_mean is None else np.asarray(feat_mean, np.float32)
    _view(m, "feat_std")[:] = 1.0 if feat_std is None else np.asarray(feat_std, np.float32)
    tm = np.zeros(3, np.float32)
    ts = np.ones(3, np.float32)
    if tgt_mean is not None:
        tm[:dim] = np.asarray(tgt_mean, np.float32)[:dim]
    if tgt_std is not None:
        ts[:dim] = np.asarray(tgt_std, np.float32)[:dim]
    _view(m, "tgt_mean")[:] = tm
    _view(m, "tgt_std")[:] = ts
    return m


def mlp_arrays(m: aqs_mlp) -> dict:
    """Copies of the parameters ([in, out], w3 and b3 cut to dim outputs)
    and of the standardisation."""
    d = m.dim
    out = {k: _view(m, k).reshape(SHAPES[k]).copy() for k in PARAMS}
    out["w3"] = out["w3"][:, :d].copy()
    out["b3"] = out["b3"][:d].copy()
    out["feat_mean"] = _view(m, "feat_mean").copy()
    out["feat_std"] = _view(m, "feat_std").copy()
    out["tgt_mean"] = _view(m, "tgt_mean")[:d].copy()
    out["tgt_std"] = _view(m, "tgt_std")[:d].copy()
    return out


def _stream_ptr(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _check_dev(t, dtype, shape=None):
    import torch
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous {dtype} device tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")


def train(model: aqs_mlp, feat, target, orders, params: TrainParams | None = None,
          static: bool = False) -> np.ndarray:
    """Train model in place on the GPU.  feat: (n, 64) float32 device tensor,
    target: (n, dim) float32, orders: (epochs, n) int32 (one sample order per
    epoch).  static: through aqs_mlp_train_static (no device allocation; at
    most 65536 samples).  Returns the mean batch loss of every epoch."""
    import torch
    lib = _lib.load()
    params = params or TrainParams(epochs=int(orders.shape[0]))
    n = int(feat.shape[0])
    _check_dev(feat, torch.float32, (n, 64))
    _check_dev(target, torch.float32, (n, model.dim))
    _check_dev(orders, torch.int32, (params.epochs, n))
    hist = np.zeros(params.epochs, dtype=np.float32)
    cp = params.to_c()
    name = "aqs_mlp_train_static" if static else "aqs_mlp_train"
    check(getattr(lib, name)(ctypes.byref(cp), n, ctypes.c_void_p(feat.data_ptr()),
                             ctypes.c_void_p(target.data_ptr()), ctypes.c_void_p(orders.data_ptr()),
                             ctypes.byref(model), hist.ctypes.data_as(_lib.c_float_p), _stream_ptr(feat)),
          name)
    return hist


def gradients(model: aqs_mlp, feat, target, huber_delta: float = 1.0):
    """(loss, gradient dict) of the mean Huber loss over all samples, one batch."""
    import torch
    lib = _lib.load()
    n = int(feat.shape[0])
    _check_dev(feat, torch.float32, (n, 64))
    _check_dev(target, torch.float32, (n, model.dim))
    g = aqs_mlp()
    loss = ctypes.c_float()
    check(lib.aqs_mlp_gradients(ctypes.byref(model), n, ctypes.c_void_p(feat.data_ptr()),
                                ctypes.c_void_p(target.data_ptr()), float(huber_delta), ctypes.byref(g),
                                ctypes.byref(loss), _stream_ptr(feat)), "aqs_mlp_gradients")
    return loss.value, mlp_arrays(g)


def collect_samples(engine, slot: int, spare: int, steps: int):
    """Training samples from `steps` plain AQS steps of the inherent
    structure in `slot` (Eq. 12): the descriptors at each inherent structure
    and the non-affine displacement per unit strain of the step that follows
    it.  `spare` (same atom count) holds the previous inherent structure.
    Returns (feat (steps*n, 64), target (steps*n, dim)) float32 device
    tensors and the per-step records."""
    import torch
    n = int(engine.n_atoms[slot])
    feat = torch.empty((steps * n, 64), dtype=torch.float32, device=engine.device)
    tgt = torch.empty((steps * n, engine.dim), dtype=torch.float32, device=engine.device)
    recs = []
    for s in range(steps):
        engine.copy_replica(slot, spare)
        engine.learned_features(spare, out=feat[s * n:(s + 1) * n])
        r = engine.minimize([slot], n_steps=[1])
        recs.append(r[0, 1])
        if r[0, 1]["status"] != 0:
            raise RuntimeError(f"plain AQS step {s} did not converge (status {r[0, 1]['status']})")
        engine.learned_targets(spare, slot, out=tgt[s * n:(s + 1) * n])
    return feat, tgt, recs

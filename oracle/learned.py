"""Learned start of an AQS step -- CPU oracle, TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the GPU path.

The paper (arXiv 2507.20802) minimises from the affinely deformed
configuration F r (Eq. 12, Sec. 2.1) and names better starting points for
the minimiser as future work (Sec. 5).  The learned start replaces the
plain start F r by F r + dgamma (u_hat - mean u_hat), where u_hat is the
non-affine displacement per unit strain predicted for each atom by a small
per-atom network from descriptors of its neighbourhood at the previous
inherent structure.  Definitions (this project's, see the functions):

* descriptors, 64 per atom at the inherent structure, minimum image in the
  current box, neighbours j within the pair cutoff r_d = rc_ab of the
  potential (2.5 sigma_ab), smooth cutoff f_c(r) = (cos(pi r / r_d) + 1) / 2:
  - radial, 2 neighbour species x 24 Gaussians exp(-(r - mu_b)^2 / (2 w^2)),
    mu_b = 0.6 + b w, w = (2.5 - 0.6) / 23, each weighted by f_c;
  - angular, 16 lab-frame directions n_k: sum_j f_c max(0, n_k . r_ij/r)^2;
    2D: n_k at angles 2 pi k / 16; 3D: the 16 points of a Fibonacci sphere.
* network 64 -> 128 -> SiLU -> 128 -> SiLU -> d, BF16 weights and
  activations at the layer inputs, FP32 accumulation, biases and SiLU
  (``mlp_forward`` with ``emulate=True`` rounds where the GPU rounds);
* target: u_i / dgamma with u_i = minimg(r_i(IS_k) - F r_i(IS_(k-1))) from
  plain AQS steps; features standardised with training-set mean and std
  (FP32) and rounded to BF16, targets with trimmed statistics (samples
  farther than 5 std from the mean, recomputed three times, are left out:
  plastic jumps);
* loss: Huber (delta in standardised units), mean over samples and
  components; optimiser: Adam.

Parity status: descriptors pinned by an explicit image-sum brute force and
closed-form invariants; the network by finite differences (FP64 mode) and by
torch's CPU layers; Huber and Adam by torch's CPU implementations; the BF16
rounding by torch's bfloat16 conversion.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

N_RADIAL = 24
N_SPECIES = 2
N_ANGULAR = 16
N_FEAT = N_SPECIES * N_RADIAL + N_ANGULAR  # 64
HIDDEN = 128
MU_LO, MU_HI = 0.6, 2.5
WIDTH = (MU_HI - MU_LO) / (N_RADIAL - 1)


# ---------------------------------------------------------------------------
# descriptors

def directions(dim: int) -> np.ndarray:
    """The 16 unit vectors n_k of the angular features."""
    k = np.arange(N_ANGULAR, dtype=np.float64)
    if dim == 2:
        a = 2.0 * math.pi * k / N_ANGULAR
        return np.stack([np.cos(a), np.sin(a)], axis=1)
    z = 1.0 - (2.0 * k + 1.0) / N_ANGULAR
    rho = np.sqrt(1.0 - z * z)
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def centres() -> np.ndarray:
    return MU_LO + WIDTH * np.arange(N_RADIAL, dtype=np.float64)


def pair_cutoffs(pot) -> np.ndarray:
    """r_d for each type pair: the potential's cutoff rc_ab = rc_factor sigma_ab."""
    return pot.rc_factor * np.asarray(pot.sigma, dtype=np.float64)


def descriptors(pos: np.ndarray, types: np.ndarray, H: np.ndarray, pot, idx=None,
                chunk: int = 256) -> np.ndarray:
    """Descriptors (FP64, [len(idx), 64]) of atoms idx (all by default).

    Neighbours by the minimum image in box H (valid while every r_d is below
    half the smallest perpendicular width of H, which the caller's box
    satisfies)."""
    pos = np.asarray(pos, dtype=np.float64)
    n, dim = pos.shape
    types = np.asarray(types).astype(np.int64)
    idx = np.arange(n) if idx is None else np.asarray(idx, dtype=np.int64)
    Hinv = np.linalg.inv(H)
    rd = pair_cutoffs(pot)
    mu = centres()
    nk = directions(dim)
    out = np.zeros((len(idx), N_FEAT), dtype=np.float64)
    for c0 in range(0, len(idx), chunk):
        ii = idx[c0:c0 + chunk]
        d = pos[None, :, :] - pos[ii, None, :]            # r_j - r_i
        s = d @ Hinv.T
        s -= np.rint(s)
        d = s @ H.T
        r = np.sqrt((d * d).sum(-1))
        rcut = rd[types[ii][:, None], types[None, :]]
        live = (r < rcut) & (np.arange(n)[None, :] != ii[:, None])
        a, j = np.nonzero(live)
        rr = r[a, j]
        fc = 0.5 * (np.cos(math.pi * rr / rcut[a, j]) + 1.0)
        g = np.exp(-((rr[:, None] - mu[None, :]) ** 2) / (2.0 * WIDTH * WIDTH)) * fc[:, None]
        col = types[j][:, None] * N_RADIAL + np.arange(N_RADIAL)[None, :]
        np.add.at(out[c0:c0 + len(ii)], (np.repeat(a, N_RADIAL), col.ravel()), g.ravel())
        u = d[a, j] / rr[:, None]
        proj = np.maximum(u @ nk.T, 0.0)
        np.add.at(out[c0:c0 + len(ii)], (np.repeat(a, N_ANGULAR),
                                         np.tile(np.arange(N_SPECIES * N_RADIAL, N_FEAT), len(a))),
                  (fc[:, None] * proj * proj).ravel())
    return out


def nonaffine_targets(prev_is: np.ndarray, next_is: np.ndarray, H_next: np.ndarray,
                      dgamma: float, steps: int = 1) -> np.ndarray:
    """u_i / dgamma, u_i = minimg(r_i(IS_k) - F r_i(IS_(k-1))) in the box of
    IS_k; F is the simple shear by steps * dgamma (Eq. 16)."""
    x = np.array(prev_is, dtype=np.float64, copy=True)
    x[:, 0] = x[:, 0] + (steps * dgamma) * x[:, 1]
    d = np.asarray(next_is, dtype=np.float64) - x
    Hinv = np.linalg.inv(H_next)
    s = d @ Hinv.T
    s -= np.rint(s)
    return (s @ H_next.T) / (steps * dgamma)


# ---------------------------------------------------------------------------
# BF16 and the network

def bf16(x) -> np.ndarray:
    """Round FP32 values to the nearest BF16 (ties to even), returned as FP32.
    NaN stays NaN; overflow rounds to infinity as IEEE rounding does."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = x.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).copy()
    nan = np.isnan(x)
    out[nan] = np.float32(np.nan)
    return out


def silu(a):
    return a / (1.0 + np.exp(-a))


def dsilu(a):
    s = 1.0 / (1.0 + np.exp(-a))
    return s * (1.0 + a * (1.0 - s))


@dataclass
class MLP:
    """Weights in the [in, out] layout (FP32 masters or FP64), biases,
    feature and target standardisation."""
    dim: int
    w1: np.ndarray
    b1: np.ndarray
    w2: np.ndarray
    b2: np.ndarray
    w3: np.ndarray
    b3: np.ndarray
    feat_mean: np.ndarray = field(default_factory=lambda: np.zeros(N_FEAT, np.float32))
    feat_std: np.ndarray = field(default_factory=lambda: np.ones(N_FEAT, np.float32))
    tgt_mean: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))
    tgt_std: np.ndarray = field(default_factory=lambda: np.ones(3, np.float32))

    PARAMS = ("w1", "b1", "w2", "b2", "w3", "b3")

    def copy(self) -> "MLP":
        return MLP(self.dim, *[np.array(getattr(self, k), copy=True) for k in
                               self.PARAMS + ("feat_mean", "feat_std", "tgt_mean", "tgt_std")])


def mlp_from_arrays(dim: int, arrays: dict) -> MLP:
    """The network with the given initial parameters (FP32 copies)."""
    return MLP(dim, *[np.array(arrays[k], dtype=np.float32, copy=True) for k in MLP.PARAMS])


def standardise(raw: np.ndarray, m: MLP) -> np.ndarray:
    """z = bf16((fp32(x) - mean) / std), FP32 arithmetic."""
    x = np.asarray(raw).astype(np.float32)
    return bf16((x - m.feat_mean.astype(np.float32)) / m.feat_std.astype(np.float32))


def _mm(a, b):
    """Product of BF16-valued FP32 matrices with an exact (FP64) sum, rounded
    once to FP32: the value an FP32-accumulating matrix core approaches."""
    return (a.astype(np.float64) @ b.astype(np.float64)).astype(np.float32)


def mlp_forward(z: np.ndarray, m: MLP, emulate: bool = True):
    """Network output y (standardised target units) and the activations.

    emulate=True: weights and layer inputs in BF16, sums in FP32, SiLU and
    biases in FP32, hidden activations rounded to BF16 before the next
    layer.  emulate=False: FP64 throughout (finite-difference checks)."""
    if emulate:
        z = bf16(z)
        w1, w2, w3 = bf16(m.w1), bf16(m.w2), bf16(m.w3)
        a1 = _mm(z, w1) + m.b1.astype(np.float32)
        h1 = bf16(silu(a1))
        a2 = _mm(h1, w2) + m.b2.astype(np.float32)
        h2 = bf16(silu(a2))
        y = _mm(h2, w3) + m.b3[:m.dim].astype(np.float32)
    else:
        z = np.asarray(z, np.float64)
        a1 = z @ m.w1.astype(np.float64) + m.b1
        h1 = silu(a1)
        a2 = h1 @ m.w2.astype(np.float64) + m.b2
        h2 = silu(a2)
        y = h2 @ m.w3.astype(np.float64) + m.b3[:m.dim]
    return y, (z, a1, h1, a2, h2)


def huber(e, delta: float):
    ae = np.abs(e)
    return np.where(ae <= delta, 0.5 * e * e, delta * (ae - 0.5 * delta))


def loss_and_grads(z: np.ndarray, t: np.ndarray, m: MLP, delta: float = 1.0,
                   emulate: bool = True, weight=None):
    """Mean Huber loss over samples and components and its gradients with
    respect to (w1, b1, w2, b2, w3, b3), by back-propagation.  weight: 0/1
    per sample (samples of weight 0 add nothing; the mean still divides by
    the batch size).

    emulate=True rounds the back-propagated signals to BF16 where they enter
    a matrix product (the output error, dL/da2, dL/da1), as the GPU's matrix
    cores take them; bias gradients sum the unrounded FP32 signals."""
    y, (zz, a1, h1, a2, h2) = mlp_forward(z, m, emulate)
    B, d = y.shape
    e = y - t
    w = np.ones(B) if weight is None else np.asarray(weight, dtype=np.float64)
    loss = float(np.sum(w[:, None] * huber(e.astype(np.float64), delta)) / (B * d))
    if emulate:
        f32 = np.float32
        g = (np.clip(e, -delta, delta) / f32(B * d)).astype(f32) * w[:, None].astype(f32)
        gb = bf16(g)
        w2b, w3b = bf16(m.w2), bf16(m.w3)
        dw3 = _mm(h2.T, gb)
        db3 = g.astype(np.float64).sum(0).astype(f32)
        dh2 = _mm(gb, w3b.T)
        dz2 = (dh2 * dsilu(a2)).astype(f32)
        dz2b = bf16(dz2)
        dw2 = _mm(h1.T, dz2b)
        db2 = dz2.astype(np.float64).sum(0).astype(f32)
        dh1 = _mm(dz2b, w2b.T)
        dz1 = (dh1 * dsilu(a1)).astype(f32)
        dz1b = bf16(dz1)
        dw1 = _mm(zz.T, dz1b)
        db1 = dz1.astype(np.float64).sum(0).astype(f32)
    else:
        g = np.clip(e, -delta, delta) / (B * d) * w[:, None]
        dw3 = h2.T @ g
        db3 = g.sum(0)
        dh2 = g @ m.w3.astype(np.float64).T
        dz2 = dh2 * dsilu(a2)
        dw2 = h1.T @ dz2
        db2 = dz2.sum(0)
        dh1 = dz2 @ m.w2.astype(np.float64).T
        dz1 = dh1 * dsilu(a1)
        dw1 = zz.T @ dz1
        db1 = dz1.sum(0)
    return loss, {"w1": dw1, "b1": db1, "w2": dw2, "b2": db2, "w3": dw3, "b3": db3}


@dataclass
class AdamState:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: dict = field(default_factory=dict)
    v: dict = field(default_factory=dict)


def adam_step(model: MLP, grads: dict, st: AdamState) -> None:
    """One Adam update (Kingma and Ba, Algorithm 1) of the FP32 masters,
    computed in FP32 as the GPU does."""
    f32 = np.float32
    st.t += 1
    c1 = f32(1.0) - f32(st.beta1) ** f32(st.t)
    c2 = f32(1.0) - f32(st.beta2) ** f32(st.t)
    for k in MLP.PARAMS:
        g = np.asarray(grads[k], dtype=f32)
        w = getattr(model, k)
        if k == "b3":
            g = np.concatenate([g, np.zeros(len(w) - len(g), f32)])
        m = st.m.get(k, np.zeros_like(w, dtype=f32))
        v = st.v.get(k, np.zeros_like(w, dtype=f32))
        m = f32(st.beta1) * m + f32(1.0 - st.beta1) * g
        v = f32(st.beta2) * v + f32(1.0 - st.beta2) * g * g
        mh = m / c1
        vh = v / c2
        setattr(model, k, (w - f32(st.lr) * mh / (np.sqrt(vh) + f32(st.eps))).astype(f32))
        st.m[k], st.v[k] = m, v


def _stats64(x: np.ndarray, mask=None):
    if mask is not None:
        x = x[mask]
    mean = x.mean(0)
    std = np.sqrt(((x - mean) ** 2).mean(0))
    return mean, std


def feature_stats(raw: np.ndarray):
    """Mean and population std per column (FP64 sums, FP32 result); a
    column with zero spread gets std 1."""
    mean, std = _stats64(np.asarray(raw, dtype=np.float64))
    std = np.where(std > 0.0, std, 1.0)
    return mean.astype(np.float32), std.astype(np.float32)


TRIM_KAPPA = 5.0
TRIM_ROUNDS = 3


def target_stats(raw: np.ndarray, kappa: float = TRIM_KAPPA, rounds: int = TRIM_ROUNDS):
    """Trimmed statistics of the targets: mean and std over all samples,
    then `rounds` times over the samples whose every component lies within
    kappa std of the mean (FP64).  The samples outside the last window
    (plastic rearrangements: displacements that no smooth predictor can
    follow) get weight 0 in the loss.  Returns FP32 mean, std and the
    boolean mask of kept samples."""
    x = np.asarray(raw, dtype=np.float64)
    mean, std = _stats64(x)
    mask = np.ones(len(x), dtype=bool)
    for _ in range(rounds):
        mask = np.all(np.abs(x - mean) <= kappa * std, axis=1)
        mean, std = _stats64(x, mask)
    mask = np.all(np.abs(x - mean) <= kappa * std, axis=1)
    std = np.where(std > 0.0, std, 1.0)
    return mean.astype(np.float32), std.astype(np.float32), mask


def train(raw_feat: np.ndarray, raw_tgt: np.ndarray, model: MLP, perms: np.ndarray,
          batch: int = 4096, delta: float = 1.0, adam: AdamState | None = None,
          emulate: bool = True):
    """Fit the network: feature statistics from the whole set, trimmed
    target statistics (``target_stats``; trimmed samples get weight 0),
    then for each epoch e the samples in the order perms[e], cut into
    consecutive batches (the last one may be short), one Adam step per
    batch.  Returns the mean batch loss of every epoch."""
    adam = adam or AdamState()
    model.feat_mean, model.feat_std = feature_stats(raw_feat)
    tm, ts, keep = target_stats(raw_tgt)
    d = model.dim
    model.tgt_mean = np.zeros(3, np.float32)
    model.tgt_std = np.ones(3, np.float32)
    model.tgt_mean[:d], model.tgt_std[:d] = tm, ts
    z_all = standardise(raw_feat, model)
    t_all = ((np.asarray(raw_tgt).astype(np.float32) - tm) / ts).astype(np.float32)
    hist = []
    for p in perms:
        losses = []
        for b0 in range(0, len(p), batch):
            sel = p[b0:b0 + batch]
            loss, g = loss_and_grads(z_all[sel], t_all[sel], model, delta, emulate, keep[sel])
            adam_step(model, g, adam)
            losses.append(loss)
        hist.append(float(np.mean(losses)))
    return hist


def predict(raw_feat: np.ndarray, m: MLP, emulate: bool = True) -> np.ndarray:
    """u_hat per atom (FP32, [n, d]): network output times the target std
    plus the target mean."""
    y, _ = mlp_forward(standardise(raw_feat, m), m, emulate)
    d = m.dim
    return (y * m.tgt_std[:d].astype(np.float32) + m.tgt_mean[:d].astype(np.float32)).astype(np.float32)


# ---------------------------------------------------------------------------
# the learned start

PLAIN, LEARNED, FALLBACK = 0, 1, 2
MAX_LEARNED_MOVE = 0.1  # sigma_AA


def learned_start(is_pos: np.ndarray, u_hat: np.ndarray, dgamma: float):
    """Plain start F r (Eq. 16) and the learned start F r + dgamma (u_hat -
    mean u_hat); ok is False if any u_hat is not finite or some atom would
    move farther than MAX_LEARNED_MOVE."""
    x = np.array(is_pos, dtype=np.float64, copy=True)
    x[:, 0] = x[:, 0] + dgamma * x[:, 1]
    u = np.asarray(u_hat, dtype=np.float64)
    ok = bool(np.all(np.isfinite(u)))
    ok = ok and float(np.max(np.sqrt((u * u).sum(1)))) * dgamma <= MAX_LEARNED_MOVE
    if not ok:
        return x, x.copy(), False
    mean = u.mean(0)
    return x, x + dgamma * (u - mean), True


def extrapolated_uhat(prev_is: np.ndarray, is_pos: np.ndarray, H: np.ndarray,
                      dgamma: float) -> np.ndarray:
    """The extrapolation the paper's conclusion (Sec. 5) proposes: the next
    step's non-affine displacement per unit strain is predicted by the last
    one, u_hat = minimg(r(IS_k) - F r(IS_(k-1))) / dgamma in the box of IS_k.
    The start then follows learned_start / choose_start; the first fine step
    has no history and starts from F r."""
    return nonaffine_targets(prev_is, is_pos, H, dgamma)


def choose_start(plain, learned, ok, types, H, pot, energy_forces):
    """The start FIRE begins from: the learned one unless it was rejected or
    its energy or max |F_i| exceeds the plain start's."""
    if not ok:
        return plain, FALLBACK
    Ep, Fp = energy_forces(plain, types, H, pot)[:2]
    El, Fl = energy_forces(learned, types, H, pot)[:2]
    fp = float(np.sqrt((Fp * Fp).sum(1)).max())
    fl = float(np.sqrt((Fl * Fl).sum(1)).max())
    if El > Ep or fl > fp:
        return plain, FALLBACK
    return learned, LEARNED

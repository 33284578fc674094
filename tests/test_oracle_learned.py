"""Pins of the learned-start oracle (oracle/learned.py) against checks that
do not reuse its code: an explicit image-sum brute force, closed-form
invariants, torch's CPU layers, autograd, Huber loss and Adam, and finite
differences."""
import math

import numpy as np
import pytest
import torch

import aqs_synth as S
import oracle as O
from oracle import learned as Lr

POT = O.kob_andersen()


def brute_descriptors(pos, types, H, pot, rng_images=1):
    """Pure-Python loops over atoms and explicit lattice images H n,
    n in {-1, 0, 1}^d (no minimum-image convention)."""
    n, dim = pos.shape
    feats = np.zeros((n, 64))
    shifts = [np.array(v) for v in np.ndindex(*([2 * rng_images + 1] * dim))]
    mus = [0.6 + b * (1.9 / 23.0) for b in range(24)]
    w = 1.9 / 23.0
    if dim == 2:
        dirs = [(math.cos(2 * math.pi * k / 16), math.sin(2 * math.pi * k / 16)) for k in range(16)]
    else:
        ga = math.pi * (3.0 - math.sqrt(5.0))
        dirs = []
        for k in range(16):
            z = 1.0 - (2 * k + 1) / 16.0
            rho = math.sqrt(1.0 - z * z)
            dirs.append((rho * math.cos(k * ga), rho * math.sin(k * ga), z))
    for i in range(n):
        for j in range(n):
            for sh in shifts:
                img = H @ (sh - rng_images)
                if i == j and not np.any(sh - rng_images):
                    continue
                d = pos[j] + img - pos[i]
                r = math.sqrt(float(d @ d))
                rd = 2.5 * pot.sigma[types[i]][types[j]]
                if r >= rd:
                    continue
                fc = 0.5 * (math.cos(math.pi * r / rd) + 1.0)
                for b, mu in enumerate(mus):
                    feats[i, 24 * types[j] + b] += math.exp(-(r - mu) ** 2 / (2 * w * w)) * fc
                for k, nk in enumerate(dirs):
                    c = sum(nk[q] * d[q] for q in range(dim)) / r
                    feats[i, 48 + k] += fc * max(0.0, c) ** 2
    return feats


@pytest.mark.parametrize("dim,n,L,gamma", [(2, 60, 7.0, 0.3), (3, 40, 6.0, -0.2)])
def test_descriptors_match_image_sum(dim, n, L, gamma):
    rng = S.rng_for(91, dim)
    pos = rng.uniform(0, L, size=(n, dim))
    types = (rng.uniform(size=n) < 0.3).astype(np.int64)
    H = O.box_matrix(dim, L, gamma)
    got = Lr.descriptors(pos, types, H, POT)
    ref = brute_descriptors(pos, types, H, POT)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    assert np.abs(ref).sum() > 10.0  # the systems do have neighbours


def test_angular_features_sum_to_four_fc_in_2d():
    """16 equally spaced directions: for any unit u, sum_k max(0, n_k.u)^2 =
    (1/2) sum_k cos^2 = 4, so the angular features of an atom sum to
    4 sum_j f_c(r_ij)."""
    rng = S.rng_for(92)
    L = 9.0
    pos = rng.uniform(0, L, size=(90, 2))
    types = (rng.uniform(size=90) < 0.35).astype(np.int64)
    H = O.box_matrix(2, L, 0.1)
    f = Lr.descriptors(pos, types, H, POT)
    fcsum = np.zeros(90)
    for i in range(90):
        for j in range(90):
            if i == j:
                continue
            d = pos[j] - pos[i]
            s = np.linalg.solve(H, d)
            s -= np.rint(s)
            r = np.linalg.norm(H @ s)
            rd = 2.5 * POT.sigma[types[i]][types[j]]
            if r < rd:
                fcsum[i] += 0.5 * (math.cos(math.pi * r / rd) + 1.0)
    assert np.allclose(f[:, 48:].sum(1), 4.0 * fcsum, rtol=1e-13, atol=1e-13)


def test_descriptor_invariances():
    """Translation, relabelling and the lattice remap gamma -> gamma + 1
    (the same periodic system) leave the features unchanged."""
    pos, types, L, dim = _glass()
    H = O.box_matrix(dim, L, 0.2)
    f = Lr.descriptors(pos, types, H, POT)
    f_t = Lr.descriptors(pos + np.array([0.37, -1.21]), types, H, POT)
    perm = S.rng_for(93).permutation(len(types))
    f_p = Lr.descriptors(pos[perm], types[perm], H, POT)
    f_r = Lr.descriptors(pos, types, O.box_matrix(dim, L, 1.2), POT)
    assert np.abs(f_t - f).max() < 1e-11
    assert np.abs(f_p - f[perm]).max() < 1e-12
    assert np.abs(f_r - f).max() < 1e-11


def _glass():
    from gpu_common import load_glass
    return load_glass("glass2d_256")


def test_bf16_rounding_matches_torch():
    rng = S.rng_for(94)
    x = np.concatenate([rng.normal(size=4000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 4000),
                        np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -1.0 - 2.0 ** -8, 3.4e38, -3.4e38,
                                  1e-40, -1e-42, 0.0, -0.0, np.inf, -np.inf], dtype=np.float32)])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = Lr.bf16(x)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert np.isnan(Lr.bf16(np.array([np.nan], np.float32)))[0]


def _model(dim=3, seed=5):
    return Lr.mlp_from_arrays(dim, S.mlp_init(dim, 95, seed))


def _torch_forward(z, m):
    t = lambda a: torch.from_numpy(np.asarray(a, np.float64))
    h = torch.nn.functional.silu(torch.nn.functional.linear(t(z), t(m.w1).T, t(m.b1)))
    h = torch.nn.functional.silu(torch.nn.functional.linear(h, t(m.w2).T, t(m.b2)))
    return torch.nn.functional.linear(h, t(m.w3).T, t(m.b3[:m.dim]))


def test_fp64_forward_matches_torch_layers():
    m = _model()
    z = S.rng_for(96).normal(size=(50, 64))
    y, _ = Lr.mlp_forward(z, m, emulate=False)
    assert np.allclose(y, _torch_forward(z, m).numpy(), rtol=1e-13, atol=1e-13)


def test_bf16_forward_is_close_to_fp64():
    m = _model()
    z = Lr.bf16(S.rng_for(97).normal(size=(200, 64)).astype(np.float32))
    y16, _ = Lr.mlp_forward(z, m, emulate=True)
    y64, _ = Lr.mlp_forward(z.astype(np.float64), m, emulate=False)
    assert np.abs(y16 - y64).max() < 2e-2 * np.abs(y64).max()
    assert np.abs(y16 - y64).max() > 0.0   # the rounding is really applied


def test_fp64_gradients_match_autograd_and_finite_differences():
    m = _model(dim=2)
    rng = S.rng_for(98)
    z = rng.normal(size=(40, 64))
    t = 2.0 * rng.normal(size=(40, 2))   # some errors beyond the Huber delta
    loss, g = Lr.loss_and_grads(z, t, m, delta=1.0, emulate=False)
    tw = {k: torch.tensor(np.asarray(getattr(m, k), np.float64), requires_grad=True) for k in Lr.MLP.PARAMS}
    zz = torch.from_numpy(z)
    h = torch.nn.functional.silu(zz @ tw["w1"] + tw["b1"])
    h = torch.nn.functional.silu(h @ tw["w2"] + tw["b2"])
    y = h @ tw["w3"] + tw["b3"]
    tl = torch.nn.functional.huber_loss(y, torch.from_numpy(t), reduction="mean", delta=1.0)
    tl.backward()
    assert abs(loss - tl.item()) < 1e-14
    for k in Lr.MLP.PARAMS:
        assert np.allclose(g[k], tw[k].grad.numpy(), rtol=1e-11, atol=1e-15), k
    # central differences on a few entries of every parameter
    for k in Lr.MLP.PARAMS:
        w = getattr(m, k).astype(np.float64)
        setattr(m, k, w)
        flat = w.reshape(-1)
        for q in S.rng_for(99, len(flat)).choice(len(flat), min(3, len(flat)), replace=False):
            h = 1e-6
            old = flat[q]
            flat[q] = old + h
            lp, _ = Lr.loss_and_grads(z, t, m, 1.0, emulate=False)
            flat[q] = old - h
            lm, _ = Lr.loss_and_grads(z, t, m, 1.0, emulate=False)
            flat[q] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - np.asarray(g[k]).reshape(-1)[q]) <= 1e-6 * max(1e-6, abs(fd)) + 1e-10, (k, q)


def test_bf16_gradients_are_close_to_fp64():
    m = _model(dim=3)
    rng = S.rng_for(100)
    z = Lr.bf16(rng.normal(size=(512, 64)).astype(np.float32))
    t = rng.normal(size=(512, 3)).astype(np.float32)
    _, g16 = Lr.loss_and_grads(z, t, m, 1.0, emulate=True)
    _, g64 = Lr.loss_and_grads(z.astype(np.float64), t.astype(np.float64), m, 1.0, emulate=False)
    for k in Lr.MLP.PARAMS:
        rel = np.linalg.norm(g16[k] - g64[k]) / np.linalg.norm(g64[k])
        assert rel < 3e-2, (k, rel)


def test_adam_matches_torch():
    m = _model(dim=2)
    rng = S.rng_for(101)
    st = Lr.AdamState(lr=1e-3)
    tw = [torch.tensor(getattr(m, k).copy(), requires_grad=True) for k in Lr.MLP.PARAMS]
    opt = torch.optim.Adam(tw, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(4):
        grads = {k: rng.normal(size=getattr(m, k).shape).astype(np.float32) * 1e-3 for k in Lr.MLP.PARAMS}
        Lr.adam_step(m, grads, st)
        for p, k in zip(tw, Lr.MLP.PARAMS):
            p.grad = torch.from_numpy(grads[k])
        opt.step()
    for p, k in zip(tw, Lr.MLP.PARAMS):
        assert np.allclose(getattr(m, k), p.detach().numpy(), rtol=1e-6, atol=1e-7), k


def test_training_fits_a_learnable_target():
    """Targets that are a smooth function of the features: the loss falls
    by an order of magnitude within a few epochs."""
    rng = S.rng_for(102)
    n = 3000
    x = rng.normal(size=(n, 64)) * 3.0 + 1.0
    A = rng.normal(size=(64, 2)) / 8.0
    y = np.tanh(x @ A) * 5.0 + 2.0
    m = _model(dim=2)
    hist = Lr.train(x, y, m, S.epoch_orders(n, 12, 103), batch=256, adam=Lr.AdamState(lr=3e-3))
    assert hist[-1] < 0.1 * hist[0]
    u = Lr.predict(x[:500], m)
    assert np.sqrt(np.mean((u - y[:500]) ** 2)) < 0.3 * y.std()


def test_targets_recover_a_planted_displacement():
    pos, types, L, dim = _glass()
    dg = 1e-3
    H1 = O.strain_box(dim, L, 1, dg)
    u = S.rng_for(104).normal(size=pos.shape) * 1e-4
    nxt = O.affine(pos, dg) + u
    nxt[::7, 0] += L    # a whole box vector changes nothing
    got = Lr.nonaffine_targets(pos, nxt, H1, dg)
    assert np.abs(got * dg - u).max() < 1e-12


def test_learned_start_rules():
    pos, types, L, dim = _glass()
    dg = 1e-4
    n = len(types)
    plain, learned, ok = Lr.learned_start(pos, np.full((n, 2), 3.25, np.float32), dg)
    assert ok and np.array_equal(plain, learned)            # a uniform u_hat is no move
    assert np.array_equal(plain, O.affine(pos, dg))
    uh = S.rng_for(105).normal(size=(n, 2)).astype(np.float32)
    _, learned, ok = Lr.learned_start(pos, uh, dg)
    assert ok and np.abs((learned - plain).sum(0)).max() < 1e-15 * n   # no net translation
    bad = uh.copy()
    bad[3, 1] = np.nan
    assert not Lr.learned_start(pos, bad, dg)[2]
    big = uh.copy()
    big[5] = [0.11 / dg, 0.0]
    assert not Lr.learned_start(pos, big, dg)[2]
    H = O.strain_box(dim, L, 1, dg)
    # the start picked is never worse than the plain one in E and max |F_i|
    x, which = Lr.choose_start(plain, learned, True, types, H, POT, O.energy_forces)
    Ep, Fp = O.energy_forces(plain, types, H, POT)[:2]
    Ex, Fx = O.energy_forces(x, types, H, POT)[:2]
    assert Ex <= Ep and np.sqrt((Fx ** 2).sum(1)).max() <= np.sqrt((Fp ** 2).sum(1)).max()
    assert which in (Lr.LEARNED, Lr.FALLBACK)


def test_extrapolated_start_continues_a_planted_displacement():
    """r(IS_k) = F r(IS_(k-1)) + u: the extrapolated start of step k + 1 is
    F r(IS_k) + (u - mean u), whatever box vectors the atoms were wrapped
    by; a purely affine step predicts no displacement (start = F r)."""
    pos, types, L, dim = _glass()
    dg = 1e-4
    H1 = O.strain_box(dim, L, 1, dg)
    u = S.rng_for(107).normal(size=pos.shape) * 2e-4 + np.array([3e-5, -1e-5])
    is1 = O.affine(pos, dg) + u
    is1[::5, 0] -= L
    uh = Lr.extrapolated_uhat(pos, is1, H1, dg)
    plain, start, ok = Lr.learned_start(is1, uh, dg)
    assert ok
    assert np.abs(start - (O.affine(is1, dg) + (u - u.mean(0)))).max() < 1e-12
    uh0 = Lr.extrapolated_uhat(pos, O.affine(pos, dg), H1, dg)
    assert np.array_equal(uh0, np.zeros_like(uh0))
    plain, start, ok = Lr.learned_start(O.affine(pos, dg), uh0, dg)
    assert ok and np.array_equal(start, plain)


def test_extrapolated_starts_keep_the_plain_inherent_structures():
    """A short chain at small strain steps: starting each minimisation from
    the extrapolated start reaches the plain chain's inherent structures
    (Eq. 20) with fewer FIRE iterations in total."""
    pos, types, L, dim = _glass()
    dg, nst = 1e-5, 5
    fp = O.FireParams(dt0=0.01, dt_max=0.03, dt_min=2e-4, f_inc=1.2, f_dec=0.9, alpha0=0.2, f_alpha=0.95,
                      n_delay=5)
    x_p, x_e, prev = pos, pos, None
    it_p = it_e = 0
    for k in range(1, nst + 1):
        H = O.strain_box(dim, L, k, dg)
        rp = O.fire(O.affine(x_p, dg), types, H, POT, fp)
        if prev is None:
            x0 = O.affine(x_e, dg)
        else:
            uh = Lr.extrapolated_uhat(prev, x_e, O.strain_box(dim, L, k - 1, dg), dg)
            plain, start, ok = Lr.learned_start(x_e, uh, dg)
            x0, _ = Lr.choose_start(plain, start, ok, types, H, POT, O.energy_forces)
        re_ = O.fire(x0, types, H, POT, fp)
        assert rp.status == re_.status == O.CONVERGED
        assert O.compare(rp.pos, re_.pos, H)[0] < 1e-6
        it_p += rp.iters
        it_e += re_.iters
        prev, x_p, x_e = x_e, rp.pos, re_.pos
    assert it_e < it_p


def test_trimmed_target_statistics_drop_plastic_outliers():
    """Gaussian targets plus a few huge jumps: the trimmed statistics are
    those of the Gaussian part and exactly the jumps are left out."""
    rng = S.rng_for(106)
    t = rng.normal(size=(20000, 3)) * np.array([2.0, 0.5, 1.0]) + np.array([0.3, -1.0, 0.0])
    jumps = rng.choice(20000, 25, replace=False)
    t[jumps] += rng.choice([-1, 1], size=(25, 3)) * 4000.0
    mean, std, keep = Lr.target_stats(t)
    assert set(np.nonzero(~keep)[0]) == set(jumps)
    assert np.allclose(mean, [0.3, -1.0, 0.0], atol=0.05)
    assert np.allclose(std, [2.0, 0.5, 1.0], rtol=0.03)
    full = Lr.feature_stats(t)[1]
    assert np.all(full > 50 * std)   # the untrimmed std is useless

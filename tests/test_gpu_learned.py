"""GPU parity of the learned start (descriptors, BF16 network inference and
training, non-affine targets, the learned start inside the device chain)
against the CPU oracle (oracle/learned.py), through the C ABI."""
import numpy as np
import pytest

import aqs_synth as S
import oracle as O
from oracle import learned as Lr
from gpu_common import E_REL_TOL, fire_pair, load_glass

pytestmark = pytest.mark.gpu
POT = O.kob_andersen()


def _torch():
    import torch
    return torch


def engine(dim, ns, L, dg, **kw):
    from paper_2507_20802_amd import Engine
    return Engine(dim, ns, L, dg, **kw)


def oracle_model(dim, raw_feat, raw_tgt, seed=3):
    """A seeded network with the oracle's standardisation of the given data."""
    m = Lr.mlp_from_arrays(dim, S.mlp_init(dim, 300, seed))
    m.feat_mean, m.feat_std = Lr.feature_stats(raw_feat)
    tm, ts = Lr.feature_stats(raw_tgt)
    m.tgt_mean = np.zeros(3, np.float32)
    m.tgt_std = np.ones(3, np.float32)
    m.tgt_mean[:dim], m.tgt_std[:dim] = tm, ts
    return m


def to_c(m):
    from paper_2507_20802_amd import learned
    return learned.make_mlp(m.dim, {k: getattr(m, k) for k in Lr.MLP.PARAMS}, m.feat_mean, m.feat_std,
                            m.tgt_mean[:m.dim], m.tgt_std[:m.dim])


@pytest.mark.parametrize("name,k,dg", [("glass2d_1000", 3, 1e-3), ("glass3d_1500", 2, 5e-3)])
def test_descriptors_match_oracle(name, k, dg):
    pos, types, L, dim = load_glass(name)
    x = O.affine(pos, k * dg)
    eng = engine(dim, [len(types)], L, dg)
    eng.set_replica(0, types, x, k)
    got = eng.learned_features(0).cpu().numpy()
    ref = Lr.descriptors(x, types, O.strain_box(dim, L, k, dg), POT)
    assert np.abs(got - ref.astype(np.float32)).max() <= 3e-7 * max(1.0, np.abs(ref).max())
    assert ref[:, :48].sum() > 0 and ref[:, 48:].sum() > 0


def test_descriptors_at_full_size_sampled():
    """3D, 32768 atoms (the benchmark's size), strained box: 256 sampled atoms."""
    s = S.uniform_glass_start(3, 32768, 3, 0)
    dg, k = 5e-5, 120
    x = O.affine(s.pos, k * dg)
    eng = engine(3, [32768], s.L, dg)
    eng.set_replica(0, s.types, x, k)
    got = eng.learned_features(0).cpu().numpy()
    idx = S.rng_for(301).choice(32768, 256, replace=False)
    ref = Lr.descriptors(x, s.types, O.strain_box(3, s.L, k, dg), POT, idx=idx)
    assert np.abs(got[idx] - ref.astype(np.float32)).max() <= 3e-7 * max(1.0, np.abs(ref).max())


def test_targets_match_oracle():
    pos, types, L, dim = load_glass("glass2d_1000")
    dg = 1e-4
    fire, ofire = fire_pair()
    eng = engine(dim, [len(types)] * 2, L, dg, fire=fire)
    eng.set_replica(0, types, pos, 0)
    eng.copy_replica(0, 1)
    eng.minimize([1], n_steps=[2])
    got = eng.learned_targets(0, 1).cpu().numpy()
    nxt = eng.positions(1)
    ref = Lr.nonaffine_targets(pos, nxt, O.strain_box(dim, L, 2, dg), dg, steps=2)
    assert np.abs(got - ref.astype(np.float32)).max() <= 1e-6 * max(1.0, np.abs(ref).max())
    assert np.abs(ref).max() > 1.0     # a real non-affine field


@pytest.mark.parametrize("name", ["glass2d_1000", "glass3d_1500"])
def test_inference_matches_bf16_oracle(name):
    pos, types, L, dim = load_glass(name)
    eng = engine(dim, [len(types)], L, 1e-4)
    eng.set_replica(0, types, pos, 0)
    raw = Lr.descriptors(pos, types, O.strain_box(dim, L, 0, 1e-4), POT)
    tgt = S.rng_for(302).normal(size=(len(types), dim)) * 3.0 + 0.5
    m = oracle_model(dim, raw, tgt)
    eng.learned_load(to_c(m))
    got = eng.learned_predict(0).cpu().numpy()
    ref = Lr.predict(raw, m, emulate=True)
    scale = np.abs(ref).max()
    err = np.abs(got - ref)
    print("inference max err / scale", err.max() / scale, "median", np.median(err) / scale)
    # sums in another order can round a hidden activation to the neighbouring
    # BF16 value (2^-8 relative) now and then; measured 1.2e-4 to 2.4e-4
    assert err.max() <= 1e-3 * scale
    assert np.median(err) <= 1e-5 * scale


def _train_set(dim, n, seed):
    rng = S.rng_for(303, seed)
    x = np.abs(rng.normal(size=(n, 64))) * 2.0
    y = np.tanh(x[:, :dim] - x[:, dim:2 * dim]) * 3.0 + 0.2 * rng.normal(size=(n, dim))
    return x.astype(np.float32), y.astype(np.float32)


@pytest.mark.parametrize("dim,n", [(2, 1000), (3, 4096), (3, 77)])
def test_gradients_match_bf16_oracle(dim, n):
    from paper_2507_20802_amd import learned
    torch = _torch()
    x, y = _train_set(dim, n, dim)
    m = oracle_model(dim, x, y, seed=dim)
    z = Lr.standardise(x, m)
    t = ((y - m.tgt_mean[:dim]) / m.tgt_std[:dim]).astype(np.float32)
    loss_ref, g_ref = Lr.loss_and_grads(z, t, m, 1.0, emulate=True)
    loss, g = learned.gradients(to_c(m), torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), 1.0)
    assert abs(loss - loss_ref) <= 1e-5 * abs(loss_ref)
    for k in Lr.MLP.PARAMS:
        rel = np.linalg.norm(g[k] - g_ref[k]) / np.linalg.norm(g_ref[k])
        # element by element, against the largest gradient of the parameter
        elem = np.abs(g[k] - g_ref[k]).max() / np.abs(g_ref[k]).max()
        print(k, "norm", rel, "element", elem)
        assert rel <= 1e-3, (k, rel)
        assert elem <= 1e-3, (k, elem)


def test_training_steps_match_oracle():
    """Three Adam steps (one epoch, batch 1024 of 2500 samples: the last
    batch short) from the same initial weights and sample order."""
    from paper_2507_20802_amd import learned
    torch = _torch()
    dim, n = 2, 2500
    x, y = _train_set(dim, n, 7)
    y[::97] += 500.0    # plastic jumps: trimmed out of the statistics and the loss
    init = S.mlp_init(dim, 304)
    orders = S.epoch_orders(n, 1, 305)
    m = Lr.mlp_from_arrays(dim, init)
    hist_ref = Lr.train(x, y, m, orders, batch=1024, adam=Lr.AdamState(lr=1e-3))
    cm = learned.make_mlp(dim, init)
    hist = learned.train(cm, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(),
                         torch.from_numpy(orders).cuda(), learned.TrainParams(batch=1024, epochs=1))
    got = learned.mlp_arrays(cm)
    assert np.allclose(got["feat_mean"], m.feat_mean, rtol=1e-6, atol=1e-7)
    assert np.allclose(got["feat_std"], m.feat_std, rtol=1e-6)
    assert np.allclose(got["tgt_mean"], m.tgt_mean[:dim], rtol=1e-6, atol=1e-7)
    assert np.allclose(got["tgt_std"], m.tgt_std[:dim], rtol=1e-6)
    assert np.all(m.tgt_std[:dim] < 10.0)   # the jumps are out of the statistics
    assert abs(hist[0] - hist_ref[0]) <= 1e-4 * abs(hist_ref[0])
    for k in Lr.MLP.PARAMS:
        d = np.abs(got[k] - getattr(m, k))
        print(k, "max", d.max(), "share > 1e-6", np.mean(d > 1e-6), "share > 1e-5", np.mean(d > 1e-5))
        # Adam moves every weight by about lr per step; rounding can only flip
        # the sign of steps whose gradient is at the rounding level
        assert d.max() <= 6.1e-3, (k, d.max())
        assert np.mean(d > 1e-6) < 0.02, (k, np.mean(d > 1e-6))


def test_training_learns_and_is_deterministic():
    from paper_2507_20802_amd import learned
    torch = _torch()
    dim, n = 3, 20000
    x, y = _train_set(dim, n, 9)
    orders = torch.from_numpy(S.epoch_orders(n, 8, 306)).cuda()
    xs, ys = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    m1 = learned.make_mlp(dim, S.mlp_init(dim, 307))
    m2 = learned.make_mlp(dim, S.mlp_init(dim, 307))
    p = learned.TrainParams(batch=2048, epochs=8, lr=3e-3)
    h1 = learned.train(m1, xs, ys, orders, p)
    h2 = learned.train(m2, xs, ys, orders, p)
    assert np.array_equal(h1, h2)
    a1, a2 = learned.mlp_arrays(m1), learned.mlp_arrays(m2)
    assert all(np.array_equal(a1[k], a2[k]) for k in a1)
    assert h1[-1] < 0.3 * h1[0]


def _trained_model(dim, L, types, pos, dg, steps, epochs=30):
    """Network trained on `steps` plain AQS steps of the given glass."""
    from paper_2507_20802_amd import learned
    torch = _torch()
    fire, _ = fire_pair()
    eng = engine(dim, [len(types)] * 2, L, dg, fire=fire)
    eng.set_replica(0, types, pos, 0)
    feat, tgt, _ = learned.collect_samples(eng, 0, 1, steps)
    n = feat.shape[0]
    orders = torch.from_numpy(S.epoch_orders(n, epochs, 308)).cuda()
    m = learned.make_mlp(dim, S.mlp_init(dim, 309))
    hist = learned.train(m, feat, tgt, orders, learned.TrainParams(batch=1024, epochs=epochs))
    return m, hist


def test_learned_chain_reaches_the_plain_inherent_structures():
    """Fine AQS steps with the learned start on the device: every step ends
    in the oracle's plain-start inherent structure (Eq. 20 with delta_eq =
    1e-4, energy to 1e-10), whatever start was used."""
    pos_tr, types_tr, L, dim = load_glass("glass2d_1000")
    dg, nst = 1e-4, 6
    m, hist = _trained_model(dim, L, types_tr, pos_tr, dg, 12, epochs=20)
    assert hist[-1] < hist[0]
    pos, types, L2, _ = load_glass("glass2d_256")
    fire, ofire = fire_pair()
    from paper_2507_20802_amd import AQS_START_LEARNED
    eng = engine(dim, [len(types)], L2, dg, fire=fire)
    eng.learned_load(m)
    eng.set_replica(0, types, pos, 0)
    recs = eng.minimize([0], n_steps=[nst], start=AQS_START_LEARNED)[0]
    x = pos
    starts = []
    for k in range(1, nst + 1):
        H = O.strain_box(dim, L2, k, dg)
        r = O.fire(O.affine(x, dg), types, H, POT, ofire)
        x = r.pos
        assert recs[k]["status"] == 0
        assert abs(recs[k]["energy"] - r.E) <= E_REL_TOL * abs(r.E)
        starts.append(int(recs[k]["start"]))
    assert O.compare(eng.positions(0), x, O.strain_box(dim, L2, nst, dg))[0] < 1e-4
    assert set(starts) <= {1, 2}
    print("starts", starts, "iters", recs["iters"].tolist())


def test_learned_start_gain_on_its_own_history():
    """What the trained network gains over the method without it: trained on
    the non-affine displacements of 24 plain AQS steps of a glass (small
    elastic steps, dgamma = 1e-5), it starts the next 8 steps.  Every step
    reaches the plain start's inherent structure (Eq. 20, energies to
    1e-10), and the learned starts take fewer FIRE iterations in total."""
    from paper_2507_20802_amd import AQS_START_LEARNED, AQS_START_PLAIN, learned
    torch = _torch()
    pos, types, L, dim = load_glass("glass2d_256")
    fire, _ = fire_pair()
    # 200 epochs: the start must beat the plain one in max |F_i| too, which
    # needs the fit of the displacement field to be nearly exact (after 60
    # epochs R^2 = 0.994 on the next step, and one atom's force still
    # exceeds the plain start's)
    dg, hist_steps, nst, epochs = 1e-5, 24, 8, 200
    eng = engine(dim, [len(types)] * 2, L, dg, fire=fire)
    eng.set_replica(0, types, pos, 0)
    feat, tgt, _ = learned.collect_samples(eng, 0, 1, hist_steps)
    start_is = eng.positions(0)
    orders = torch.from_numpy(S.epoch_orders(feat.shape[0], epochs, 310)).cuda()
    m = learned.make_mlp(dim, S.mlp_init(dim, 311))
    loss = learned.train(m, feat, tgt, orders, learned.TrainParams(batch=256, epochs=epochs))
    assert loss[-1] < 0.01 * loss[0]
    out = {}
    for mode in (AQS_START_PLAIN, AQS_START_LEARNED):
        e = engine(dim, [len(types)], L, dg, fire=fire)
        if mode == AQS_START_LEARNED:
            e.learned_load(m)
        e.set_replica(0, types, start_is, hist_steps)
        rec = e.minimize([0], n_steps=[nst], start=mode)[0]
        assert np.all(rec["status"] == 0)
        out[mode] = (rec, e.positions(0))
    rp, xp = out[AQS_START_PLAIN]
    rl, xl = out[AQS_START_LEARNED]
    assert np.allclose(rl["energy"], rp["energy"], rtol=E_REL_TOL, atol=0)
    assert O.compare(xl, xp, O.strain_box(dim, L, hist_steps + nst, dg))[0] < 1e-6
    it_p, it_l = int(rp["iters"][1:].sum()), int(rl["iters"][1:].sum())
    used = int((rl["start"][1:] == 1).sum())
    print(f"loss {loss[0]:.3g} -> {loss[-1]:.3g}; FIRE iterations plain {it_p} learned {it_l}; "
          f"learned starts used {used}/{nst}")
    assert used >= 1 and it_l < it_p


def _oracle_learned_chain(pos, types, L, dim, dg, k0, nst, m, ofire):
    """The learned start in the oracle from the inherent structure pos at
    strain index k0: at every inherent structure the descriptors and the
    BF16-emulating network predict u_hat, the start follows learned_start /
    choose_start, FIRE minimises.  Returns per step (E, start code, IS)."""
    out, x = [], pos
    for k in range(k0 + 1, k0 + nst + 1):
        H = O.strain_box(dim, L, k, dg)
        raw = Lr.descriptors(x, types, O.strain_box(dim, L, k - 1, dg), POT)
        uh = Lr.predict(raw, m, emulate=True)
        plain, start, ok = Lr.learned_start(x, uh, dg)
        x0, which = Lr.choose_start(plain, start, ok, types, H, POT, O.energy_forces)
        r = O.fire(x0, types, H, POT, ofire)
        assert r.status == O.CONVERGED
        out.append((r.E, which, r.pos))
        x = r.pos
    return out


def _oracle_mlp(arrays, dim):
    m = Lr.mlp_from_arrays(dim, {k: arrays[k] for k in Lr.MLP.PARAMS})
    m.feat_mean, m.feat_std = arrays["feat_mean"], arrays["feat_std"]
    m.tgt_mean = np.zeros(3, np.float32)
    m.tgt_std = np.ones(3, np.float32)
    m.tgt_mean[:dim], m.tgt_std[:dim] = arrays["tgt_mean"], arrays["tgt_std"]
    return m


def test_learned_chain_matches_the_oracle():
    """The network trained on the GPU (on 24 plain steps of the glass's
    history) starts 6 fine steps on the device and in the oracle (same
    weights, the oracle's own BF16-emulating predictions): the same start
    decision at every step (learned or fallback, choose_start's rule),
    energies within 1e-10 relative and the final configuration within
    1e-8 sigma, certified by the oracle's forces."""
    from paper_2507_20802_amd import AQS_START_FALLBACK, AQS_START_LEARNED, learned
    from gpu_common import FTOL, POS_TOL, certified_fmax
    torch = _torch()
    pos, types, L, dim = load_glass("glass2d_256")
    fire, ofire = fire_pair()
    dg, hist_steps, nst, epochs = 1e-5, 24, 6, 200
    eng = engine(dim, [len(types)] * 2, L, dg, fire=fire)
    eng.set_replica(0, types, pos, 0)
    feat, tgt, _ = learned.collect_samples(eng, 0, 1, hist_steps)
    start_is = eng.positions(0)
    orders = torch.from_numpy(S.epoch_orders(feat.shape[0], epochs, 310)).cuda()
    cm = learned.make_mlp(dim, S.mlp_init(dim, 311))
    learned.train(cm, feat, tgt, orders, learned.TrainParams(batch=256, epochs=epochs))
    m = _oracle_mlp(learned.mlp_arrays(cm), dim)
    # both sides continue from the history's last inherent structure
    ref = _oracle_learned_chain(start_is, types, L, dim, dg, hist_steps, nst, m, ofire)
    e = engine(dim, [len(types)], L, dg, fire=fire)
    e.learned_load(cm)
    e.set_replica(0, types, start_is, hist_steps)
    rec = e.minimize([0], n_steps=[nst], start=AQS_START_LEARNED)[0]
    codes = []
    for k in range(1, nst + 1):
        E, which, _ = ref[k - 1]
        want = AQS_START_LEARNED if which == Lr.LEARNED else AQS_START_FALLBACK
        codes.append(int(rec[k]["start"]))
        assert rec[k]["status"] == 0
        assert rec[k]["start"] == want, (k, rec[k]["start"], want)
        assert abs(rec[k]["energy"] - E) <= E_REL_TOL * abs(E)
    H = O.strain_box(dim, L, hist_steps + nst, dg)
    got = e.positions(0)
    print("start codes", codes, "final distance", O.compare(got, ref[-1][2], H)[0])
    assert O.compare(got, ref[-1][2], H)[0] <= POS_TOL
    assert certified_fmax(got, types, H) < FTOL
    assert AQS_START_LEARNED in codes


def test_broken_network_falls_back_bit_for_bit():
    """A network whose weights are not finite predicts non-finite
    displacements: every fine step falls back to the plain start (record
    AQS_START_FALLBACK), and the chain is the plain chain bit for bit --
    the same iterations, energies and final positions."""
    from paper_2507_20802_amd import AQS_START_FALLBACK, AQS_START_LEARNED, AQS_START_PLAIN, learned
    pos, types, L, dim = load_glass("glass2d_256")
    fire, _ = fire_pair()
    dg, nst = 1e-4, 4
    arrays = S.mlp_init(dim, 312)
    arrays["w2"] = arrays["w2"].copy()
    arrays["w2"][3, 5] = np.nan
    bad = learned.make_mlp(dim, arrays)
    out = {}
    for mode in (AQS_START_PLAIN, AQS_START_LEARNED):
        e = engine(dim, [len(types)], L, dg, fire=fire)
        if mode == AQS_START_LEARNED:
            e.learned_load(bad)
        e.set_replica(0, types, pos, 0)
        out[mode] = (e.minimize([0], n_steps=[nst], start=mode)[0], e.positions(0))
    rp, xp = out[AQS_START_PLAIN]
    rl, xl = out[AQS_START_LEARNED]
    assert np.all(rl["start"][1:] == AQS_START_FALLBACK)
    assert np.array_equal(rl["iters"], rp["iters"])
    assert np.array_equal(rl["energy"], rp["energy"])
    assert np.array_equal(xl, xp)

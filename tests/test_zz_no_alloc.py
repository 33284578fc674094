"""The training entry point without device allocation (aqs_mlp_train_static)
against aqs_mlp_train, through the C ABI: the same trained weights,
standardisation and loss history bit for bit, on two calls in a row (the
second with fewer samples, another output dimension and smaller batches, so
stale contents of the shared device array would show), and the capacity
errors before anything runs."""
import ctypes

import numpy as np
import pytest

import aqs_synth as S

pytestmark = pytest.mark.gpu


def _case(n, dim, epochs, seed):
    import torch
    rng = S.rng_for(2507, 20802, 77, seed)
    feat = rng.normal(0.0, 1.0, size=(n, 64)) * rng.uniform(0.1, 3.0, size=64) + rng.normal(0, 2, size=64)
    tgt = rng.normal(0.0, 1.0, size=(n, dim)) + 0.3 * feat[:, :dim]
    # a few plastic-jump-like outliers, which the trimmed statistics leave out
    jump = rng.choice(n, size=max(1, n // 500), replace=False)
    tgt[jump] *= 200.0
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(feat.astype(np.float32)).to(dev),
            torch.from_numpy(tgt.astype(np.float32)).to(dev),
            torch.from_numpy(S.epoch_orders(n, epochs, 77, seed)).to(dev))


def _train(static, dim, feat, tgt, orders, batch, seed):
    from paper_2507_20802_amd import learned
    model = learned.make_mlp(dim, S.mlp_init(dim, 77, seed))
    hist = learned.train(model, feat, tgt, orders,
                         learned.TrainParams(batch=batch, epochs=int(orders.shape[0])), static=static)
    return learned.mlp_arrays(model), hist


def test_static_training_equals_allocating_training_on_two_calls():
    import torch
    torch.cuda.set_device(0)
    # (samples, outputs, epochs, batch): the second call is smaller
    for n, dim, epochs, batch in ((40000, 3, 3, 4096), (7000, 2, 2, 1024)):
        feat, tgt, orders = _case(n, dim, epochs, n)
        want, hw = _train(False, dim, feat, tgt, orders, batch, n)
        got, hg = _train(True, dim, feat, tgt, orders, batch, n)
        print(f"n {n} dim {dim}: loss {hw[0]:.4f} -> {hw[-1]:.4f}")
        assert np.isfinite(hw).all() and hw[-1] < hw[0]
        assert np.array_equal(hg, hw)
        for k in want:
            assert want[k].shape == got[k].shape, k
            assert np.array_equal(got[k], want[k]), k


def test_static_training_refuses_sizes_beyond_its_array():
    from paper_2507_20802_amd import _lib, learned
    from paper_2507_20802_amd._lib import AQS_ECAPACITY
    lib = _lib.load()
    model = learned.make_mlp(3, S.mlp_init(3, 77, 1))
    before = learned.mlp_arrays(model)
    dummy = ctypes.c_void_p(16)   # never dereferenced: the sizes are refused first
    hist = np.zeros(8, np.float32)
    for n, batch, epochs in ((65537, 4096, 1), (65536, 8192, 1), (1000, 512, 4097)):
        cp = learned.TrainParams(batch=batch, epochs=epochs).to_c()
        rc = lib.aqs_mlp_train_static(ctypes.byref(cp), n, dummy, dummy, dummy, ctypes.byref(model),
                                      hist.ctypes.data_as(_lib.c_float_p), None)
        print(n, batch, epochs, rc, lib.aqs_last_error().decode())
        assert rc == AQS_ECAPACITY
    after = learned.mlp_arrays(model)
    assert all(np.array_equal(before[k], after[k]) for k in before)

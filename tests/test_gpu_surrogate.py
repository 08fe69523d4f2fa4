"""GPU: the surrogate's hand-written training kernels against the FP64
oracle (forward, loss and every parameter gradient), reproducibility, and
the ensemble fallback rule."""

import sys

import numpy as np
import pytest

from oracle import surrogate as sg

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dgd():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1907_06191_amd import dgd as d
    return d


def _data(n, seed):
    rng = np.random.default_rng(seed)
    imgs = (rng.random((n, 64, 64)) < rng.uniform(0.2, 0.6, (n, 1, 1))).astype(np.uint8)
    ld = rng.uniform(0.0, np.log(50.0), n)
    occ = imgs.reshape(n, -1).mean(1)
    tg = np.stack([1 - 0.8 * occ * np.tanh(ld), 0.01 * (occ - 0.4), 1 - 0.7 * occ * np.tanh(ld)], 1)
    return imgs, ld, tg


@pytest.mark.parametrize("C,H", [(32, 256), (8, 24)])
def test_loss_and_gradient_match_oracle(dgd, C, H):
    say(f"surrogate gradient parity C={C} H={H}")
    s = dgd.dgd_surrogate_create(1, C, H, 11)
    try:
        # perturb the biases away from zero so every gradient is exercised
        p = dgd.dgd_surrogate_get_params(s, 0)
        p = p + np.random.default_rng(3).normal(0, 0.02, p.size).astype(np.float32)
        dgd.dgd_surrogate_set_params(s, 0, p)
        imgs, ld, tg = _data(6, 5)
        loss, g = dgd.dgd_surrogate_loss_grad(s, 0, imgs, ld, tg)
        lref, gref = sg.loss_and_grad(p.astype(np.float64), imgs.astype(float), ld, tg, C, H)
        rel = np.abs(g - gref).max() / np.abs(gref).max()
        say(f"  loss gpu {loss:.8e} oracle {lref:.8e}; grad max rel {rel:.2e}")
        assert abs(loss - lref) <= 1e-5 * abs(lref)
        assert rel < 1e-4
    finally:
        dgd.dgd_surrogate_destroy(s)


def test_training_is_reproducible_and_learns(dgd):
    imgs, ld, tg = _data(512, 7)
    runs = []
    for _ in range(2):
        s = dgd.Surrogate(n_members=2, channels=8, hidden=32, seed=5)
        losses = s.train(imgs, ld, tg, epochs=6, batch=64, lr=2e-3, shuffle_seed=9)
        runs.append((losses, dgd.dgd_surrogate_get_params(s.handle, 1)))
        s.close()
    say(f"surrogate losses {runs[0][0]}")
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])
    assert (runs[0][0][:, -1] < 0.5 * runs[0][0][:, 0]).all()


def test_ensemble_spread_and_fallback(dgd):
    imgs, ld, tg = _data(300, 8)
    s = dgd.Surrogate(n_members=3, channels=4, hidden=16, seed=1)
    mean, spread, flag = s.predict(imgs, ld, threshold=1e-3)
    outs = []
    for m in range(3):
        one = dgd.dgd_surrogate_create(1, 4, 16, 0)
        dgd.dgd_surrogate_set_params(one, 0, dgd.dgd_surrogate_get_params(s.handle, m))
        o, _, _ = dgd.dgd_surrogate_predict(one, imgs, ld, 1.0)
        outs.append(o)
        dgd.dgd_surrogate_destroy(one)
    outs = np.stack(outs)
    assert np.allclose(mean, outs.mean(0), rtol=1e-6, atol=1e-7)
    sp = (outs.max(0) - outs.min(0)).max(1)
    assert np.allclose(spread, sp, rtol=1e-6, atol=1e-7)
    assert np.array_equal(flag, sp > 1e-3)
    s.close()

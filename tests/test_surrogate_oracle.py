"""Pins of the FP64 surrogate reference (CPU): its convolution against
SciPy's 2D correlation, pooling adjointness, and its analytic gradient
against central finite differences (V15)."""

import numpy as np
from scipy.signal import correlate2d

from oracle import surrogate as sg


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 9, 9))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = sg.conv3x3(x, w, b)
    for bi in range(2):
        for o in range(4):
            ref = sum(correlate2d(x[bi, c], w[o, c], mode="same") for c in range(3)) + b[o]
            assert np.abs(out[bi, o] - ref).max() < 1e-12


def test_conv_and_pool_adjoints():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 8, 8))
    w = rng.standard_normal((5, 3, 3, 3))
    dz = rng.standard_normal((2, 5, 8, 8))
    dx, dw, db = sg.conv3x3_backward(x, w, dz)
    # <conv(x), dz> is linear in x and in w: its gradients are dx and dw
    f = lambda xx, ww: float((sg.conv3x3(xx, ww, np.zeros(5)) * dz).sum())  # noqa: E731
    v = rng.standard_normal(x.shape)
    assert abs(f(x + v, w) - f(x, w) - (dx * v).sum()) < 1e-9 * abs((dx * v).sum())
    u = rng.standard_normal(w.shape)
    assert abs(f(x, w + u) - f(x, w) - (dw * u).sum()) < 1e-9 * abs((dw * u).sum())
    assert np.allclose(db, dz.sum(axis=(0, 2, 3)))
    y = rng.standard_normal((2, 3, 4, 4))
    assert abs((sg.pool2(x) * y).sum() - (x * sg.pool2_backward(y)).sum()) < 1e-12


def test_gradient_matches_finite_differences():
    """V15: every parameter of a reduced-width net (C = 3, H = 5)."""
    C, H = 3, 5
    rng = np.random.default_rng(2)
    theta = sg.init_params(rng, C, H) + 0.05 * rng.standard_normal(sg.n_params(C, H))
    imgs = (rng.random((3, 64, 64)) < 0.4).astype(float)
    ld = rng.uniform(0, 4, 3)
    tg = rng.standard_normal((3, 3))
    loss, g = sg.loss_and_grad(theta, imgs, ld, tg, C, H)
    eps = 1e-6
    fd = np.zeros_like(g)
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = eps
        lp = float(((sg.forward(theta + e, imgs, ld, C, H) - tg) ** 2).mean())
        lm = float(((sg.forward(theta - e, imgs, ld, C, H) - tg) ** 2).mean())
        fd[k] = (lp - lm) / (2 * eps)
    err = np.abs(fd - g).max() / np.abs(g).max()
    assert err < 1e-6, err


def test_parameter_count_of_the_full_network():
    assert sg.n_params(32, 256) == 292003

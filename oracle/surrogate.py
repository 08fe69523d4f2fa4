"""FP64 reference of the learned surrogate (oracle, test infrastructure).

The paper has no learned component; it motivates fast simulators partly by
training learning algorithms on simulated data (section 1).  The surrogate
maps a 64 x 64 binary occupancy image of a substrate (1 = axon cell) and
log(Delta / 1 ms) to the three unique entries of Sigma / (2 D Delta).

Architecture (the reading taken where the workload leaves it open):
  4 x [conv 3x3, zero pad 1, C channels, + bias, ReLU, 2x2 average pool]
      64x64x1 -> 32x32xC -> 16x16xC -> 8x8xC -> 4x4xC
  flatten (channel-major: c, y, x) -> 16 C values, append log Delta
  3 x [dense H units + bias, ReLU], dense 3 outputs + bias
  loss: mean over the batch and the 3 outputs of the squared error.
C = 32, H = 256 gives 292,003 parameters.

Parameters are one flat float64 vector in the order
  conv1.w [C,1,3,3], conv1.b [C], conv2.w [C,C,3,3], conv2.b, conv3.w,
  conv3.b, conv4.w, conv4.b, fc1.w [H, 16C+1], fc1.b [H], fc2.w [H,H],
  fc2.b, fc3.w [H,H], fc3.b, head.w [3,H], head.b [3]
(weights row-major, output index first).
"""

from __future__ import annotations

import numpy as np

IMG = 64


def layer_shapes(C: int = 32, H: int = 256):
    shapes = []
    cin = 1
    for _ in range(4):
        shapes.append(("conv", (C, cin, 3, 3)))
        shapes.append(("bias", (C,)))
        cin = C
    feat = C * 16 + 1
    for _ in range(3):
        shapes.append(("dense", (H, feat)))
        shapes.append(("bias", (H,)))
        feat = H
    shapes.append(("dense", (3, H)))
    shapes.append(("bias", (3,)))
    return shapes


def n_params(C: int = 32, H: int = 256) -> int:
    return int(sum(np.prod(s) for _, s in layer_shapes(C, H)))


def unpack(theta, C=32, H=256):
    out = []
    k = 0
    for _, s in layer_shapes(C, H):
        n = int(np.prod(s))
        out.append(theta[k:k + n].reshape(s))
        k += n
    return out


def init_params(rng, C=32, H=256) -> np.ndarray:
    """He-uniform weights, zero biases."""
    parts = []
    for kind, s in layer_shapes(C, H):
        if kind == "bias":
            parts.append(np.zeros(s))
        else:
            fan_in = int(np.prod(s[1:]))
            lim = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, size=s))
    return np.concatenate([p.ravel() for p in parts])


def conv3x3(x, w, b):
    """Cross-correlation with zero padding 1: x [B,Ci,Hh,Ww], w [Co,Ci,3,3]."""
    B, Ci, Hh, Ww = x.shape
    xp = np.zeros((B, Ci, Hh + 2, Ww + 2))
    xp[:, :, 1:-1, 1:-1] = x
    out = np.zeros((B, w.shape[0], Hh, Ww))
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + Hh, kx:kx + Ww]             # [B,Ci,Hh,Ww]
            out += np.einsum("bchw,oc->bohw", patch, w[:, :, ky, kx])
    return out + b[None, :, None, None]


def conv3x3_backward(x, w, dz):
    """Gradients of conv3x3 wrt x, w, b given dz = dL/d(out)."""
    B, Ci, Hh, Ww = x.shape
    xp = np.zeros((B, Ci, Hh + 2, Ww + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + Hh, kx:kx + Ww]
            dw[:, :, ky, kx] = np.einsum("bohw,bchw->oc", dz, patch)
            dxp[:, :, ky:ky + Hh, kx:kx + Ww] += np.einsum("bohw,oc->bchw", dz, w[:, :, ky, kx])
    return dxp[:, :, 1:-1, 1:-1], dw, dz.sum(axis=(0, 2, 3))


def pool2(x):
    B, C, Hh, Ww = x.shape
    return x.reshape(B, C, Hh // 2, 2, Ww // 2, 2).mean(axis=(3, 5))


def pool2_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=2), 2, axis=3) * 0.25


def forward(theta, images, log_delta, C=32, H=256, keep=False):
    """Outputs [B, 3] (and the activations needed by backward)."""
    P = unpack(theta, C, H)
    x = np.asarray(images, dtype=np.float64)[:, None, :, :]
    cache = []
    for L in range(4):
        w, b = P[2 * L], P[2 * L + 1]
        z = conv3x3(x, w, b)
        a = np.maximum(z, 0.0)
        cache.append((x, z))
        x = pool2(a)
    feat = np.concatenate([x.reshape(x.shape[0], -1), np.asarray(log_delta, float)[:, None]], axis=1)
    h = feat
    dense = []
    for L in range(3):
        W, b = P[8 + 2 * L], P[9 + 2 * L]
        z = h @ W.T + b
        dense.append((h, z))
        h = np.maximum(z, 0.0)
    out = h @ P[14].T + P[15]
    dense.append((h, out))
    if keep:
        return out, (cache, dense)
    return out


def loss_and_grad(theta, images, log_delta, target, C=32, H=256):
    """Mean squared error and its gradient wrt theta (FP64)."""
    P = unpack(theta, C, H)
    out, (cache, dense) = forward(theta, images, log_delta, C, H, keep=True)
    B = out.shape[0]
    diff = out - target
    loss = float((diff ** 2).mean())
    g = [None] * len(P)
    dout = 2.0 * diff / diff.size
    h, _ = dense[3]
    g[14] = dout.T @ h
    g[15] = dout.sum(0)
    dh = dout @ P[14]
    for L in (2, 1, 0):
        hin, z = dense[L]
        dz = dh * (z > 0)
        g[8 + 2 * L] = dz.T @ hin
        g[9 + 2 * L] = dz.sum(0)
        dh = dz @ P[8 + 2 * L]
    dfeat = dh[:, :-1].reshape(B, C, 4, 4)
    da = dfeat
    for L in (3, 2, 1, 0):
        xin, z = cache[L]
        dpre = pool2_backward(da) * (z > 0)
        dx, dw, db = conv3x3_backward(xin, P[2 * L], dpre)
        g[2 * L], g[2 * L + 1] = dw, db
        da = dx
    grad = np.concatenate([x.ravel() for x in g])
    return loss, grad

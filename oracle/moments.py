"""Exact moments of the discrete solution and the covariance readings.

Section 4.1 of the paper turns each solution into a density (centring and
normalisation), mixes the m densities and fits a Gaussian, whose covariance
it computes by quadrature of the nodal values.  Reading taken here: the fit
is the moment estimator, and the integrals are exact for the piecewise
polynomial solution.

Per start point x0 the oracle returns six moments of u about x0:
  M0 = int u,  (mx, my) = int (x - x0) u,  (Mxx, Mxy, Myy) = int (x - x0)(x - x0)^T u,
summed over elements with element-local offsets: on element K with cell
centre c_K, x - x0 = h*xi + d_K with d_K = c_K - x0, and the local integrals
int psi_k xi^a eta^b are exact (``sipg.LocalOps.Wmom``).

Three covariance readings are derived from the moments:
  Sigma_A = M2 / M0                 (about the start point),
  Sigma_B = mean_i (M2_i/M0_i - mu_i mu_i^T),   mu_i = m1_i / M0_i,
  Sigma_C = mean_i Sigma_A,i - mubar mubar^T,   mubar = mean_i mu_i
(C is the covariance of the mixture about its mean, as in section 4.1).
"""

from __future__ import annotations

import numpy as np

from .sipg import Operator


def moments(op: Operator, U: np.ndarray, x0s: np.ndarray) -> np.ndarray:
    """Moments [R, 6] = (M0, mx, my, Mxx, Mxy, Myy) of U [ndof, R] about x0s [R, 2]."""
    mesh = op.mesh
    h = mesh.h
    Np = op.Np
    R = U.shape[1]
    Ue = U.reshape(mesh.n_elements, Np, R)
    xc = (mesh.cell_i + 0.5) * h
    yc = (mesh.cell_j + 0.5) * h
    out = np.zeros((R, 6))
    for o in (0, 1):
        sel = np.flatnonzero(mesh.orient == o)
        W = op.loc.Wmom[o]                                   # [6, Np] dimensionless
        scale = h * h * np.array([1.0, h, h, h * h, h * h, h * h])
        I = np.einsum("ak,ekr->ear", W * scale[:, None], Ue[sel])   # [n, 6, R]
        i0, ix, iy, ixx, ixy, iyy = (I[:, a, :] for a in range(6))
        dx = xc[sel, None] - x0s[None, :, 0]                 # [n, R]
        dy = yc[sel, None] - x0s[None, :, 1]
        out[:, 0] += i0.sum(0)
        out[:, 1] += (ix + dx * i0).sum(0)
        out[:, 2] += (iy + dy * i0).sum(0)
        out[:, 3] += (ixx + 2.0 * dx * ix + dx * dx * i0).sum(0)
        out[:, 4] += (ixy + dx * iy + dy * ix + dx * dy * i0).sum(0)
        out[:, 5] += (iyy + 2.0 * dy * iy + dy * dy * i0).sum(0)
    return out


def sigma_a(mom: np.ndarray) -> np.ndarray:
    """Sigma about the start point, [..., 3] = (xx, xy, yy)."""
    return mom[..., 3:6] / mom[..., 0:1]


def sigma_b(mom: np.ndarray) -> np.ndarray:
    """Per-point covariance about its own mean, [..., 3]."""
    m0 = mom[..., 0]
    mx = mom[..., 1] / m0
    my = mom[..., 2] / m0
    s = sigma_a(mom).copy()
    s[..., 0] -= mx * mx
    s[..., 1] -= mx * my
    s[..., 2] -= my * my
    return s


def mixture(mom: np.ndarray) -> dict:
    """Mixture readings over start points (axis 0 of mom [R, ..., 6])."""
    sa = sigma_a(mom)
    m0 = mom[..., 0]
    mu = np.stack([mom[..., 1] / m0, mom[..., 2] / m0], axis=-1)
    mubar = mu.mean(0)
    A = sa.mean(0)
    B = sigma_b(mom).mean(0)
    C = A.copy()
    C[..., 0] -= mubar[..., 0] ** 2
    C[..., 1] -= mubar[..., 0] * mubar[..., 1]
    C[..., 2] -= mubar[..., 1] ** 2
    return dict(A=A, B=B, C=C)


def rel_err(s, ref):
    """Frobenius relative error of symmetric 2x2 matrices stored as (xx, xy, yy)."""
    def fro(v):
        return np.sqrt(v[..., 0] ** 2 + 2.0 * v[..., 1] ** 2 + v[..., 2] ** 2)
    return fro(np.asarray(s) - np.asarray(ref)) / fro(np.asarray(ref))

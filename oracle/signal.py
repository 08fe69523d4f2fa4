"""Narrow-pulse q-space signal of the ensemble average propagator (oracle,
test infrastructure).

The paper describes the displacement law of the diffusing molecules by the
ensemble average propagator P(r, Delta) (section 1) and names the
diffusion-weighted MR signal, the Fourier transform of P, as the use of the
simulated propagator (section 5).  For a start point x0 whose solution u
has unit initial mass, P(r, Delta) = u(x0 + r, Delta), so the signal is

    E(q) = int u(x, Delta) exp(i q . (x - x0)) dx,

q in rad/um (angular wavenumber, no 2 pi).  E(0) = M0 (the mass), E(-q) is
the complex conjugate of E(q), and for small q
E(q) = M0 + i q.m1 - q^T M2 q / 2 + O(q^3) with the moments about x0.

The integral is taken element by element with a collapsed Gauss-Jacobi x
Gauss-Legendre product rule of n x n points (n = 16), exact for the
polynomial factor and converging super-exponentially in |q| h for the
exponential factor.
"""

from __future__ import annotations

import numpy as np

from .initial import _collapsed_rule
from .sipg import VERTS, Operator, monomials


def signal(op: Operator, U: np.ndarray, x0s: np.ndarray, qs: np.ndarray,
           n_quad: int = 16) -> np.ndarray:
    """E(q) for every right-hand side and q: complex [R, nq].

    U: coefficients [ndof, R] (the oracle's monomial basis); x0s: [R, 2]
    start points; qs: [nq, 2] wave vectors in rad/um.
    """
    mesh = op.mesh
    h = mesh.h
    Np = op.Np
    U = np.asarray(U, dtype=np.float64).reshape(mesh.n_elements, Np, -1)
    x0s = np.asarray(x0s, dtype=np.float64).reshape(-1, 2)
    qs = np.asarray(qs, dtype=np.float64).reshape(-1, 2)
    R = U.shape[2]
    mons = monomials(op.p)
    r, s, w = _collapsed_rule(n_quad)
    xc = (mesh.cell_i + 0.5) * h
    yc = (mesh.cell_j + 0.5) * h
    out = np.zeros((R, qs.shape[0]), dtype=np.complex128)
    for o in (0, 1):
        sel = np.flatnonzero(mesh.orient == o)
        if sel.size == 0:
            continue
        v0, v1, v2 = (np.array(q) for q in VERTS[o])
        xi = v0[0] + r * (v1[0] - v0[0]) + s * (v2[0] - v0[0])
        et = v0[1] + r * (v1[1] - v0[1]) + s * (v2[1] - v0[1])
        jac = abs((v1[0] - v0[0]) * (v2[1] - v0[1]) - (v2[0] - v0[0]) * (v1[1] - v0[1]))
        psi = np.stack([xi ** a * et ** b for (a, b) in mons])          # [Np, Q]
        u_q = np.einsum("kq,ekr->eqr", psi, U[sel])                      # u at the points
        X = xc[sel, None] + h * xi[None, :]                              # [n_sel, Q]
        Y = yc[sel, None] + h * et[None, :]
        wq = w * jac * h * h
        for r_ in range(R):
            dx = X - x0s[r_, 0]
            dy = Y - x0s[r_, 1]
            uw = u_q[:, :, r_] * wq[None, :]
            for k in range(qs.shape[0]):
                ph = np.exp(1j * (qs[k, 0] * dx + qs[k, 1] * dy))
                out[r_, k] += np.sum(ph * uw)
    return out


def element_integral(op: Operator, coef: np.ndarray, e: int, x0, q, n_quad: int = 16) -> complex:
    """int_K u exp(i q.(x - x0)) dx on element e alone (coef: [Np])."""
    mesh = op.mesh
    h = mesh.h
    o = int(mesh.orient[e])
    r, s, w = _collapsed_rule(n_quad)
    v0, v1, v2 = (np.array(p) for p in VERTS[o])
    xi = v0[0] + r * (v1[0] - v0[0]) + s * (v2[0] - v0[0])
    et = v0[1] + r * (v1[1] - v0[1]) + s * (v2[1] - v0[1])
    jac = abs((v1[0] - v0[0]) * (v2[1] - v0[1]) - (v2[0] - v0[0]) * (v1[1] - v0[1]))
    u = sum(c * xi ** a * et ** b for c, (a, b) in zip(coef, monomials(op.p)))
    X = (mesh.cell_i[e] + 0.5) * h + h * xi
    Y = (mesh.cell_j[e] + 0.5) * h + h * et
    ph = np.exp(1j * (q[0] * (X - x0[0]) + q[1] * (Y - x0[1])))
    return complex(np.sum(w * jac * h * h * u * ph))

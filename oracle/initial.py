"""Initial data: L2 projection of a Gaussian pulse, normalised to unit mass.

The paper starts each solve from a Dirac pulse at a start point (section
4.1) and normalises every solution to a density.  Reading taken here: the
pulse is a Gaussian g(x) = exp(-|x - x0|^2 / (2 sigma0^2)) restricted to the
active triangles, L2-projected elementwise onto P_p and divided by the mass
of the projection, so that mass falling on removed cells or outside the box
is discarded before normalising.  (A projection, not nodal interpolation:
it keeps every moment of degree <= p of the restricted Gaussian.)

Quadrature: a collapsed (Duffy) product rule on each triangle, Gauss-Jacobi
(alpha = 1) in the collapsed direction times Gauss-Legendre in the other,
n x n points (n = 14 by default), accurate to ~1e-15 relative for the pulse
widths used here.  Elements whose cell lies farther than 12 sigma0 from x0
are skipped (the Gaussian is below exp(-72) there).
"""

from __future__ import annotations

import numpy as np
from scipy.special import roots_jacobi, roots_legendre

from .sipg import VERTS, Operator, monomials


def _collapsed_rule(n):
    """Points (r, s) and weights on the unit triangle, exact to degree 2n-2."""
    xv, wv = roots_jacobi(n, 1.0, 0.0)      # weight (1 - x) on [-1, 1]
    xu, wu = roots_legendre(n)
    v = 0.5 * (1.0 + xv)
    wv = 0.25 * wv                          # int_0^1 (1 - v) f dv
    u = 0.5 * (1.0 + xu)
    wu = 0.5 * wu
    r = (u[:, None] * (1.0 - v[None, :])).ravel()
    s = np.broadcast_to(v[None, :], (n, n)).ravel()
    w = (wu[:, None] * wv[None, :]).ravel()
    return r, s, w


def project_dirac(op: Operator, x0: np.ndarray) -> np.ndarray:
    """L2 projection of the point mass at x0 (the paper's Dirac pulse):
    on the triangle holding x0, u = M_K^-1 psi(x0), so int u v = v(x0) for
    every v of the space; its mass is exactly 1.  The triangle: cell
    (floor(x/h), floor(y/h)), T0 when x0 lies on or below the cell's
    diagonal, else T1."""
    mesh = op.mesh
    h = mesh.h
    i = min(int(np.floor(x0[0] / h)), mesh.N - 1)
    j = min(int(np.floor(x0[1] / h)), mesh.N - 1)
    fx, fy = x0[0] / h - i, x0[1] / h - j
    o = 0 if fx >= fy else 1
    hit = np.flatnonzero((mesh.cell_i == i) & (mesh.cell_j == j) & (mesh.orient == o))
    if hit.size != 1:
        raise ValueError("the point lies in a removed cell or outside the box")
    xi, et = fx - 0.5, fy - 0.5
    psi = np.array([xi ** a * et ** b for (a, b) in monomials(op.p)])
    coef = np.zeros((mesh.n_elements, op.Np))
    coef[hit[0]] = op.Minv_blocks[o] @ psi
    return coef.ravel()


def project_gaussian(op: Operator, x0: np.ndarray, sigma0: float, n_quad: int = 14,
                     cutoff: float = 12.0) -> np.ndarray:
    """Unit-mass L2 projection of the Gaussian at x0 (coefficients [ndof]);
    sigma0 = 0 gives the projected point mass (project_dirac)."""
    if sigma0 == 0:
        return project_dirac(op, np.asarray(x0, dtype=np.float64))
    mesh = op.mesh
    h = mesh.h
    Np = op.Np
    mons = monomials(op.p)
    r, s, w = _collapsed_rule(n_quad)
    xc = (mesh.cell_i + 0.5) * h
    yc = (mesh.cell_j + 0.5) * h
    # distance from x0 to the cell square
    ddx = np.maximum(np.abs(xc - x0[0]) - 0.5 * h, 0.0)
    ddy = np.maximum(np.abs(yc - x0[1]) - 0.5 * h, 0.0)
    near = ddx * ddx + ddy * ddy <= (cutoff * sigma0) ** 2
    coef = np.zeros((mesh.n_elements, Np))
    for o in (0, 1):
        sel = np.flatnonzero(near & (mesh.orient == o))
        if sel.size == 0:
            continue
        v0, v1, v2 = (np.array(q) for q in VERTS[o])
        xi = v0[0] + r * (v1[0] - v0[0]) + s * (v2[0] - v0[0])
        et = v0[1] + r * (v1[1] - v0[1]) + s * (v2[1] - v0[1])
        jac = abs((v1[0] - v0[0]) * (v2[1] - v0[1]) - (v2[0] - v0[0]) * (v1[1] - v0[1]))
        X = xc[sel, None] + h * xi[None, :]
        Y = yc[sel, None] + h * et[None, :]
        g = np.exp(-((X - x0[0]) ** 2 + (Y - x0[1]) ** 2) / (2.0 * sigma0 * sigma0))
        psi = np.stack([xi ** a * et ** b for (a, b) in mons])          # [Np, Q]
        rhs = (g * (w * jac * h * h)[None, :]) @ psi.T                   # [n_sel, Np]
        coef[sel] = rhs @ op.Minv_blocks[o].T
    mass = 0.0
    for o in (0, 1):
        sel = mesh.orient == o
        mass += float((coef[sel] @ (h * h * op.loc.Wmom[o][0])).sum())
    return (coef / mass).ravel()

"""Symmetric interior-penalty DG operator on the pixel-triangle mesh (oracle).

The paper writes diffusion as the first-order system q = grad u,
u_t = div(k q) (eq. (6)), with element weak forms (eq. (7)), a central flux
for u and a harmonic-mean flux for q (section 3.2).  The main path uses the
primal symmetric interior-penalty form instead, on the extracellular
triangles only (removed axon cells, zero flux on their faces):

  a(u, v) = sum_K int_K D grad u . grad v
          - sum_F int_F ( {D grad u}.n [v] + {D grad v}.n [u] )
          + sum_F int_F sigma_F [u][v],       sigma_F = eta p^2 D / h,

[w] = w- - w+, {w} = (w- + w+)/2, n pointing from - to +, sums over
interior faces only (wall and box faces contribute nothing: zero Neumann
data, eq. (3)).  h is the cell edge for all three face types.  The
semi-discrete system is M du/dt = -A u.

With an absorbing outer box (the paper's eq. (4), u = 0 on the square's
edges) each box face F of an active triangle adds the same terms with the
outside value zero (Nitsche):
  - int_F ( D grad u . n v + D grad v . n u ) + int_F sigma_F u v.

Basis: the oracle uses a modal basis, monomials xi**a * eta**b (a + b <= p)
in the cell-centred scaled coordinates xi = (x - x_c)/h, eta = (y - y_c)/h,
on purpose different from the nodal Lagrange basis of the paper (eq. (8))
that the GPU path uses.  The discrete solution does not depend on the basis.
All integrals are exact (``poly``).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

from . import poly
from .mesh import FACE_OFFSETS, Mesh

H = 0.5
# Triangle vertices in the scaled cell-centred frame.
VERTS = {0: [(-H, -H), (H, -H), (H, H)], 1: [(-H, -H), (H, H), (-H, H)]}
# Faces: (start, end, outward normal scaled by the face length in h units).
# The scaled normal of the diagonal is (-1, 1) for T0 (length sqrt 2 times
# unit normal (-1, 1)/sqrt 2).
FACES = {
    0: [((-H, -H), (H, -H), (0.0, -1.0), 1.0),
        ((H, -H), (H, H), (1.0, 0.0), 1.0),
        ((H, H), (-H, -H), (-1.0, 1.0), math.sqrt(2.0))],
    1: [((H, H), (-H, H), (0.0, 1.0), 1.0),
        ((-H, H), (-H, -H), (-1.0, 0.0), 1.0),
        ((-H, -H), (H, H), (1.0, -1.0), math.sqrt(2.0))],
}
MOMENT_POWERS = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]


def monomials(p):
    return [(d - b, b) for d in range(p + 1) for b in range(d + 1)]


@dataclasses.dataclass
class LocalOps:
    """Dimensionless local matrices (h = 1, D = 1) for one polynomial degree."""
    p: int
    eta: float
    Mhat: list        # [o] Np x Np mass
    Khat: list        # [o] Np x Np stiffness
    Fself: list       # [o][f] Np x Np face self terms (with penalty)
    Fnbr: list        # [o][f] Np x Np face neighbour terms
    Fdir: list        # [o][f] Np x Np terms of face f with zero outside value
    Wmom: list        # [o] 6 x Np: integral of psi_k * xi^a eta^b over the triangle


def local_ops(p: int, eta: float) -> LocalOps:
    """Local SIPG matrices from exact integrals (weak form, eq. (7))."""
    mons = monomials(p)
    Np = len(mons)
    basis = [{m: 1.0} for m in mons]
    gx = [poly.dx(b) for b in basis]
    gy = [poly.dy(b) for b in basis]
    pen = eta * p * p
    Mhat, Khat, Fs, Fn, Fd, W = [], [], [], [], [], []
    for o in (0, 1):
        v = VERTS[o]
        Mo = np.zeros((Np, Np))
        Ko = np.zeros((Np, Np))
        for k in range(Np):
            for l in range(Np):
                Mo[k, l] = poly.integrate_triangle(poly.pmul(basis[k], basis[l]), *v)
                grad = poly.padd(poly.pmul(gx[k], gx[l]), poly.pmul(gy[k], gy[l]))
                Ko[k, l] = poly.integrate_triangle(grad, *v)
        Wo = np.zeros((6, Np))
        for a, (px, py) in enumerate(MOMENT_POWERS):
            for k in range(Np):
                Wo[a, k] = poly.integrate_triangle(poly.pmul(basis[k], {(px, py): 1.0}), *v)
        Fs_o, Fn_o, Fd_o = [], [], []
        for f, (p0, p1, nl, length) in enumerate(FACES[o]):
            ox, oy = FACE_OFFSETS[o][f]
            nb = [poly.shift(b, -ox, -oy) for b in basis]        # neighbour basis in my frame
            ngx = [poly.dx(b) for b in nb]
            ngy = [poly.dy(b) for b in nb]
            dn = [poly.padd(poly.pscale(gx[k], nl[0]), poly.pscale(gy[k], nl[1])) for k in range(Np)]
            dn_nb = [poly.padd(poly.pscale(ngx[k], nl[0]), poly.pscale(ngy[k], nl[1])) for k in range(Np)]
            S = np.zeros((Np, Np))
            Nm = np.zeros((Np, Np))
            Bd = np.zeros((Np, Np))
            for k in range(Np):
                for l in range(Np):
                    Bd[k, l] = (-poly.integrate_edge_param(poly.pmul(dn[l], basis[k]), p0, p1)
                                - poly.integrate_edge_param(poly.pmul(dn[k], basis[l]), p0, p1)
                                + pen * length
                                * poly.integrate_edge_param(poly.pmul(basis[k], basis[l]), p0, p1))
                    # nl already carries the face length; the penalty term
                    # carries it explicitly.
                    s = (-0.5 * poly.integrate_edge_param(poly.pmul(dn[l], basis[k]), p0, p1)
                         - 0.5 * poly.integrate_edge_param(poly.pmul(dn[k], basis[l]), p0, p1)
                         + pen * length * poly.integrate_edge_param(poly.pmul(basis[k], basis[l]), p0, p1))
                    n = (-0.5 * poly.integrate_edge_param(poly.pmul(dn_nb[l], basis[k]), p0, p1)
                         + 0.5 * poly.integrate_edge_param(poly.pmul(dn[k], nb[l]), p0, p1)
                         - pen * length * poly.integrate_edge_param(poly.pmul(basis[k], nb[l]), p0, p1))
                    S[k, l] = s
                    Nm[k, l] = n
            Fs_o.append(S)
            Fn_o.append(Nm)
            Fd_o.append(Bd)
        Mhat.append(Mo)
        Khat.append(Ko)
        Fs.append(Fs_o)
        Fn.append(Fn_o)
        Fd.append(Fd_o)
        W.append(Wo)
    return LocalOps(p=p, eta=eta, Mhat=Mhat, Khat=Khat, Fself=Fs, Fnbr=Fn, Fdir=Fd, Wmom=W)


@dataclasses.dataclass
class Operator:
    mesh: Mesh
    p: int
    D: float
    eta: float
    loc: LocalOps
    A: sp.csr_matrix          # stiffness with face terms, physical units
    M: sp.csr_matrix          # block-diagonal mass, physical units
    L: sp.csr_matrix          # -M^-1 A
    Minv_blocks: list         # [o] physical M_o^-1
    outer: str = "reflect"    # outer box: "reflect" (zero flux) or "absorb" (u = 0)

    @property
    def Np(self) -> int:
        return (self.p + 1) * (self.p + 2) // 2

    @property
    def ndof(self) -> int:
        return self.mesh.n_elements * self.Np


def _block_coo(rows_e, cols_e, block, Np):
    """COO triplets for the same Np x Np block at element pairs (rows_e, cols_e)."""
    k, l = np.meshgrid(np.arange(Np), np.arange(Np), indexing="ij")
    r = (rows_e[:, None, None] * Np + k[None]).ravel()
    c = (cols_e[:, None, None] * Np + l[None]).ravel()
    v = np.broadcast_to(block[None], (rows_e.size, Np, Np)).ravel()
    return r, c, v


def box_faces(mesh: Mesh):
    """[(o, f, elements)] of the faces on the square's edges: T0 bottom
    (f 0, row 0) and right (f 1, column N-1); T1 top (f 0, row N-1) and left
    (f 1, column 0).  The diagonal never lies on the box."""
    N = mesh.N
    T0 = mesh.orient == 0
    T1 = ~T0
    return [(0, 0, np.flatnonzero(T0 & (mesh.cell_j == 0))),
            (0, 1, np.flatnonzero(T0 & (mesh.cell_i == N - 1))),
            (1, 0, np.flatnonzero(T1 & (mesh.cell_j == N - 1))),
            (1, 1, np.flatnonzero(T1 & (mesh.cell_i == 0)))]


def assemble(mesh: Mesh, p: int, D: float, eta: float, loc: LocalOps | None = None,
             outer: str = "reflect") -> Operator:
    """Global SIPG matrices A, M and L = -M^-1 A (eq. (7) in primal form);
    outer = "absorb" imposes u = 0 on the box (eq. (4))."""
    if outer not in ("reflect", "absorb"):
        raise ValueError("outer must be 'reflect' or 'absorb'")
    loc = loc or local_ops(p, eta)
    Np = (p + 1) * (p + 2) // 2
    h = mesh.h
    E = mesh.n_elements
    active = mesh.nbr >= 0
    mask = active[:, 0] * 1 + active[:, 1] * 2 + active[:, 2] * 4
    Ar, Ac, Av = [], [], []
    Lr, Lc, Lv = [], [], []
    Minv = [np.linalg.inv(h * h * loc.Mhat[o]) for o in (0, 1)]
    for o in (0, 1):
        for m in range(8):
            sel = np.flatnonzero((mesh.orient == o) & (mask == m))
            if sel.size == 0:
                continue
            blk = loc.Khat[o].copy()
            for f in range(3):
                if m >> f & 1:
                    blk = blk + loc.Fself[o][f]
            blk = D * blk
            r, c, v = _block_coo(sel, sel, blk, Np)
            Ar.append(r); Ac.append(c); Av.append(v)
            r, c, v = _block_coo(sel, sel, -Minv[o] @ blk, Np)
            Lr.append(r); Lc.append(c); Lv.append(v)
        for f in range(3):
            sel = np.flatnonzero((mesh.orient == o) & active[:, f])
            if sel.size == 0:
                continue
            blk = D * loc.Fnbr[o][f]
            r, c, v = _block_coo(sel, mesh.nbr[sel, f], blk, Np)
            Ar.append(r); Ac.append(c); Av.append(v)
            r, c, v = _block_coo(sel, mesh.nbr[sel, f], -Minv[o] @ blk, Np)
            Lr.append(r); Lc.append(c); Lv.append(v)
    if outer == "absorb":
        for o, f, sel in box_faces(mesh):
            if sel.size == 0:
                continue
            blk = D * loc.Fdir[o][f]
            r, c, v = _block_coo(sel, sel, blk, Np)
            Ar.append(r); Ac.append(c); Av.append(v)
            r, c, v = _block_coo(sel, sel, -Minv[o] @ blk, Np)
            Lr.append(r); Lc.append(c); Lv.append(v)
    n = E * Np
    cat = lambda xs: np.concatenate(xs) if xs else np.zeros(0)  # noqa: E731
    A = sp.coo_matrix((cat(Av), (cat(Ar), cat(Ac))), shape=(n, n)).tocsr()
    L = sp.coo_matrix((cat(Lv), (cat(Lr), cat(Lc))), shape=(n, n)).tocsr()
    Mr, Mc, Mv = [], [], []
    for o in (0, 1):
        sel = np.flatnonzero(mesh.orient == o)
        r, c, v = _block_coo(sel, sel, h * h * loc.Mhat[o], Np)
        Mr.append(r); Mc.append(c); Mv.append(v)
    M = sp.coo_matrix((cat(Mv), (cat(Mr), cat(Mc))), shape=(n, n)).tocsr()
    return Operator(mesh=mesh, p=p, D=D, eta=eta, loc=loc, A=A, M=M, L=L, Minv_blocks=Minv,
                    outer=outer)

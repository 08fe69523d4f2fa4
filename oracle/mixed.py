"""The paper's own formulation on all pixels (oracle, test infrastructure).

First-order system (eq. (6)): q = grad u, u_t = div(k q), with k = D in
the extracellular cells and k = 0 in the axon cells, which are kept in the
mesh (section 1: the whole domain is solved, null work in the axons).
Element weak forms (eq. (7)) with the fluxes of section 3.2:

  int_K q . w = int_dK {u} w . n ds - int_K u div w dx,
  int_K u_t v = int_dK k_h {q} . n v ds - int_K k q . grad v dx,

{a} = (a- + a+)/2 (central flux for u), k_h = 2 k- k+ / (k- + k+) (the
harmonic mean, 0 when either side is an axon cell: no flow between axon
and extracellular cells).  On the square's edges (zero flux, the default
outer condition of the library): the u-flux is u- itself and the q-flux is
zero.  With the gradient of the trial function moved back,

  q = grad_h u + sum_F lift_F((u+ - u-)/2),

so in each element q is the broken gradient plus the face terms; the
update of u reads q of the element and of its face neighbours.  Semi-
discrete system: q = G u, du/dt = Q q, L = Q G.  The axon rows of Q are
zero, so u stays at its initial value (zero) there.

Basis and integrals as in ``sipg``: monomials in the cell-centred scaled
frame, exact polynomial integrals.  Readings where the paper is silent:
the outer box flux (above) and the initial pulse, restricted to the
extracellular cells and normalised to unit mass as for the primal form.
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla

from . import poly
from .bounds import X_RK3
from .initial import project_dirac, project_gaussian
from .moments import moments
from .mesh import FACE_OFFSETS, Mesh, build_mesh
from .sipg import FACES, VERTS, Operator, local_ops, monomials


@dataclasses.dataclass
class MixedLocalOps:
    """Dimensionless local matrices (h = 1) of the mixed form."""
    p: int
    Mhat: list     # [o] mass
    Gx: list       # [o] Gx[k, l] = int (d psi_l / d xi) psi_k
    Gy: list       # [o]
    Ps: list       # [o][f] int_f psi_k psi_l (edge parameter measure)
    Pn: list       # [o][f] int_f psi_k psi'_l (neighbour's basis)
    nl: list       # [o][f] outward normal times the face length (h = 1)


def mixed_local_ops(p: int) -> MixedLocalOps:
    mons = monomials(p)
    Np = len(mons)
    basis = [{m: 1.0} for m in mons]
    gx = [poly.dx(b) for b in basis]
    gy = [poly.dy(b) for b in basis]
    Mh, Gx, Gy, Ps, Pn, NL = [], [], [], [], [], []
    for o in (0, 1):
        v = VERTS[o]
        M = np.zeros((Np, Np))
        X = np.zeros((Np, Np))
        Y = np.zeros((Np, Np))
        for k in range(Np):
            for l in range(Np):
                M[k, l] = poly.integrate_triangle(poly.pmul(basis[k], basis[l]), *v)
                X[k, l] = poly.integrate_triangle(poly.pmul(gx[l], basis[k]), *v)
                Y[k, l] = poly.integrate_triangle(poly.pmul(gy[l], basis[k]), *v)
        ps_o, pn_o, nl_o = [], [], []
        for f, (p0, p1, nl, _length) in enumerate(FACES[o]):
            ox, oy = FACE_OFFSETS[o][f]
            nb = [poly.shift(b, -ox, -oy) for b in basis]
            S = np.zeros((Np, Np))
            N = np.zeros((Np, Np))
            for k in range(Np):
                for l in range(Np):
                    S[k, l] = poly.integrate_edge_param(poly.pmul(basis[k], basis[l]), p0, p1)
                    N[k, l] = poly.integrate_edge_param(poly.pmul(basis[k], nb[l]), p0, p1)
            ps_o.append(S)
            pn_o.append(N)
            nl_o.append(np.asarray(nl, dtype=np.float64))
        Mh.append(M); Gx.append(X); Gy.append(Y); Ps.append(ps_o); Pn.append(pn_o); NL.append(nl_o)
    return MixedLocalOps(p=p, Mhat=Mh, Gx=Gx, Gy=Gy, Ps=Ps, Pn=Pn, nl=NL)


@dataclasses.dataclass
class MixedOperator(Operator):
    """Operator of the mixed form; ``L`` = Q G, ``A`` = -M L (not symmetric
    where k jumps).  ``kel``: k per element; ``G``: [2 ndof, ndof] (q_x rows
    first); ``Q``: [ndof, 2 ndof]."""
    kel: np.ndarray = None
    G: sp.csr_matrix = None
    Q: sp.csr_matrix = None
    mloc: MixedLocalOps = None

    @property
    def extracellular(self) -> np.ndarray:
        return self.kel > 0


def _coo(rows_e, cols_e, blocks, Np, row_off=0, col_off=0):
    """Triplets of one Np x Np block per element pair; blocks [n, Np, Np]."""
    k, l = np.meshgrid(np.arange(Np), np.arange(Np), indexing="ij")
    r = (row_off + rows_e[:, None, None] * Np + k[None]).ravel()
    c = (col_off + cols_e[:, None, None] * Np + l[None]).ravel()
    return r, c, np.asarray(blocks).ravel()


def cell_conductivity(mesh: Mesh, disks: np.ndarray, D: float) -> np.ndarray:
    """k per element: D, or 0 when the cell's centroid lies strictly inside
    a disk (the cells the primal form removes)."""
    h = mesh.h
    xc = (mesh.cell_i + 0.5) * h
    yc = (mesh.cell_j + 0.5) * h
    axon = np.zeros(mesh.n_elements, dtype=bool)
    for cx, cy, r in np.asarray(disks, dtype=np.float64).reshape(-1, 3):
        axon |= (xc - cx) ** 2 + (yc - cy) ** 2 < r * r
    return np.where(axon, 0.0, float(D))


def assemble_mixed(L: float, N: int, disks: np.ndarray, p: int, D: float,
                   kel: np.ndarray | None = None) -> MixedOperator:
    """G, Q and L = Q G on the full N x N pixel mesh; kel overrides k per
    element (default: D outside the disks, 0 inside)."""
    mesh = build_mesh(L, N, np.zeros((0, 3)))
    h = mesh.h
    E = mesh.n_elements
    ml = mixed_local_ops(p)
    Np = len(monomials(p))
    n = E * Np
    k = cell_conductivity(mesh, disks, D) if kel is None else np.asarray(kel, dtype=np.float64)
    Mi = [np.linalg.inv(ml.Mhat[o]) for o in (0, 1)]
    Gr, Gc, Gv = [], [], []
    Qr, Qc, Qv = [], [], []

    def put(R, C, V, trip):
        R.append(trip[0]); C.append(trip[1]); V.append(trip[2])

    for o in (0, 1):
        sel = np.flatnonzero(mesh.orient == o)
        if sel.size == 0:
            continue
        # q = grad_h u: (1/h) Mhat^-1 Gx u
        for comp, Gm in enumerate((ml.Gx[o], ml.Gy[o])):
            blk = np.broadcast_to(Mi[o] @ Gm / h, (sel.size, Np, Np))
            put(Gr, Gc, Gv, _coo(sel, sel, blk, Np, row_off=comp * n))
            # u_t volume term: -(k / h) Mhat^-1 Gm^T q_comp
            blk = (-k[sel] / h)[:, None, None] * (Mi[o] @ Gm.T)[None]
            put(Qr, Qc, Qv, _coo(sel, sel, blk, Np, col_off=comp * n))
        for f in range(3):
            sf = sel[mesh.nbr[sel, f] >= 0]
            if sf.size == 0:
                continue
            nb = mesh.nbr[sf, f]
            nl = ml.nl[o][f]
            kh = np.where((k[sf] > 0) & (k[nb] > 0), 2 * k[sf] * k[nb] / np.maximum(k[sf] + k[nb], 1e-300), 0.0)
            for comp in (0, 1):
                # lifting of the central u-flux: + (1/2) n (u+ - u-) on the face
                s = np.broadcast_to(-0.5 * nl[comp] * (Mi[o] @ ml.Ps[o][f]) / h, (sf.size, Np, Np))
                t = np.broadcast_to(0.5 * nl[comp] * (Mi[o] @ ml.Pn[o][f]) / h, (sf.size, Np, Np))
                put(Gr, Gc, Gv, _coo(sf, sf, s, Np, row_off=comp * n))
                put(Gr, Gc, Gv, _coo(sf, nb, t, Np, row_off=comp * n))
                # q-flux: k_h (q- + q+)/2 . n
                s = (0.5 * kh * nl[comp] / h)[:, None, None] * (Mi[o] @ ml.Ps[o][f])[None]
                t = (0.5 * kh * nl[comp] / h)[:, None, None] * (Mi[o] @ ml.Pn[o][f])[None]
                put(Qr, Qc, Qv, _coo(sf, sf, s, Np, col_off=comp * n))
                put(Qr, Qc, Qv, _coo(sf, nb, t, Np, col_off=comp * n))
    cat = np.concatenate
    G = sp.coo_matrix((cat(Gv), (cat(Gr), cat(Gc))), shape=(2 * n, n)).tocsr()
    Q = sp.coo_matrix((cat(Qv), (cat(Qr), cat(Qc))), shape=(n, 2 * n)).tocsr()
    Lm = (Q @ G).tocsr()
    loc = local_ops(p, 10.0)          # mass and moment weights (penalty unused)
    Mr, Mc, Mv = [], [], []
    for o in (0, 1):
        sel = np.flatnonzero(mesh.orient == o)
        r, c, v = _coo(sel, sel, np.broadcast_to(h * h * loc.Mhat[o], (sel.size, Np, Np)), Np)
        Mr.append(r); Mc.append(c); Mv.append(v)
    M = sp.coo_matrix((cat(Mv), (cat(Mr), cat(Mc))), shape=(n, n)).tocsr()
    Minv = [np.linalg.inv(h * h * loc.Mhat[o]) for o in (0, 1)]
    return MixedOperator(mesh=mesh, p=p, D=float(D), eta=0.0, loc=loc, A=-(M @ Lm).tocsr(), M=M,
                         L=Lm, Minv_blocks=Minv, kel=k, G=G, Q=Q, mloc=ml)


def initial_block(op: MixedOperator, points: np.ndarray, sigma0: float) -> np.ndarray:
    """Initial coefficients [ndof, R]: the Gaussian of section 4.1 projected
    on every element, set to zero in the axon cells and scaled to unit mass
    (sigma0 = 0: the projected point mass, whose triangle must be
    extracellular)."""
    Np = op.Np
    ext = np.repeat(op.extracellular, Np)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    cols = []
    for x0 in pts:
        if sigma0 == 0:
            u = project_dirac(op, x0)
            if np.abs(u[~ext]).max(initial=0.0) > 0:
                raise ValueError("the start point lies in an axon cell")
        else:
            u = project_gaussian(op, x0, sigma0)
            u[~ext] = 0.0
            u = u / moments(op, u[:, None], x0[None])[0, 0]
        cols.append(u)
    return np.stack(cols, axis=1)


def spectral_radius(op: MixedOperator) -> float:
    """Largest |eigenvalue| of L (ARPACK)."""
    return float(np.abs(sla.eigs(op.L, k=1, which="LM", return_eigenvectors=False, tol=1e-10)[0]))


def step_rule(op: MixedOperator) -> dict:
    """dt = 0.9 X / (1.01 rho), X the real stability limit of SSP-RK3 (the
    spectrum lies near the negative real axis)."""
    rho = spectral_radius(op)
    return {"dt_nom": 0.9 * X_RK3 / (1.01 * rho), "rho": rho}

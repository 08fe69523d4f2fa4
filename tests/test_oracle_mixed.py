"""Pins of the oracle's mixed form (eq. (6)-(7) with the fluxes of section
3.2, all pixels kept, k = 0 in the axon cells), on the CPU:

* a linear field has its exact gradient (the central u-flux lifting
  vanishes on continuous fields);
* the element mean of q next to an axon cell follows from the weak form
  with a constant test function: int_K q = sum over faces of {u} n |f|;
* with constant k the operator is M-symmetric and negative semi-definite
  with one zero mode; with axons the axon rows vanish and mass is kept;
* free-space covariance (sigma0^2 + 2 D t) I exactly for p >= 2;
* zero-flux box against the method-of-images moments, converging;
* the mixed and primal forms approach each other on a disk geometry.
"""

import math

import numpy as np
import pytest

from closed_forms import box_moments
from oracle import bounds, moments as mom, timeint
from oracle import mixed
from oracle import solve as osolve
from oracle.sipg import FACES

NO_DISKS = np.zeros((0, 3))


def _linear_coeffs(op, a, b, c):
    """Monomial coefficients of u = a + b x + c y on every element."""
    m = op.mesh
    h = m.h
    U = np.zeros((m.n_elements, op.Np))
    U[:, 0] = a + b * (m.cell_i + 0.5) * h + c * (m.cell_j + 0.5) * h
    U[:, 1] = b * h          # xi
    U[:, 2] = c * h          # eta
    return U.ravel()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_linear_field_exact_gradient(p):
    op = mixed.assemble_mixed(3.0, 6, NO_DISKS, p, 1.3)
    u = _linear_coeffs(op, 0.7, -1.9, 2.4)
    q = op.G @ u
    n = op.ndof
    qx = q[:n].reshape(-1, op.Np)
    qy = q[n:].reshape(-1, op.Np)
    tol = 1e-11           # rounding through the monomial mass inverse (P3: 2.5e-12)
    assert np.abs(qx[:, 0] + 1.9).max() < tol and np.abs(qx[:, 1:]).max() < tol
    assert np.abs(qy[:, 0] - 2.4).max() < tol and np.abs(qy[:, 1:]).max() < tol
    # div q = 0: elements away from the box (whose q-flux is zero) keep u
    ut = (op.L @ u).reshape(-1, op.Np)
    m = op.mesh
    inner = (m.nbr >= 0).all(axis=1)
    assert np.abs(ut[inner]).max() < 1e-12 * abs(op.L).max() * np.abs(u).max()


def test_element_mean_of_q_next_to_an_axon():
    """u = c on extracellular cells, 0 in axon cells: with the constant test
    function the weak form gives int_K q = sum_f {u}_f n_f |f| (the broken
    gradient integrates to zero), i.e. -(c/2) times the axon faces' n |f|."""
    disks = np.array([[1.5, 1.5, 0.45]])
    p, D, c = 2, 1.0, 0.8
    op = mixed.assemble_mixed(3.0, 6, disks, p, D)
    m = op.mesh
    h = m.h
    ext = op.extracellular
    u = np.zeros((m.n_elements, op.Np))
    u[ext, 0] = c
    q = op.G @ u.ravel()
    n = op.ndof
    W = [op.loc.Wmom[o][0] for o in (0, 1)]         # int psi_k over the triangle (h = 1)
    checked = 0
    for e in np.flatnonzero(ext):
        o = int(m.orient[e])
        want = np.zeros(2)
        for f in range(3):
            nb = m.nbr[e, f]
            if nb < 0:
                continue                              # box face: u-flux u- = c, cancels below
            nl = np.asarray(FACES[o][f][2])
            if not ext[nb]:
                want += -0.5 * c * nl * h
        got = np.array([W[o] @ q[:n].reshape(-1, op.Np)[e], W[o] @ q[n:].reshape(-1, op.Np)[e]]) * h * h
        assert np.abs(got - want).max() < 1e-12
        checked += int(np.abs(want).max() > 0)
    assert checked >= 4


@pytest.mark.parametrize("p", [1, 2])
def test_constant_k_symmetric_negative_one_zero_mode(p):
    op = mixed.assemble_mixed(2.0, 4, NO_DISKS, p, 1.0)
    ML = (op.M @ op.L).toarray()
    assert np.abs(ML - ML.T).max() < 1e-11 * np.abs(ML).max()
    ev = np.linalg.eigvalsh(0.5 * (ML + ML.T))
    assert ev.max() < 1e-9 * np.abs(ev).max()
    assert (np.abs(ev) < 1e-9 * np.abs(ev).max()).sum() == 1


@pytest.mark.parametrize("p", [1, 2, 3])
def test_axons_frozen_and_mass_kept(p):
    disks = np.array([[1.0, 1.1, 0.5], [2.3, 2.2, 0.4]])
    op = mixed.assemble_mixed(3.0, 8, disks, p, 2.0)
    Np = op.Np
    L = op.L.toarray()
    ax = np.repeat(~op.extracellular, Np)
    assert ax.sum() > 0
    assert np.abs(L[ax]).max() == 0.0
    # mass functional: int u = sum over elements of Wmom[o][0] . u_K h^2
    w = np.concatenate([op.loc.Wmom[int(o)][0] * op.mesh.h ** 2 for o in op.mesh.orient])
    assert np.abs(w @ L).max() < 1e-12 * np.abs(L).max()
    # constants everywhere (axons included) are stationary
    one = _linear_coeffs(op, 1.0, 0.0, 0.0)
    assert np.abs(L @ one).max() < 1e-11 * np.abs(L).max()


@pytest.mark.parametrize("p", [2, 3])
def test_free_space_covariance_exact(p):
    """Walls far away: moments of degree <= 2 evolve exactly, so
    Sigma = (sigma0^2 + 2 D t) I and the mean offset stays zero."""
    D, s0, t = 2.0, 0.3, 0.1
    op = mixed.assemble_mixed(12.0, 48, NO_DISKS, p, D)
    x0 = np.array([[6.02, 5.97]])
    U0 = mixed.initial_block(op, x0, s0)
    b = 1.01 * mixed.spectral_radius(op)
    r = timeint.expm_deltas(op.L, U0, [t], b, on_delta=lambda k, U: mom.moments(op, U, x0))[0][0]
    S = r[3:] / r[0]
    v = s0 * s0 + 2 * D * t
    assert abs(r[0] - 1) < 1e-12
    assert abs(S[0] - v) < 1e-9 and abs(S[2] - v) < 1e-9 and abs(S[1]) < 1e-9
    assert np.abs(r[1:3]).max() < 1e-9


@pytest.mark.parametrize("p,order", [(1, 1.5), (2, 2.5)])
def test_box_converges_to_images_solution(p, order):
    """Zero-flux box [0, 6]^2 (the u-flux on the edges is the inside
    value): Sigma_A against the method-of-images moments, observed order."""
    w, D, s0, t = 6.0, 2.0, 0.4, 1.0
    x0 = np.array([[2.7, 3.3]])
    ref = np.array(box_moments(w, x0[0], s0, D, t))
    errs = []
    for N in (12, 24, 48):
        op = mixed.assemble_mixed(w, N, NO_DISKS, p, D)
        U0 = mixed.initial_block(op, x0, s0)
        b = 1.01 * mixed.spectral_radius(op)
        r = timeint.expm_deltas(op.L, U0, [t], b, on_delta=lambda k, U: mom.moments(op, U, x0))[0][0]
        assert abs(r[0] - 1.0) < 1e-10
        errs.append(float(mom.rel_err(r[3:] / r[0], ref[3:] / ref[0])))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 1e-3
    assert min(rates) > order, (errs, rates)


def test_mixed_and_primal_forms_approach_each_other():
    """Same disk geometry, P2: the mixed form (all pixels, k = 0 in axons)
    and the primal form (axon cells removed) discretise the same problem;
    their Sigma difference falls as h halves, and both keep unit mass."""
    from scipy.sparse.linalg import expm_multiply
    L, D, s0, t = 4.0, 1.0, 0.25, 0.3
    disks = np.array([[2.0, 2.0, 1.1]])
    x0 = np.array([[0.7, 0.9]])
    diffs = []
    for N in (8, 16, 32):
        op = mixed.assemble_mixed(L, N, disks, 2, D)
        u = expm_multiply(op.L * t, mixed.initial_block(op, x0, s0)[:, 0])
        a = mom.moments(op, u[:, None], x0)[0]
        ps = osolve.prepare(L, N, disks, 2, D, 10.0)
        v = expm_multiply(ps.op.L * t, osolve.initial_block(ps.op, x0, s0)[:, 0])
        b = mom.moments(ps.op, v[:, None], x0)[0]
        assert abs(a[0] - 1) < 1e-10 and abs(b[0] - 1) < 1e-10      # expm_multiply rounding
        diffs.append(np.abs(a[3:] / a[0] - b[3:] / b[0]).max())
    assert diffs[1] < 0.8 * diffs[0] and diffs[2] < 0.8 * diffs[1], diffs


def test_step_rule_and_point_mass():
    disks = np.array([[1.5, 1.5, 0.6]])
    op = mixed.assemble_mixed(3.0, 12, disks, 2, 2.0)
    rule = mixed.step_rule(op)
    assert rule["dt_nom"] * rule["rho"] < bounds.X_RK3
    # the mixed form's spectrum is far below the penalised primal form's
    ps = osolve.prepare(3.0, 12, disks, 2, 2.0, 10.0)
    assert rule["rho"] < 0.2 * ps.dt["lambda_max"]
    U = mixed.initial_block(op, np.array([[0.4, 0.5]]), 0.0)
    r = mom.moments(op, U, np.array([[0.4, 0.5]]))[0]
    assert abs(r[0] - 1) < 1e-13 and np.abs(r[1:]).max() < 1e-13
    with pytest.raises(ValueError):
        mixed.initial_block(op, np.array([[1.5, 1.5]]), 0.0)

"""Pins of the oracle's absorbing outer box (u = 0 on the square's edges,
the paper's eq. (4)) and of the projected point mass (its Dirac pulse),
on the CPU: the lowest eigenvalue 2 D pi^2 / L^2 of the box, the survival
probability of a point mass in closed form (Fourier sine series), monotone
mass decay, and the exact low moments of the projected point mass."""

import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle import bounds, initial, mesh as meshmod, moments as mom, sipg, timeint

L, D = 4.0, 2.0


def _op(p, N, outer="absorb", disks=None):
    m = meshmod.build_mesh(L, N, np.zeros((0, 3)) if disks is None else disks)
    return sipg.assemble(m, p, D, 10.0, outer=outer)


def _lam_min(op):
    B = bounds.symmetric_operator(op)
    return float(sla.eigsh(B, k=1, sigma=0, which="LM", return_eigenvectors=False)[0])


def _survival_1d(a, t, n_terms=400):
    m = np.arange(1, 2 * n_terms, 2)
    return float((4.0 / (m * np.pi) * np.sin(m * np.pi * a / L)
                  * np.exp(-D * m ** 2 * np.pi ** 2 * t / L ** 2)).sum())


def test_absorbing_box_lowest_eigenvalue():
    """-D Laplacian with u = 0 on a square of side L: lowest eigenvalue
    2 D pi^2 / L^2; the SIPG discretisation converges to it at order 2p."""
    exact = 2.0 * D * np.pi ** 2 / L ** 2
    op = _op(3, 8)
    A = op.A.toarray()
    assert np.abs(A - A.T).max() < 1e-12 * np.abs(A).max()
    assert abs(_lam_min(op) / exact - 1) < 1e-6
    e8 = abs(_lam_min(_op(2, 8)) / exact - 1)
    e16 = abs(_lam_min(_op(2, 16)) / exact - 1)
    assert e8 / e16 > 2.0 ** 3.5
    # the zero-flux box keeps a zero eigenvalue (the constant)
    assert _lam_min(_op(2, 8, outer="reflect")) < 1e-9


def test_absorbing_box_survival_closed_form_and_decay():
    """Point mass at x0 in the absorbing box: M0(t) = S(x0) S(y0),
    S(a, t) = sum over odd m of 4/(m pi) sin(m pi a / L) exp(-D m^2 pi^2 t / L^2)."""
    x0 = np.array([1.3, 2.1])
    op = _op(3, 16)
    b = 1.01 * bounds.lambda_max(op)
    U0 = initial.project_dirac(op, x0)[:, None]
    ts = [0.05, 0.1, 0.3, 0.6, 1.0]
    M = timeint.expm_deltas(op.L, U0, ts, b,
                            on_delta=lambda k, U: mom.moments(op, U, x0[None])[0])
    m0 = np.array([r[0] for r in M])
    ref = np.array([_survival_1d(x0[0], t) * _survival_1d(x0[1], t) for t in ts])
    assert np.abs(m0[1:] - ref[1:]).max() < 2e-6
    assert (np.diff(m0) < 0).all() and m0[0] < 1.0


def test_absorbing_box_with_disks_mass_decays():
    """Disks touching the box edge remove box faces with their cells: the
    operator stays symmetric positive definite and the mass still decays."""
    disks = np.array([[0.2, 2.0, 0.6], [3.9, 1.0, 0.5], [2.0, 2.0, 0.7]])
    op = _op(2, 16, disks=disks)
    A = op.A.toarray()
    assert np.abs(A - A.T).max() < 1e-12 * np.abs(A).max()
    assert _lam_min(op) > 0.5
    b = 1.01 * bounds.lambda_max(op)
    x0 = np.array([[1.1, 3.0]])
    U0 = initial.project_dirac(op, x0[0])[:, None]
    M = timeint.expm_deltas(op.L, U0, [0.1, 0.2, 0.4], b,
                            on_delta=lambda k, U: mom.moments(op, U, x0)[0, 0])
    assert M[0] < 1.0 and M[1] < M[0] and M[2] < M[1]


@pytest.mark.parametrize("p", [1, 2, 3])
def test_projected_point_mass_moments(p):
    """int (Pi delta) v = v(x0) for every v of the space: unit mass, zero
    first moment about x0 (p >= 1), zero second moments (p >= 2)."""
    op = _op(p, 8, outer="reflect")
    x0 = np.array([[1.37, 2.61]])
    U = initial.project_dirac(op, x0[0])[:, None]
    M = mom.moments(op, U, x0)[0]
    assert abs(M[0] - 1) < 1e-13
    assert np.abs(M[1:3]).max() < 1e-13
    if p >= 2:
        assert np.abs(M[3:6]).max() < 1e-13
    # a point on a cell's diagonal lies in its T0 triangle
    h = op.mesh.h
    xd = np.array([(3 + 0.25) * h, (5 + 0.25) * h])
    Ud = initial.project_dirac(op, xd).reshape(op.mesh.n_elements, op.Np)
    e = np.flatnonzero(np.abs(Ud).sum(1) > 0)
    assert e.size == 1 and op.mesh.orient[e[0]] == 0


def test_point_mass_free_space_covariance():
    """Zero-flux box far away: the covariance of the spreading point mass is
    2 D t I exactly for p >= 2 (moments of degree <= 2 evolve exactly)."""
    m = meshmod.build_mesh(12.0, 48, np.zeros((0, 3)))
    op = sipg.assemble(m, 2, D, 10.0)
    b = 1.01 * bounds.lambda_max(op)
    x0 = np.array([[6.02, 5.97]])
    U0 = initial.project_dirac(op, x0[0])[:, None]
    t = 0.1                              # walls 9.5 standard deviations away
    M = timeint.expm_deltas(op.L, U0, [t], b, on_delta=lambda k, U: mom.moments(op, U, x0)[0])[0]
    S = mom.sigma_a(M)
    assert abs(S[0] - 2 * D * t) < 1e-9 and abs(S[2] - 2 * D * t) < 1e-9 and abs(S[1]) < 1e-9

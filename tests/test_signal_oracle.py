"""Pins of the oracle's q-space signal E(q) = int u exp(i q.(x - x0)) dx
(CPU): the mass at q = 0, conjugate symmetry, the small-q expansion against
the (separately pinned) moments, brute-force quadrature on one element, the
mirror symmetry of the mesh, and the free-space closed form."""

import numpy as np
from scipy import integrate

from oracle import bounds, mesh as meshmod, moments as mom, sipg
from oracle import signal as osig
from oracle import solve as osolve
from oracle import timeint

DISKS = np.array([[3.0, 2.0, 0.8], [5.5, 4.7, 0.7], [1.7, 6.1, 0.9]])
X0 = np.array([[4.2, 3.1], [2.6, 4.4]])


def _evolved(disks, x0, p=2, t=0.4, L=8.0, N=32):
    m = meshmod.build_mesh(L, N, disks)
    op = sipg.assemble(m, p, 2.0, 10.0)
    b = 1.01 * bounds.lambda_max(op)
    U0 = osolve.initial_block(op, x0, 0.3)
    U = timeint.expm_deltas(op.L, U0, [t], b, on_delta=lambda k, V: V.copy())[0]
    return op, U


def _qs(mags, n_dir=6, seed=0):
    ang = np.random.default_rng(seed).uniform(0, 2 * np.pi, n_dir)
    return np.array([[a * np.cos(th), a * np.sin(th)] for a in mags for th in ang])


def test_signal_mass_conjugate_and_small_q():
    op, U = _evolved(DISKS, X0)
    M = mom.moments(op, U, X0)                                   # [R, 6]
    E0 = osig.signal(op, U, X0, np.zeros((1, 2)))[:, 0]
    assert np.allclose(E0.real, M[:, 0], rtol=1e-14, atol=0)
    assert np.abs(E0.imag).max() == 0.0
    qs = _qs([0.7, 2.0])
    Ep = osig.signal(op, U, X0, qs)
    Em = osig.signal(op, U, X0, -qs)
    assert np.abs(Ep - np.conj(Em)).max() < 1e-14
    # E(eps u) = M0 + i eps u.m1 - eps^2 u^T M2 u / 2 + O(eps^3)
    eps = 1e-3
    dirs = _qs([1.0], n_dir=5, seed=3)
    Es = osig.signal(op, U, X0, eps * dirs)
    for r in range(X0.shape[0]):
        m1 = M[r, 1:3]
        M2 = np.array([[M[r, 3], M[r, 4]], [M[r, 4], M[r, 5]]])
        for k, u in enumerate(dirs):
            first = eps * (u @ m1)
            second = 0.5 * eps ** 2 * (u @ M2 @ u)
            assert abs(Es[r, k].imag - first) < 1e-4 * abs(first) + 1e-14
            assert abs((M[r, 0] - Es[r, k].real) - second) < 1e-4 * second


def test_signal_element_integral_brute_force():
    """One element, a random polynomial, |q| h ~ 2: the collapsed product
    rule against adaptive 2D quadrature of the real and imaginary parts."""
    m = meshmod.build_mesh(2.0, 4, np.zeros((0, 3)))
    op = sipg.assemble(m, 3, 2.0, 10.0)
    rng = np.random.default_rng(1)
    h = m.h
    for e in (3, 4):
        coef = rng.normal(size=op.Np)
        x0 = np.array([0.3, 1.7])
        q = np.array([2.9, -3.7])
        got = osig.element_integral(op, coef, e, x0, q)
        o = int(m.orient[e])
        xc, yc = (m.cell_i[e] + 0.5) * h, (m.cell_j[e] + 0.5) * h
        mons = sipg.monomials(op.p)

        def f(yy, xx, part):
            xi, et = (xx - xc) / h, (yy - yc) / h
            u = sum(c * xi ** a * et ** b for c, (a, b) in zip(coef, mons))
            ph = q[0] * (xx - x0[0]) + q[1] * (yy - x0[1])
            return u * (np.cos(ph) if part == 0 else np.sin(ph))

        x_lo, x_hi = xc - h / 2, xc + h / 2
        if o == 0:   # lower right: below the diagonal y - yc <= x - xc
            lo, hi = (lambda xx: yc - h / 2), (lambda xx: yc + (xx - xc))
        else:        # upper left
            lo, hi = (lambda xx: yc + (xx - xc)), (lambda xx: yc + h / 2)
        ref = [integrate.dblquad(f, x_lo, x_hi, lo, hi, args=(k,), epsabs=1e-15, epsrel=1e-13)[0]
               for k in (0, 1)]
        assert abs(got.real - ref[0]) < 1e-12 * (abs(ref[0]) + abs(ref[1]))
        assert abs(got.imag - ref[1]) < 1e-12 * (abs(ref[0]) + abs(ref[1]))


def test_signal_mirror_symmetry():
    """(x, y) -> (y, x) maps the mesh onto itself: E of the mirrored problem
    at (q_y, q_x) equals E at (q_x, q_y)."""
    qs = _qs([0.5, 1.5], n_dir=4, seed=5)
    op, U = _evolved(DISKS, X0[:1])
    opm, Um = _evolved(DISKS[:, [1, 0, 2]], X0[:1, [1, 0]])
    a = osig.signal(op, U, X0[:1], qs)
    b = osig.signal(opm, Um, X0[:1, [1, 0]], qs[:, [1, 0]])
    assert np.abs(a - b).max() < 1e-10 * np.abs(a).max()


def test_signal_free_space_gaussian():
    """Walls 6 um (6.4 standard deviations) away: the pulse stays a Gaussian
    of variance sigma0^2 + 2 D t per axis, E = exp(-|q|^2 (sigma0^2 + 2 D t)
    / 2), up to the discretisation error: P3 at h = 0.25 um within 5e-7 for
    |q| <= 2, and P2 converging at order > 3 when h halves."""
    x0 = np.array([[6.0, 6.0]])
    t = 0.2
    var = 0.3 ** 2 + 2 * 2.0 * t
    qs = _qs([0.5, 1.0, 2.0], n_dir=4, seed=7)
    ref = np.exp(-0.5 * (qs ** 2).sum(1) * var)
    op, U = _evolved(np.zeros((0, 3)), x0, p=3, t=t, L=12.0, N=48)
    assert np.abs(osig.signal(op, U, x0, qs)[0] - ref).max() < 5e-7
    err = []
    for N in (48, 96):
        op, U = _evolved(np.zeros((0, 3)), x0, p=2, t=t, L=12.0, N=N)
        err.append(np.abs(osig.signal(op, U, x0, qs)[0] - ref).max())
    assert err[0] / err[1] > 2.0 ** 3

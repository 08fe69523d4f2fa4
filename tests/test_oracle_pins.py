"""Pins of the FP64 oracle against what the mathematics and the paper fix.

Each test names the property it checks and why a plausible mistake in the
oracle (a dropped term, a wrong sign, index or normal, a transposed block,
a wrong RK coefficient, a wrong moment weight) would fail it.
"""

import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import bounds, initial, mesh as meshmod, moments as mom, poly, sipg, timeint
from oracle import solve as osolve
from tests.closed_forms import box_moments

NO_DISKS = np.zeros((0, 3))


# ---------------------------------------------------------------- poly ----

def test_poly_triangle_integrals_match_brute_quadrature():
    """Exact monomial integrals vs a fine midpoint rule on a sub-grid of the
    triangle (independent of the closed form m! n! / (m+n+2)!)."""
    rng = np.random.default_rng(0)
    verts = [(0.3, -0.2), (1.7, 0.4), (0.1, 1.3)]
    p = {(a, b): rng.standard_normal() for a in range(4) for b in range(4 - a)}
    exact = poly.integrate_triangle(p, *verts)
    # midpoint rule on n^2 sub-triangles of a uniform split
    n = 400
    v0, v1, v2 = (np.array(v) for v in verts)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = i + j < n
    r = (i[keep] + 1.0 / 3.0) / n
    s = (j[keep] + 1.0 / 3.0) / n
    up = (i + j < n - 1)
    r2 = (i[up] + 2.0 / 3.0) / n
    s2 = (j[up] + 2.0 / 3.0) / n
    R = np.concatenate([r, r2])
    S = np.concatenate([s, s2])
    X = v0[0] + R * (v1 - v0)[0] + S * (v2 - v0)[0]
    Y = v0[1] + R * (v1 - v0)[1] + S * (v2 - v0)[1]
    vals = sum(c * X ** a * Y ** b for (a, b), c in p.items())
    area = 0.5 * abs((v1 - v0)[0] * (v2 - v0)[1] - (v2 - v0)[0] * (v1 - v0)[1])
    brute = vals.sum() * area / n ** 2
    assert abs(exact - brute) < 1e-5 * max(1.0, abs(exact))


def test_poly_edge_integral_and_shift():
    p = {(2, 1): 1.5, (0, 3): -2.0, (1, 0): 0.5}
    q = poly.shift(p, 0.7, -0.3)
    for x, y in [(0.1, 0.2), (-1.0, 2.0)]:
        pv = sum(c * (x + 0.7) ** a * (y - 0.3) ** b for (a, b), c in p.items())
        qv = sum(c * x ** a * y ** b for (a, b), c in q.items())
        assert abs(pv - qv) < 1e-12
    # integral along a segment vs Simpson on 2001 points
    p0, p1 = (0.2, -0.4), (1.1, 0.9)
    t = np.linspace(0, 1, 2001)
    X = p0[0] + t * (p1[0] - p0[0])
    Y = p0[1] + t * (p1[1] - p0[1])
    f = sum(c * X ** a * Y ** b for (a, b), c in p.items())
    simpson = (f[0] + f[-1] + 4 * f[1:-1:2].sum() + 2 * f[2:-1:2].sum()) / (3 * 2000)
    assert abs(poly.integrate_edge_param(p, p0, p1) - simpson) < 1e-10


# ---------------------------------------------------------------- mesh ----

def test_mesh_cell_removal_hand_counted():
    """A disk centred on a cell centroid: neighbouring centroids sit at h,
    sqrt(2) h and 2 h, so radii just below / at / above those distances
    remove 1, 1, 5, 5, 9 cells (strict inequality: a centroid on the circle
    stays; h = 1 makes the boundary case exact in FP64)."""
    L, N = 8.0, 8
    h = L / N
    c = (3.5 * h, 4.5 * h)
    s2 = math.sqrt(2.0)
    for r, removed in [(0.999 * h, 1), (1.0 * h, 1), (1.001 * h, 5),
                       (0.999 * s2 * h, 5), (1.001 * s2 * h, 9)]:
        m = meshmod.build_mesh(L, N, np.array([[c[0], c[1], r]]))
        assert int((~m.active_cell).sum()) == removed, r
        assert m.n_elements == 2 * (N * N - removed)
    # face count on the free mesh: N^2 diagonals + 2 N (N-1) edges
    m = meshmod.build_mesh(L, N, NO_DISKS)
    assert m.n_interior_faces() == N * N + 2 * N * (N - 1)


def test_moments_of_a_polynomial_field():
    """The moment functional on a field known in closed form: the bilinear
    f(x, y) = (x - a)(y - b) + c lies in P2, so its modal coefficients are
    exact, and its moments over the box [0, w]^2 about x0 follow from 1D
    integrals int_0^w (x - x0)^k (x - a)^j dx.  Pins every moment weight
    and offset term, including the cross term of Mxy."""
    w, N = 3.0, 6
    a, b, c = 0.7, 2.1, 0.4
    x0 = np.array([[1.1, 1.9]])
    m = meshmod.build_mesh(w, N, NO_DISKS)
    op = sipg.assemble(m, 2, 1.0, 10.0)
    h = m.h
    U = np.zeros((m.n_elements, op.Np))
    mons = sipg.monomials(2)
    for e in range(m.n_elements):
        xc, yc = (m.cell_i[e] + 0.5) * h, (m.cell_j[e] + 0.5) * h
        # f in local coords: (h xi + xc - a)(h eta + yc - b) + c
        coef = {(0, 0): (xc - a) * (yc - b) + c, (1, 0): h * (yc - b),
                (0, 1): h * (xc - a), (1, 1): h * h}
        U[e] = [coef.get(mn, 0.0) for mn in mons]
    got = mom.moments(op, U.reshape(-1, 1), x0)[0]

    def I(k, j, s, t):       # int_0^w (x - s)^k (x - t)^j dx, exact by expansion
        xs = np.polynomial.polynomial
        pk = xs.polypow([-s, 1.0], k)
        pj = xs.polypow([-t, 1.0], j)
        q = xs.polyint(xs.polymul(pk, pj))
        return xs.polyval(w, q) - xs.polyval(0.0, q)

    X0, Y0 = x0[0]
    def moment(kx, ky):
        return I(kx, 1, X0, a) * I(ky, 1, Y0, b) + c * I(kx, 0, X0, 0) * I(ky, 0, Y0, 0)
    expect = [moment(0, 0), moment(1, 0), moment(0, 1), moment(2, 0), moment(1, 1), moment(0, 2)]
    assert np.allclose(got, expect, rtol=1e-13, atol=1e-13)


def _constant_vector(op):
    c = np.zeros((op.mesh.n_elements, op.Np))
    c[:, 0] = 1.0            # the constant function in the monomial basis
    return c.ravel()


# A line of disks cuts the 6 x 6 grid into two pieces.
SPLIT_DISKS = np.array([[(i + 0.5), 2.5, 0.55] for i in range(6)])


@pytest.mark.parametrize("p", [1, 2, 3])
def test_V1_V2_V3_constants_symmetry_coercivity(p):
    """V1: A annihilates constants and the pencil (A, M) has exactly one zero
    eigenvalue per connected component (a missing face term or a face on a
    removed cell breaks the count).  V2: A = A^T, M SPD (a wrong sign or a
    transposed neighbour block breaks symmetry).  V3: every other eigenvalue
    is positive (penalty sign and size)."""
    for disks, comps in [(np.array([[1.5, 2.5, 0.6], [4.2, 4.4, 0.7]]), None), (SPLIT_DISKS, 2)]:
        m = meshmod.build_mesh(6.0, 6, disks)
        ncomp = m.n_components()
        if comps is not None:
            assert ncomp == comps
        op = sipg.assemble(m, p, 1.7, 10.0)
        A = op.A.toarray()
        M = op.M.toarray()
        assert np.abs(A @ _constant_vector(op)).max() < 1e-12 * np.abs(A).max()
        assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
        assert np.linalg.eigvalsh(M).min() > 0
        ev = scipy.linalg.eigh(A, M, eigvals_only=True)
        scale = ev.max()
        nzero = int((np.abs(ev) < 1e-10 * scale).sum())
        assert nzero == ncomp
        assert ev[nzero:].min() > 1e-6 * scale


def test_V2_dot_product_on_larger_mesh():
    m = meshmod.build_mesh(10.0, 40, np.array([[3.0, 4.0, 1.1], [7.0, 6.5, 0.9]]))
    op = sipg.assemble(m, 2, 2.0, 10.0)
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal((2, op.ndof))
    a, b = v @ (op.A @ u), u @ (op.A @ v)
    assert abs(a - b) < 1e-12 * (abs(a) + abs(b))


# ------------------------------------------------------- free diffusion ----

@pytest.mark.parametrize("p", [2, 3])
def test_V5_V6_free_space_exact_covariance(p):
    """V5: for p >= 2 the quadratics lie in the space, so the L2 projection
    keeps Sigma(0) = sigma0^2 I and the symmetric form gives
    d/dt int x x^T u = 2 D M0 I up to wall terms; Sigma_A = (sigma0^2 + 2 D t) I
    holds to roundoff before the walls are reached.  V6: the first moment
    stays at zero.  (Chebyshev flow: the exact semi-discrete solution.)"""
    # walls stay >= 7.5 sigma away at the last time
    L, N, ts = (16.0, 64, [0.1, 0.25]) if p == 2 else (12.0, 48, [0.05, 0.12])
    D, s0 = 2.0, 0.3
    m = meshmod.build_mesh(L, N, NO_DISKS)
    op = sipg.assemble(m, p, D, 10.0)
    b = 1.01 * bounds.lambda_max(op)
    x0 = np.array([[L / 2 + 0.013, L / 2 - 0.021]])
    U0 = osolve.initial_block(op, x0, s0)
    res = [mom.moments(op, U0, x0)[0]]
    res += [r[0] for r in timeint.expm_deltas(op.L, U0, ts, b,
                                              on_delta=lambda k, U: mom.moments(op, U, x0))]
    for t, r in zip([0.0] + ts, res):
        expect = s0 * s0 + 2 * D * t
        assert abs(r[0] - 1.0) < 1e-11          # roundoff of ~10^3 recurrence terms
        assert abs(r[1]) < 1e-11 and abs(r[2]) < 1e-11
        sa = r[3:] / r[0]
        assert abs(sa[0] / expect - 1) < 1e-10
        assert abs(sa[2] / expect - 1) < 1e-10
        assert abs(sa[1]) < 1e-10 * expect


def test_V5_rk3_exact_on_quadratic_moments():
    """RK3 with the landing schedule maps int x x^T u exactly like the flow
    (a wrong Shu-Osher coefficient or a wrong dt_k breaks this)."""
    L, N, D, s0 = 8.0, 32, 2.0, 0.3
    m = meshmod.build_mesh(L, N, NO_DISKS)
    op = sipg.assemble(m, 2, D, 10.0)
    dt = bounds.dt_rule(op)
    x0 = np.array([[4.0 + 0.05, 4.0 - 0.03]])
    U0 = osolve.initial_block(op, x0, s0)
    deltas = [0.02, 0.05]
    res = timeint.rk3(op.L, U0, deltas, dt["dt_nom"], on_delta=lambda k, U: mom.moments(op, U, x0)[0])
    for t, r in zip(deltas, res):
        expect = s0 * s0 + 2 * D * t
        assert abs(r[0] - 1.0) < 1e-12
        assert abs(r[3] / r[0] / expect - 1) < 1e-10
        assert abs(r[5] / r[0] / expect - 1) < 1e-10


def test_paper_free_diffusion_value(golden_dir):
    """The paper's free-diffusion check (section 4.2): k = 450 um^2/s,
    T = 0.036 s gives 2 T k = 32.4 um^2 on the diagonal.  Our Gaussian start
    adds sigma0^2; subtracting it must give the paper's number."""
    with open(os.path.join(golden_dir, "paper_free_diffusion.json")) as f:
        g = json.load(f)
    D = g["k_um2_per_s"] * 1e-3            # um^2/ms
    T = g["T_s"] * 1e3                     # ms
    L, N, s0 = 80.0, 80, 0.3
    m = meshmod.build_mesh(L, N, NO_DISKS)
    op = sipg.assemble(m, 2, D, 10.0)
    b = 1.01 * bounds.lambda_max(op)
    x0 = np.array([[40.0, 40.0]])
    U0 = osolve.initial_block(op, x0, s0)
    r = timeint.expm_deltas(op.L, U0, [T], b, on_delta=lambda k, U: mom.moments(op, U, x0))[0][0]
    sa = r[3:] / r[0]
    assert abs(sa[0] - s0 * s0 - g["sigma_diag_analytic"]) < 1e-8
    assert abs(sa[2] - s0 * s0 - g["sigma_diag_analytic"]) < 1e-8
    assert abs(sa[1]) < 1e-8


# ------------------------------------------------------------- walls ----

@pytest.mark.parametrize("p,order", [(1, 1.8), (2, 2.8)])
def test_V7_box_converges_to_images_solution(p, order):
    """V7: zero-flux box [0, 6]^2 without disks (walls on grid lines).  The
    exact PDE moments come from the method of images; the DG error in
    Sigma_A must fall at an observed order of at least p + 1 (minus slack)."""
    w, D, s0, t = 6.0, 2.0, 0.4, 1.0
    x0 = np.array([[2.7, 3.3]])
    ref = np.array(box_moments(w, x0[0], s0, D, t))
    ref_sa = ref[3:] / ref[0]
    errs = []
    for N in (12, 24, 48):
        m = meshmod.build_mesh(w, N, NO_DISKS)
        op = sipg.assemble(m, p, D, 10.0)
        b = 1.01 * bounds.lambda_max(op)
        U0 = osolve.initial_block(op, x0, s0)
        r = timeint.expm_deltas(op.L, U0, [t], b, on_delta=lambda k, U: mom.moments(op, U, x0))[0][0]
        assert abs(r[0] - 1.0) < 1e-10         # roundoff of ~4k recurrence terms
        errs.append(float(mom.rel_err(r[3:] / r[0], ref_sa)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 1e-3
    assert min(rates) > order, (errs, rates)


def test_V7_channel_long_time_limit():
    """North-star channel limit: between parallel walls a distance w apart the
    per-point covariance across the channel tends to w^2 / 12 (uniform
    density).  Box [0, 4]^2, long time."""
    w, D = 4.0, 2.0
    m = meshmod.build_mesh(w, 16, NO_DISKS)
    op = sipg.assemble(m, 2, D, 10.0)
    b = 1.01 * bounds.lambda_max(op)
    x0 = np.array([[1.3, 2.9]])
    U0 = osolve.initial_block(op, x0, 0.3)
    r = timeint.expm_deltas(op.L, U0, [30.0], b, on_delta=lambda k, U: mom.moments(op, U, x0))[0]
    sb = mom.sigma_b(r)[0]
    assert abs(sb[0] - w * w / 12) < 1e-8
    assert abs(sb[2] - w * w / 12) < 1e-8
    assert abs(sb[1]) < 1e-8


def test_V4_mass_conserved_with_disks_rk3():
    """V4: zero flux on walls and antisymmetric face fluxes keep M0 = 1."""
    disks = np.array([[3.0, 3.0, 0.8], [5.2, 4.1, 0.6], [2.2, 6.0, 0.9]])
    m = meshmod.build_mesh(8.0, 32, disks)
    op = sipg.assemble(m, 1, 2.0, 10.0)
    dt = bounds.dt_rule(op)
    x0 = np.array([[4.1, 4.9], [6.3, 2.2]])
    U0 = osolve.initial_block(op, x0, 0.3)
    res = timeint.rk3(op.L, U0, [0.2, 0.5], dt["dt_nom"],
                      on_delta=lambda k, U: mom.moments(op, U, x0))
    for r in res:
        assert np.abs(r[:, 0] - 1.0).max() < 1e-12


def test_V8_mirror_transposes_sigma():
    """V8: with the main diagonal, (x, y) -> (y, x) maps the mesh to itself
    (T0 <-> T1), so transposing disks and start point transposes Sigma."""
    disks = np.array([[3.0, 2.0, 0.8], [5.5, 4.7, 0.7], [1.7, 6.1, 0.9]])
    x0 = np.array([[4.2, 3.1]])
    out = []
    for d, x in [(disks, x0), (disks[:, [1, 0, 2]], x0[:, [1, 0]])]:
        m = meshmod.build_mesh(8.0, 32, d)
        op = sipg.assemble(m, 2, 2.0, 10.0)
        b = 1.01 * bounds.lambda_max(op)
        U0 = osolve.initial_block(op, x, 0.3)
        out.append(timeint.expm_deltas(op.L, U0, [0.7], b,
                                       on_delta=lambda k, U: mom.moments(op, U, x))[0][0])
    a, t = out
    tol = 1e-10                              # roundoff of the Chebyshev recurrence
    assert abs(a[0] - t[0]) < tol
    assert abs(a[1] - t[2]) < tol * abs(a[1]) and abs(a[2] - t[1]) < tol * abs(a[2])
    assert abs(a[3] - t[5]) < tol * abs(a[3])
    assert abs(a[5] - t[3]) < tol * abs(a[5])
    assert abs(a[4] - t[4]) < tol * abs(a[3])


# -------------------------------------------------- brute force, tiny ----

def test_V9_rk3_and_cheb_vs_dense_eigendecomposition():
    """V9: on a tiny mesh with removed cells, n RK3 steps equal
    R(dt L)^n u0 with R(z) = 1 + z + z^2/2 + z^3/6 applied through a dense
    eigendecomposition, and the Chebyshev flow equals the dense exponential."""
    disks = np.array([[1.5, 2.5, 0.6], [3.7, 1.2, 0.5]])
    m = meshmod.build_mesh(5.0, 5, disks)
    op = sipg.assemble(m, 2, 2.0, 10.0)
    A, M = op.A.toarray(), op.M.toarray()
    lam, V = scipy.linalg.eigh(A, M)      # V^T M V = I, A V = M V diag(lam)
    x0 = np.array([[2.6, 3.4]])
    u0 = osolve.initial_block(op, x0, 0.4)[:, 0]
    dt = bounds.dt_rule(op, lam=float(lam[-1]))
    n, dtk = bounds.schedule([0.03], dt["dt_nom"])[0]
    z = -dtk * lam
    R = 1 + z + z * z / 2 + z ** 3 / 6
    c = V.T @ (M @ u0)
    expect = V @ (R ** n * c)
    got = timeint.rk3(op.L, u0[:, None], [0.03], dt["dt_nom"])[0][:, 0]
    assert np.abs(got - expect).max() < 1e-12 * np.abs(expect).max()
    cheb = timeint.expm_cheb(op.L, u0[:, None], 0.03, 1.01 * lam[-1])[:, 0]
    exact = V @ (np.exp(-0.03 * lam) * c)
    assert np.abs(cheb - exact).max() < 1e-12 * np.abs(exact).max()


def test_V12_stability_constant_and_dt_rule():
    """V12: the SSP-RK3 real stability limit satisfies R(-X) = -1 with
    |R(-x)| <= 1 on [0, X]; the chosen dt keeps dt * lambda_max below it."""
    X = bounds.X_RK3
    R = lambda x: 1 - x + x * x / 2 - x ** 3 / 6  # noqa: E731
    assert abs(R(X) + 1) < 1e-13
    xs = np.linspace(0, X, 10001)
    assert np.abs(R(xs)).max() <= 1 + 1e-12
    assert abs(R(X * 1.001)) > 1
    m = meshmod.build_mesh(8.0, 16, np.array([[3.0, 3.0, 0.8]]))
    for p in (1, 2, 3):
        op = sipg.assemble(m, p, 2.0, 10.0)
        d = bounds.dt_rule(op)
        lam = float(scipy.linalg.eigh(op.A.toarray(), op.M.toarray(), eigvals_only=True)[-1])
        assert d["dt_nom"] * lam <= X
        assert d["rule"] == "stability"      # the workload formula alone is unstable


def test_V13_chebyshev_matches_rk3_on_small_workload():
    """V13: the exponential integrator and RK3 agree on Sigma to 1e-9 on the
    small workload's mesh (RK3 time error is negligible for the modes that
    carry Sigma)."""
    from workloads import config, make_geometry, start_points
    c = config("box20-p1")
    g = make_geometry(c["L"], c["N"], c["geom_seed"], n_disks=c["n_disks"])
    pts = start_points(g.disks, g.L, g.N, 1, np.random.default_rng(c["point_seed"]))
    prob = osolve.prepare(g.L, g.N, g.disks, c["p"], c["D"], c["eta"])
    deltas = [0.25, 0.5]
    a = osolve.solve(prob, pts, c["sigma0"], deltas, method="rk3")
    b = osolve.solve(prob, pts, c["sigma0"], deltas, method="cheb")
    err = mom.rel_err(mom.sigma_a(a), mom.sigma_a(b))
    assert err.max() < 1e-9, err


# ------------------------------------------------------ penalty size ----

@pytest.mark.parametrize("outer", ["reflect", "absorb"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_penalty_magnitude_checkerboard(p, outer):
    """Reading R2 fixes sigma_F = eta p^2 D / h with h the cell edge on all
    three face types.  On a disk-free N x N mesh take u = +1 on every T0 and
    -1 on every T1: grad u = 0, so only the penalty survives, and [u] = +-2
    on every interior face: u^T A u = sigma * 4 * (total interior face
    length) = 4 eta p^2 D (sqrt(2) N^2 + 2 N (N - 1)), with N^2 diagonals of
    length sqrt(2) h and 2 N (N - 1) edges of length h.  With the absorbing
    box each of the 4 N box faces adds sigma * h * 1^2.  u^T M u = N^2 h^2.
    p instead of p^2, a missing D, the diagonal without its sqrt(2) length,
    or h/sqrt(2) on the diagonal each move the quotient."""
    N, L, D, eta = 5, 3.0, 1.7, 10.0
    h = L / N
    m = meshmod.build_mesh(L, N, NO_DISKS)
    op = sipg.assemble(m, p, D, eta, outer=outer)
    u = np.zeros((m.n_elements, op.Np))
    u[:, 0] = np.where(m.orient == 0, 1.0, -1.0)      # constants in the monomial basis
    u = u.ravel()
    num = 4.0 * eta * p * p * D * (math.sqrt(2.0) * N * N + 2.0 * N * (N - 1))
    if outer == "absorb":
        num += 4.0 * N * eta * p * p * D
    expect = num / (N * N * h * h)
    got = (u @ (op.A @ u)) / (u @ (op.M @ u))
    assert abs(got - expect) < 1e-12 * expect


# ------------------------------------------------------------ mixture ----

def test_mixture_hand_computed_two_points():
    """Section 4.1's three covariance readings on a two-point case worked by
    hand.  Point 1: M0 = 1, m1 = (1, 0), M2 = (2, 0, 1) -> Sigma_A = (2, 0, 1),
    mu = (1, 0), Sigma_B = (1, 0, 1).  Point 2: M0 = 2, m1 = (0, 2),
    M2 = (2, 2, 6) -> Sigma_A = (1, 1, 3), mu = (0, 1), Sigma_B = (1, 1, 2).
    A = (1.5, 0.5, 2), B = (1, 0.5, 1.5), mubar = (0.5, 0.5),
    C = A - mubar mubar^T = (1.25, 0.25, 1.75)."""
    mom_ = np.array([[1.0, 1.0, 0.0, 2.0, 0.0, 1.0],
                     [2.0, 0.0, 2.0, 2.0, 2.0, 6.0]])
    r = mom.mixture(mom_)
    assert np.allclose(r["A"], [1.5, 0.5, 2.0], rtol=0, atol=1e-15)
    assert np.allclose(r["B"], [1.0, 0.5, 1.5], rtol=0, atol=1e-15)
    assert np.allclose(r["C"], [1.25, 0.25, 1.75], rtol=0, atol=1e-15)


def test_mixture_matches_pooled_sample_covariance():
    """Brute force: each start point x_i carries a weighted point cloud y_ik
    (weights w_ik, total mass M0_i).  Its moments about x_i feed ``mixture``;
    the same readings follow from numpy's weighted covariance: B is the mean
    of the per-point covariances, and C is the covariance of the pooled
    displacements y_ik - x_i with weights w_ik / (m M0_i) (the equal-weight
    mixture of the centred densities, about its own mean).  A swapped
    cross-moment, a missing M0 normalisation or a mean taken before
    centring fails it."""
    rng = np.random.default_rng(7)
    m, k = 5, 40
    x0 = rng.uniform(0, 10, (m, 2))
    moms, covs, pooled, pw = [], [], [], []
    for i in range(m):
        y = x0[i] + rng.normal(size=(k, 2)) * rng.uniform(0.5, 2.0, 2) + rng.uniform(-1, 1, 2)
        w = rng.uniform(0.1, 1.0, k) * rng.uniform(0.5, 2.0)
        d = y - x0[i]
        M0 = w.sum()
        moms.append([M0, (w * d[:, 0]).sum(), (w * d[:, 1]).sum(), (w * d[:, 0] ** 2).sum(),
                     (w * d[:, 0] * d[:, 1]).sum(), (w * d[:, 1] ** 2).sum()])
        covs.append(np.cov(d.T, aweights=w, bias=True))
        pooled.append(d)
        pw.append(w / (m * M0))
    r = mom.mixture(np.array(moms))
    B = np.mean(covs, axis=0)
    C = np.cov(np.concatenate(pooled).T, aweights=np.concatenate(pw), bias=True)
    sa = np.array([[mm[3] / mm[0], mm[4] / mm[0], mm[5] / mm[0]] for mm in moms]).mean(0)
    assert np.allclose(r["A"], sa, rtol=1e-13)
    assert np.allclose(r["B"], [B[0, 0], B[0, 1], B[1, 1]], rtol=1e-12, atol=1e-13)
    assert np.allclose(r["C"], [C[0, 0], C[0, 1], C[1, 1]], rtol=1e-12, atol=1e-13)

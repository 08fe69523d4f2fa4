"""GPU parity of the absorbing outer box (u = 0 on the square's edges, eq.
(4)) and of the projected point mass (the Dirac pulse of section 2.1)
against the oracle, through the C-ABI:

* the dense operator with box faces (VALU and packed kernels, FP64 and FP32)
  against the oracle's -M^-1 A after the change of basis;
* point mass + absorbing box, FP64 RK3 against the oracle's RK3 on the
  same step schedule (moments to 1e-10), and the batch path on two meshes;
* FP32 RK3 against the oracle's exact flow, and the survival probability of
  a point mass in an empty absorbing box against its closed form;
* the point mass right after creation: the GPU's initial state equals the
  oracle's projection, with unit mass and zero first moments;
* the Chebyshev exponential with the absorbing box, and the error paths.
"""

import sys

import numpy as np
import pytest

from oracle import initial as oinit, mesh as omesh, moments as omom, sipg
from oracle import solve as osolve
from oracle import timeint
from workloads import make_geometry, start_points

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dgd():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1907_06191_amd import dgd as d
    return d


def _nodal_transform(op_o, nodes):
    """T[o][i][k] = psi_k(node_i): oracle monomials (centred cell frame) to
    nodal values at the library's nodes."""
    mons = sipg.monomials(op_o.p)
    out = []
    for o in (0, 1):
        xi = nodes[o, :, 0] - 0.5
        et = nodes[o, :, 1] - 0.5
        out.append(np.stack([xi ** a * et ** b for (a, b) in mons], axis=1))
    return out


def _block_transform(mesh, m, oo, nodes, npn):
    """Block change of basis library <- oracle and the element map."""
    ci, cj, ori = mesh.elements()
    key = {(int(a), int(b), int(c)): e for e, (a, b, c) in enumerate(zip(m.cell_i, m.cell_j, m.orient))}
    perm = np.array([key[(int(a), int(b), int(c))] for a, b, c in zip(ci, cj, ori)])
    T = _nodal_transform(oo, nodes)
    E = m.n_elements
    Tb = np.zeros((E * npn, E * npn))
    for e in range(E):
        oe = perm[e]
        Tb[e * npn:(e + 1) * npn, oe * npn:(oe + 1) * npn] = T[int(ori[e])]
    return Tb


# disks touching the edges (cells and their box faces removed) and one inside
DISKS = np.array([[0.3, 2.5, 0.7], [4.2, 4.4, 0.7], [5.6, 0.4, 0.5]])


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n_rhs", ["all", 8])
def test_absorbing_operator_extraction(dgd, p, prec, n_rhs):
    """Apply the absorbing operator to every unit vector: as one block of
    all columns (one-element-per-wave kernel) and in blocks of 8 columns
    (several elements per wave); compare with the oracle's matrix."""
    import torch
    say(f"absorbing operator extraction p={p} {prec} rhs={n_rhs}")
    L, N, D = 6.0, 6, 1.7
    mesh = dgd.Mesh(L, N, DISKS)
    pr = dgd.DGD_FP64 if prec == "fp64" else dgd.DGD_FP32
    op = dgd.Operator(mesh, p, D, 10.0, pr, dt_max_ms=1e-3, outer=dgd.DGD_OUTER_ABSORB)
    npn, nodes, _ = op.info()
    m = omesh.build_mesh(L, N, DISKS)
    oo = sipg.assemble(m, p, D, 10.0, outer="absorb")
    n = m.n_elements * npn
    dtype = torch.float64 if prec == "fp64" else torch.float32
    eye = torch.eye(n, dtype=dtype, device="cuda")
    if n_rhs == "all":
        y = torch.zeros_like(eye)
        op.apply(eye, y, n)
        Lg = y
    else:
        cols = []
        for c0 in range(0, n, n_rhs):
            w = min(n_rhs, n - c0)
            x = eye[:, c0:c0 + w].contiguous()
            y = torch.zeros_like(x)
            op.apply(x, y, w)
            cols.append(y)
        Lg = torch.cat(cols, dim=1)
    torch.cuda.synchronize()
    Lg = Lg.double().cpu().numpy()
    Tb = _block_transform(mesh, m, oo, nodes, npn)
    Lref = Tb @ oo.L.toarray() @ np.linalg.inv(Tb)
    scale = np.abs(Lref).max()
    tol = (1e-12 if p < 3 else 1e-10) if prec == "fp64" else 1e-6
    err = np.abs(Lg - Lref).max() / scale
    # the box terms are present: the reflecting operator differs by O(1)
    ref_reflect = Tb @ sipg.assemble(m, p, D, 10.0).L.toarray() @ np.linalg.inv(Tb)
    say(f"  max |L_gpu - L_oracle| / max|L| = {err:.2e}; "
        f"vs reflecting {np.abs(Lg - ref_reflect).max() / scale:.2e}")
    assert err < tol
    assert np.abs(Lg - ref_reflect).max() / scale > 1e-2


def _dirac_case(nrhs, N, seed, phi=0.55):
    h = 100.0 / 512
    g = make_geometry(N * h, N, 19070619 + 1300 + seed, phi=phi)
    pts = start_points(g.disks, g.L, g.N, nrhs, np.random.default_rng(19070619 + 1301 + seed))
    return g, pts


@pytest.mark.parametrize("p", [1, 2, 3])
def test_point_mass_absorbing_rk3_fp64(dgd, p):
    """Point mass, absorbing box, FP64 state: the same RK3 step schedule as
    the oracle; moments (mass included) to 1e-10 of the largest."""
    g, pts = _dirac_case(4, 24, p)
    deltas = [0.02, 0.1, 0.3]
    prob = osolve.prepare(g.L, g.N, g.disks, p, 2.0, 10.0, outer="absorb")
    dt = prob.dt["dt_nom"]
    say(f"point mass absorbing FP64 p={p}: {prob.op.mesh.n_elements} elements, dt={dt:.3e}")
    ref = osolve.solve(prob, pts, 0.0, deltas, method="rk3")          # [R, nDelta, 6]
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, p, 2.0, 10.0, dgd.DGD_FP64, dt_max_ms=dt, outer=dgd.DGD_OUTER_ABSORB)
    sig, mom = op.solve(pts, 0.0, deltas)
    err = np.abs(mom - ref).max() / np.abs(ref).max()
    say(f"  max moment err {err:.2e}; mass at last Delta {mom[:, -1, 0]}")
    assert err < 1e-10
    assert omom.rel_err(sig, omom.sigma_a(ref)).max() < 1e-9
    assert (mom[:, -1, 0] < 1.0).all()


def test_point_mass_initial_state_matches_oracle(dgd):
    """The state right after creation (sigma0 = 0) against the oracle's
    projected point mass, mapped to nodal values; a point on a cell's
    diagonal goes to the T0 triangle on both sides."""
    g, pts = _dirac_case(3, 16, 11)
    h = g.L / g.N
    # a start point exactly on the diagonal of an active cell
    ci, cj = np.nonzero(np.ones((g.N, g.N)))
    for i, j in zip(ci, cj):
        c = np.array([(i + 0.25) * h, (j + 0.25) * h])
        if (np.hypot(g.disks[:, 0] - (i + 0.5) * h, g.disks[:, 1] - (j + 0.5) * h) >= g.disks[:, 2]).all():
            pts = np.vstack([pts, c])
            break
    for p in (1, 2, 3):
        mesh = dgd.Mesh(g.L, g.N, g.disks)
        op = dgd.Operator(mesh, p, 2.0, 10.0, dgd.DGD_FP64, dt_max_ms=1e-4,
                          outer=dgd.DGD_OUTER_ABSORB)
        npn, nodes, _ = op.info()
        m = omesh.build_mesh(g.L, g.N, g.disks)
        oo = sipg.assemble(m, p, 2.0, 10.0, outer="absorb")
        Tb = _block_transform(mesh, m, oo, nodes, npn)
        run = dgd.Run(op, pts, 0.0)
        R = pts.shape[0]
        U = dgd.dgd_run_get_state(run.handle, m.n_elements * npn * R, np.float64).reshape(-1, R)
        mom = run.moments()
        run.close()
        ref = np.stack([Tb @ oinit.project_dirac(oo, x) for x in pts], axis=1)
        err = np.abs(U - ref).max() / np.abs(ref).max()
        say(f"point mass initial state p={p}: err {err:.2e}")
        # the test's monomial-to-nodal change of basis loses ~1e-11 at p = 3
        assert err < (1e-12 if p < 3 else 1e-10)
        assert np.abs(mom[:, 0] - 1).max() < 1e-13
        assert np.abs(mom[:, 1:3]).max() < 1e-13


def test_point_mass_survival_closed_form(dgd):
    """Empty absorbing box, point mass, FP32 state on P3 (RK3): the mass
    against S(x0, t) S(y0, t), S(a, t) = sum over odd m of
    4 / (m pi) sin(m pi a / L) exp(-D m^2 pi^2 t / L^2)."""
    L, N, D = 4.0, 16, 2.0
    x0 = np.array([[1.3, 2.1], [2.0, 2.0], [0.6, 3.3]])
    ts = [0.1, 0.3, 0.6]

    def surv(a, t):
        k = np.arange(1, 800, 2)
        return float((4.0 / (k * np.pi) * np.sin(k * np.pi * a / L)
                      * np.exp(-D * k ** 2 * np.pi ** 2 * t / L ** 2)).sum())

    mesh = dgd.Mesh(L, N, np.zeros((0, 3)))
    op = dgd.Operator(mesh, 3, D, 10.0, dgd.DGD_FP32, outer=dgd.DGD_OUTER_ABSORB)
    say(f"survival closed form: dt={op.dt:.3e}")
    sig, mom = op.solve(x0, 0.0, ts)
    ref = np.array([[surv(a, t) * surv(b, t) for t in ts] for a, b in x0])
    err = np.abs(mom[..., 0] - ref).max()
    say(f"  max |M0 - S S| = {err:.2e}")
    assert err < 1e-5


def test_point_mass_absorbing_fp32_vs_exact_flow(dgd):
    """FP32 state, P2, absorbing box on a dense packing: moments within
    1e-5 (absolute; M0 <= 1) of the oracle's exact flow."""
    g, pts = _dirac_case(8, 48, 21, phi=0.6)
    deltas = [0.1, 0.4]
    prob = osolve.prepare(g.L, g.N, g.disks, 2, 2.0, 10.0, outer="absorb")
    dt = prob.dt["dt_nom"]
    say(f"point mass absorbing FP32 P2: {prob.op.mesh.n_elements} elements, dt={dt:.3e}")
    ref = osolve.solve(prob, pts, 0.0, deltas, method="cheb")
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, 2, 2.0, 10.0, dgd.DGD_FP32, dt_max_ms=dt, outer=dgd.DGD_OUTER_ABSORB)
    sig, mom = op.solve(pts, 0.0, deltas)
    err = np.abs(mom - ref).max()
    say(f"  max |moments - oracle| = {err:.2e}")
    assert err < 1e-5


def test_expm_absorbing_matches_oracle(dgd):
    """Chebyshev exponential (FP64 state) with the absorbing box and a
    Gaussian pulse against the oracle's exponential."""
    g, pts = _dirac_case(4, 32, 41)
    deltas = [0.1, 0.5]
    prob = osolve.prepare(g.L, g.N, g.disks, 2, 2.0, 10.0, outer="absorb")
    ref = osolve.solve(prob, pts, 0.3, deltas, method="cheb")
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, 2, 2.0, 10.0, dgd.DGD_FP64, outer=dgd.DGD_OUTER_ABSORB)
    sig, mom, napp = dgd.dgd_eap_solve_expm(op.handle, pts, 0.3, deltas)
    err = np.abs(mom - ref).max() / np.abs(ref).max()
    say(f"expm absorbing: {napp} applications, max moment err {err:.2e}")
    assert err < 1e-10


def test_batch_point_mass_absorbing(dgd):
    """Two meshes in one batch, point mass, absorbing box, FP64: the
    moments of each geometry match its own plain run to 1e-12 (same
    element order and per-element arithmetic) and the oracle's RK3 to
    1e-10; a batch mixing outer conditions is rejected."""
    runs = []
    for s in (52, 53):
        g, pts = _dirac_case(3, 20, s)
        runs.append((g, pts))
    meshes = [dgd.Mesh(g.L, g.N, g.disks) for g, _ in runs]
    ops = [dgd.Operator(mh, 2, 2.0, 10.0, dgd.DGD_FP64, dt_max_ms=2e-5, outer=dgd.DGD_OUTER_ABSORB)
           for mh in meshes]
    pts = np.stack([p for _, p in runs])
    deltas = [0.02, 0.06]
    bsig, bmom = dgd.dgd_eap_solve_batch(ops, pts, 0.0, deltas)
    for k, (o, (g, p)) in enumerate(zip(ops, runs)):
        sig, mom = o.solve(p, 0.0, deltas)
        err = np.abs(bmom[k] - mom).max()
        prob = osolve.prepare(g.L, g.N, g.disks, 2, 2.0, 10.0, outer="absorb")
        ref = osolve.solve(prob, p, 0.0, deltas, method="rk3", dt_nom=2e-5)
        err_o = np.abs(bmom[k] - ref).max() / np.abs(ref).max()
        say(f"batch geometry {k}: max |moments batch - plain| {err:.2e}, vs oracle {err_o:.2e}")
        assert err < 1e-12
        assert err_o < 1e-10
    mixed = dgd.Operator(meshes[1], 2, 2.0, 10.0, dgd.DGD_FP64, dt_max_ms=2e-5)
    with pytest.raises(dgd.DGDError) as e:
        dgd.dgd_eap_solve_batch([ops[0], mixed], pts, 0.0, deltas)
    assert e.value.code == dgd.DGD_EINVAL


def test_absorbing_errors(dgd):
    g, pts = _dirac_case(2, 16, 61)
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    with pytest.raises(dgd.DGDError) as e:
        dgd.Operator(mesh, 2, 2.0, 10.0, dgd.DGD_FP64, outer=7)
    assert e.value.code == dgd.DGD_EINVAL
    op = dgd.Operator(mesh, 2, 2.0, 10.0, dgd.DGD_FP64, dt_max_ms=1e-4)
    with pytest.raises(dgd.DGDError) as e:
        op.solve(pts, -0.1, [0.01])
    assert e.value.code == dgd.DGD_EINVAL
    # a start point in a removed cell
    d = g.disks[0]
    with pytest.raises(dgd.DGDError) as e:
        op.solve(np.array([[d[0], d[1]]]), 0.0, [0.01])
    assert e.value.code == dgd.DGD_ENOTFREE

"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Every case prints what it runs (flushed) before touching the GPU.
Tolerances: FP64 paths 1e-10 relative on Sigma (Frobenius norm of the 2x2
difference over the norm of the oracle's Sigma); FP32 paths 1e-4.
"""

import sys

import numpy as np
import pytest

from oracle import bounds, mesh as omesh, moments as omom, sipg
from oracle import solve as osolve
from oracle import timeint
from workloads import config, make_geometry, start_points

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
    """Block change of basis from the oracle's monomials in the centred cell
    frame to nodal values at the library's nodes: T[o][i][k] = psi_k(node_i)."""
    mons = sipg.monomials(op_o.p)
    T = []
    for o in (0, 1):
        xi = nodes[o, :, 0] - 0.5
        et = nodes[o, :, 1] - 0.5
        T.append(np.stack([xi ** a * et ** b for (a, b) in mons], axis=1))
    return T


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_V10_operator_extraction(dgd, p, prec):
    """V10: apply the GPU operator to every unit vector and compare the dense
    nodal matrix with the oracle's -M^-1 A after the change of basis."""
    import torch
    say(f"V10 operator extraction p={p} {prec}")
    disks = np.array([[1.5, 2.5, 0.6], [4.2, 4.4, 0.7], [5.6, 0.4, 0.5]])
    L, N, D = 6.0, 6, 1.7
    mesh = dgd.Mesh(L, N, disks)
    pr = dgd.DGD_FP64 if prec == "fp64" else dgd.DGD_FP32
    op = dgd.Operator(mesh, p, D, 10.0, pr, dt_max_ms=1e-3)
    npn, nodes, _ = op.info()
    m = omesh.build_mesh(L, N, disks)
    oo = sipg.assemble(m, p, D, 10.0)
    E = m.n_elements
    n = E * npn
    dtype = torch.float64 if prec == "fp64" else torch.float32
    x = torch.eye(n, dtype=dtype, device="cuda")
    y = torch.zeros_like(x)
    op.apply(x, y, n)
    torch.cuda.synchronize()
    Lg = y.double().cpu().numpy()
    # element map library -> oracle
    ci, cj, ori = mesh.elements()
    key = {(int(a), int(b), int(c)): e for e, (a, b, c) in enumerate(zip(m.cell_i, m.cell_j, m.orient))}
    perm = np.array([key[(int(a), int(b), int(c))] for a, b, c in zip(ci, cj, ori)])
    T = _nodal_transform(oo, nodes)
    Tb = np.zeros((n, n))
    for e in range(E):
        oe = perm[e]
        Tb[e * npn:(e + 1) * npn, oe * npn:(oe + 1) * npn] = T[int(ori[e])]
    Lo = oo.L.toarray()
    Lref = Tb @ Lo @ np.linalg.inv(Tb)
    scale = np.abs(Lref).max()
    # FP64: the monomial-to-nodal change of basis of this test loses ~1e-11 at p = 3
    tol = (1e-12 if p < 3 else 1e-10) if prec == "fp64" else 1e-6
    err = np.abs(Lg - Lref).max() / scale
    say(f"  max |L_gpu - L_oracle| / max|L| = {err:.2e}")
    assert err < tol


def _c1_setup():
    c = config("box20-p1")
    g = make_geometry(c["L"], c["N"], c["geom_seed"], n_disks=c["n_disks"])
    pts = start_points(g.disks, g.L, g.N, 1, np.random.default_rng(c["point_seed"]))
    return c, g, pts


def test_c1_parity_fp64(dgd):
    """Small workload in full: P1 FP64 on the 64^2 grid, Delta = 1, 2, 5 ms,
    the oracle's RK3 with the identical step schedule; 1e-10 on Sigma."""
    c, g, pts = _c1_setup()
    prob = osolve.prepare(g.L, g.N, g.disks, c["p"], c["D"], c["eta"])
    dt = prob.dt["dt_nom"]
    say(f"box20-p1 parity FP64: {prob.op.mesh.n_elements} elements, dt={dt:.4e} ms")
    ref = osolve.solve(prob, pts, c["sigma0"], c["deltas"], method="rk3")
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, c["p"], c["D"], c["eta"], dgd.DGD_FP64, dt_max_ms=dt)
    assert op.dt == dt
    sig, mom = op.solve(pts, c["sigma0"], c["deltas"])
    err = omom.rel_err(sig, omom.sigma_a(ref))
    say(f"  rel err per Delta {err.ravel()}; mass {mom[..., 0].ravel()}")
    assert err.max() < 1e-10
    assert np.abs(mom[..., 0] - 1).max() < 1e-12
    assert np.abs(mom - ref).max() < 1e-9 * np.abs(ref).max()


def _small_dense_case(nrhs=8, N=64, seed=7):
    """A 12.5 um box at the 512-grid spacing (h = 100/512) and packing 0.6."""
    h = 100.0 / 512
    L = N * h
    g = make_geometry(L, N, 19070619 + 900 + seed, phi=0.6)
    pts = start_points(g.disks, g.L, g.N, nrhs, np.random.default_rng(19070619 + 901 + seed))
    return g, pts


@pytest.mark.parametrize("p", [1, 2])
def test_fp32_parity_dense_packing(dgd, p):
    """FP32 state and operator, FP64 moments, on a dense packing at the 512-grid
    grid spacing: Sigma within 1e-4 of the oracle's exact flow (Chebyshev)
    at Delta = 0.5 and 1 ms (about 22k and 44k RK3 steps for P2)."""
    g, pts = _small_dense_case()
    deltas = [0.5, 1.0]
    prob = osolve.prepare(g.L, g.N, g.disks, p, 2.0, 10.0)
    dt = prob.dt["dt_nom"]
    say(f"FP32 parity p={p}: {prob.op.mesh.n_elements} elements, dt={dt:.3e}")
    ref = osolve.solve(prob, pts, 0.3, deltas, method="cheb")
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, p, 2.0, 10.0, dgd.DGD_FP32, dt_max_ms=dt)
    sig, mom = op.solve(pts, 0.3, deltas)
    err = omom.rel_err(sig, omom.sigma_a(ref))
    say(f"  max rel err {err.max():.2e}, max |M0-1| {np.abs(mom[..., 0] - 1).max():.2e}")
    assert err.max() < 1e-4


def _near_wall_points(g, n_random, seed):
    """Start points in active cells that touch a removed cell (or the box
    edge), 0.4 h from the cell centre toward the wall, and the retained mass
    of each point's pulse (share of a 20k-sample Gaussian, sigma0 = 0.3 um,
    landing on active cells): n_random of them at random plus the one that
    keeps the least mass."""
    m = omesh.build_mesh(g.L, g.N, g.disks)
    act, N, h = m.active_cell, g.N, g.h if hasattr(g, "h") else g.L / g.N
    cand = []
    for i in range(N):
        for j in range(N):
            if not act[i, j]:
                continue
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ni, nj = i + di, j + dj
                if 0 <= ni < N and 0 <= nj < N and not act[ni, nj]:
                    cand.append(((i + 0.5 + 0.4 * di) * h, (j + 0.5 + 0.4 * dj) * h))
    cand = np.asarray(cand)
    z = np.random.default_rng(seed).normal(size=(20000, 2)) * 0.3

    def kept(x):
        q = x[None, :] + z
        inside = (q[:, 0] >= 0) & (q[:, 0] < g.L) & (q[:, 1] >= 0) & (q[:, 1] < g.L)
        ci = np.clip((q[:, 0] / h).astype(int), 0, N - 1)
        cj = np.clip((q[:, 1] / h).astype(int), 0, N - 1)
        return float((inside & act[ci, cj]).mean())

    frac = np.array([kept(x) for x in cand])
    rng = np.random.default_rng(seed + 1)
    pick = list(rng.choice(cand.shape[0], n_random, replace=False)) + [int(np.argmin(frac))]
    return cand[pick], frac[pick]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_near_wall_pulses(dgd, prec):
    """Pulses started next to the staircase walls, one of them in a gap where
    most of its Gaussian falls on removed cells and is discarded before the
    unit-mass normalisation (initial-data reading R8): Sigma against the
    oracle's RK3 at the same step, 1e-10 (FP64) and 1e-4 (FP32)."""
    g = make_geometry(10.0, 40, 19070619 + 77, phi=0.65)
    pts, frac = _near_wall_points(g, 5, 19070619 + 78)
    say(f"near-wall pulses {prec}: retained mass {np.round(frac, 3).tolist()}")
    assert frac.min() < 0.5
    deltas = [0.02, 0.05]
    prob = osolve.prepare(g.L, g.N, g.disks, 2, 2.0, 10.0)
    dt = prob.dt["dt_nom"]
    ref = osolve.solve(prob, pts, 0.3, deltas, method="rk3")
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    pr = dgd.DGD_FP64 if prec == "fp64" else dgd.DGD_FP32
    op = dgd.Operator(mesh, 2, 2.0, 10.0, pr, dt_max_ms=dt)
    sig, mom = op.solve(pts, 0.3, deltas)
    err = omom.rel_err(sig, omom.sigma_a(ref))
    say(f"  max rel err {err.max():.2e}; |M0-1| {np.abs(mom[..., 0] - 1).max():.2e}")
    assert err.max() < (1e-10 if prec == "fp64" else 1e-4)
    op.close()
    mesh.close()


def test_determinism_graphs_and_checkpoint(dgd):
    """Two runs are bitwise equal (no atomics); graph replay equals plain
    launches bitwise; a state saved and restored into a new run continues
    bitwise like the uninterrupted run."""
    g, pts = _small_dense_case(nrhs=4, N=32, seed=3)
    prob = osolve.prepare(g.L, g.N, g.disks, 2, 2.0, 10.0)
    dt = prob.dt["dt_nom"]
    say("determinism / graphs / checkpoint, P2 FP32")
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, 2, 2.0, 10.0, dgd.DGD_FP32, dt_max_ms=dt)
    E = mesh.info()["n_active"]
    nval = E * 6 * pts.shape[0]

    def run(steps_list, graphs=True, restore=None):
        dgd.dgd_set_option("graphs", 1 if graphs else 0)
        r = dgd.Run(op, pts, 0.3)
        if restore is not None:
            dgd.dgd_run_set_state(r.handle, restore[0])
            dgd.dgd_run_set_step_count(r.handle, restore[1])
        outs = []
        for n in steps_list:
            r.advance(n, dt)
            outs.append(r.moments())
        st = (dgd.dgd_run_get_state(r.handle, nval, np.float32), dgd.dgd_run_step_count(r.handle))
        r.close()
        dgd.dgd_set_option("graphs", 1)
        return outs, st

    a, sa = run([100, 37, 64])
    b, sb = run([100, 37, 64])
    c, sc = run([100, 37, 64], graphs=False)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y)
        assert np.array_equal(x, z)
    assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[0], sc[0])
    assert sa[1] == 201
    # a largest graph that is no power of two (graphs of 24, 16, 8, 4, 2, 1
    # steps), and counts below it, replay bitwise like plain launches
    dgd.dgd_set_option("graph_steps", 24)
    try:
        e, se = run([100, 37, 64])
        f, _ = run([5, 3, 19, 1, 7])
        h, _ = run([5, 3, 19, 1, 7], graphs=False)
    finally:
        dgd.dgd_set_option("graph_steps", 32)
    assert all(np.array_equal(x, y) for x, y in zip(a, e)) and np.array_equal(sa[0], se[0])
    assert all(np.array_equal(x, y) for x, y in zip(f, h))
    # checkpoint (state and step count) after 137 steps, resume for 64
    _, s137 = run([100, 37])
    d, sd = run([64], restore=s137)
    assert np.array_equal(sd[0], sa[0])
    assert np.array_equal(d[-1], a[-1])
    # host buffers are sized from the run: a wrong count or type is refused
    # by the binding, and the C entry points check the byte count themselves
    import ctypes
    r = dgd.Run(op, pts, 0.3)
    with pytest.raises(ValueError):
        dgd.dgd_run_get_state(r.handle, nval + 1, np.float32)
    with pytest.raises(ValueError):
        dgd.dgd_run_set_state(r.handle, np.zeros(nval, np.float64))
    short = np.zeros(nval - 1, np.float32)
    assert dgd._lib.dgd_run_get_state(r.handle, short.ctypes.data, short.nbytes) == dgd.DGD_EINVAL
    assert dgd._lib.dgd_run_set_state(r.handle, short.ctypes.data, short.nbytes) == dgd.DGD_EINVAL
    m = np.zeros(4 * 6 - 1)
    assert dgd._lib.dgd_run_moments(r.handle, m.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    m.size) == dgd.DGD_EINVAL
    assert dgd.dgd_run_shape(r.handle) == (nval, 4, 4)
    r.close()


def test_graph_cache_many_steps_sizes(dgd):
    """A run advanced with 30 different steps (6 step graphs each, more than
    the run keeps) drops and recaptures its graphs on the way and stays
    bitwise equal to plain launches."""
    g, pts = _small_dense_case(nrhs=4, N=32, seed=5)
    prob = osolve.prepare(g.L, g.N, g.disks, 2, 2.0, 10.0)
    dt = prob.dt["dt_nom"]
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, 2, 2.0, 10.0, dgd.DGD_FP32, dt_max_ms=dt)
    say("graph cache over 30 step sizes")

    def run(graphs):
        dgd.dgd_set_option("graphs", 1 if graphs else 0)
        try:
            r = dgd.Run(op, pts, 0.3)
            for k in range(30):
                r.advance(3 + k % 5, dt * (1.0 - 1e-3 * k))
            m = r.moments()
            r.close()
        finally:
            dgd.dgd_set_option("graphs", 1)
        return m

    a, b = run(True), run(False)
    assert np.array_equal(a, b)
    op.close()
    mesh.close()


def test_auto_dt_is_stable(dgd):
    """The library's own step rule (device power iteration) stays inside the
    RK3 stability interval for the oracle's largest eigenvalue."""
    for p in (1, 2, 3):
        g, _ = _small_dense_case(nrhs=1, N=32, seed=11)
        m = omesh.build_mesh(g.L, g.N, g.disks)
        oo = sipg.assemble(m, p, 2.0, 10.0)
        lam = bounds.lambda_max(oo)
        mesh = dgd.Mesh(g.L, g.N, g.disks)
        op = dgd.Operator(mesh, p, 2.0, 10.0, dgd.DGD_FP32)
        dt, lam_gpu = dgd.dgd_operator_dt(op.handle)
        say(f"auto dt p={p}: lambda oracle {lam:.6e} gpu {lam_gpu:.6e} dt {dt:.4e}")
        assert abs(lam_gpu / lam - 1) < 0.02
        assert dt * lam <= bounds.X_RK3


def test_error_paths(dgd):
    """ENOTFREE for a start point in a removed cell or outside the box,
    EINVAL for a bad Delta list or a too small workspace (ENOMEM)."""
    import torch
    disks = np.array([[2.0, 2.0, 1.0]])
    mesh = dgd.Mesh(4.0, 8, disks)
    op = dgd.Operator(mesh, 1, 2.0, 10.0, dgd.DGD_FP32, dt_max_ms=1e-3)
    say("error paths")
    for bad in ([[2.0, 2.0]], [[-0.1, 1.0]], [[1.0, 4.0]]):
        with pytest.raises(dgd.DGDError) as e:
            op.solve(np.array(bad), 0.3, [0.01])
        assert e.value.code == dgd.DGD_ENOTFREE
    for deltas in ([0.02, 0.01], [0.0], [0.01, 0.01]):
        with pytest.raises(dgd.DGDError) as e:
            op.solve(np.array([[0.3, 0.3]]), 0.3, deltas)
        assert e.value.code == dgd.DGD_EINVAL
    ws = torch.zeros(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(dgd.DGDError) as e:
        op.solve(np.array([[0.3, 0.3]]), 0.3, [0.01], workspace=ws)
    assert e.value.code == dgd.DGD_ENOMEM
    # an explicitly unstable step is caught by the mass / finiteness check
    op2 = dgd.Operator(mesh, 1, 2.0, 10.0, dgd.DGD_FP32, dt_max_ms=0.05)
    with pytest.raises(dgd.DGDError) as e:
        op2.solve(np.array([[0.3, 0.3]]), 0.3, [20.0])
    assert e.value.code == dgd.DGD_EUNSTABLE


def test_torch_workspace_and_stream(dgd):
    """A torch-owned workspace and stream give the same result as the
    library's own allocation."""
    import torch
    c, g, pts = _c1_setup()
    prob = osolve.prepare(g.L, g.N, g.disks, c["p"], c["D"], c["eta"])
    dt = prob.dt["dt_nom"]
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, c["p"], c["D"], c["eta"], dgd.DGD_FP64, dt_max_ms=dt)
    say("torch workspace / stream")
    ws = torch.empty(op.workspace_size(1), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    a, _ = op.solve(pts, c["sigma0"], [0.3], workspace=ws, stream=s)
    b, _ = op.solve(pts, c["sigma0"], [0.3])
    assert np.array_equal(a, b)


def test_p3_mfma_operator_extraction(dgd):
    """The P3 matrix-core stage (right-hand sides in blocks of 16) applied to
    every unit vector reproduces the oracle's -M^-1 A (FP32 products with the
    FP64 mass correction): 1e-6 of max |L|."""
    import torch
    say("P3 MFMA operator extraction")
    disks = np.array([[1.5, 2.5, 0.6], [4.2, 4.4, 0.7], [5.6, 0.4, 0.5]])
    L, N, D = 6.0, 6, 1.7
    mesh = dgd.Mesh(L, N, disks)
    op = dgd.Operator(mesh, 3, D, 10.0, dgd.DGD_FP32, dt_max_ms=1e-3)
    npn, nodes, _ = op.info()
    m = omesh.build_mesh(L, N, disks)
    oo = sipg.assemble(m, 3, D, 10.0)
    E = m.n_elements
    n = E * npn
    R = (n + 15) // 16 * 16
    x = torch.zeros((n, R), dtype=torch.float32, device="cuda")
    x[:, :n] = torch.eye(n, dtype=torch.float32, device="cuda")
    y = torch.zeros_like(x)
    dgd.dgd_set_option("p3_mfma", 1)
    try:
        op.apply(x, y, R)
        torch.cuda.synchronize()
    finally:
        dgd.dgd_set_option("p3_mfma", 2)
    Lg = y[:, :n].double().cpu().numpy()
    ci, cj, ori = mesh.elements()
    key = {(int(a), int(b), int(c)): e for e, (a, b, c) in enumerate(zip(m.cell_i, m.cell_j, m.orient))}
    perm = np.array([key[(int(a), int(b), int(c))] for a, b, c in zip(ci, cj, ori)])
    T = _nodal_transform(oo, nodes)
    Tb = np.zeros((n, n))
    for e in range(E):
        Tb[e * npn:(e + 1) * npn, perm[e] * npn:(perm[e] + 1) * npn] = T[int(ori[e])]
    Lref = Tb @ oo.L.toarray() @ np.linalg.inv(Tb)
    err = np.abs(Lg - Lref).max() / np.abs(Lref).max()
    say(f"  max |L_mfma - L_oracle| / max|L| = {err:.2e}")
    assert err < 1e-6


def test_p3_mfma_solve_matches_valu_and_oracle(dgd):
    """P3 on a dense packing, 16 start points: the matrix-core path agrees
    with the FP64-arithmetic VALU path and with the oracle (1e-4), and keeps
    the mass to 2.5e-6.

    The FP32 state is stored with stochastic rounding, so its mass error is
    a zero-mean random walk: per stage at most sqrt(#values) x (weight x 0.4
    ulp) ~ 1e-8 here (10^4 values near 1, weights ~ 2e-3), at most ~2e-6
    after the 45k stages of this run, and measured 7.4e-7 (max over the 16
    columns and both Delta).  Round-to-nearest storage drifts linearly
    instead (2e-5 over the same run)."""
    g, pts = _small_dense_case(nrhs=16, N=32, seed=21)
    deltas = [0.05, 0.1]
    prob = osolve.prepare(g.L, g.N, g.disks, 3, 2.0, 10.0)
    dt = prob.dt["dt_nom"]
    say(f"P3 MFMA solve: {prob.op.mesh.n_elements} elements, dt={dt:.3e}")
    ref = osolve.solve(prob, pts, 0.3, deltas, method="cheb")
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, 3, 2.0, 10.0, dgd.DGD_FP32, dt_max_ms=dt)
    try:
        dgd.dgd_set_option("p3_mfma", 1)
        sig_m, mom_m = op.solve(pts, 0.3, deltas)
        dgd.dgd_set_option("p3_mfma", 0)
        sig_v, mom_v = op.solve(pts, 0.3, deltas)
    finally:
        dgd.dgd_set_option("p3_mfma", 2)
    e_ref = omom.rel_err(sig_m, omom.sigma_a(ref)).max()
    e_valu = omom.rel_err(sig_m, sig_v).max()
    drift = np.abs(mom_m[..., 0] - 1).max()
    say(f"  mfma vs oracle {e_ref:.2e}, vs valu {e_valu:.2e}, |M0-1| {drift:.2e}")
    assert e_ref < 1e-4 and e_valu < 1e-4
    assert drift < 2.5e-6


def _bf16x3_case(dgd):
    disks = np.array([[1.5, 2.5, 0.6], [4.2, 4.4, 0.7], [5.6, 0.4, 0.5]])
    L, N, D = 6.0, 6, 1.7
    mesh = dgd.Mesh(L, N, disks)
    op = dgd.Operator(mesh, 3, D, 10.0, dgd.DGD_BF16X3, dt_max_ms=1e-3)
    assert op.info()[2] == dgd.DGD_BF16X3
    m = omesh.build_mesh(L, N, disks)
    oo = sipg.assemble(m, 3, D, 10.0)
    npn, nodes, _ = op.info()
    ci, cj, ori = mesh.elements()
    key = {(int(a), int(b), int(c)): e for e, (a, b, c) in enumerate(zip(m.cell_i, m.cell_j, m.orient))}
    perm = np.array([key[(int(a), int(b), int(c))] for a, b, c in zip(ci, cj, ori)])
    T = _nodal_transform(oo, nodes)
    n = m.n_elements * npn
    Tb = np.zeros((n, n))
    for e in range(m.n_elements):
        Tb[e * npn:(e + 1) * npn, perm[e] * npn:(perm[e] + 1) * npn] = T[int(ori[e])]
    Lref = Tb @ oo.L.toarray() @ np.linalg.inv(Tb)
    return mesh, op, Lref, n


def test_bf16x3_operator_extraction_and_apply(dgd):
    """The P3 BF16 hi/lo split stage (DGD_BF16X3) against the oracle's
    -M^-1 A.  Unit vectors split exactly (0, +-1 are BF16 values), so the
    extracted operator carries only the operator's own split (A_hi + A_mid +
    A_lo, 24 significant bits, remainder below 2^-27 of each entry) and the
    FP32 accumulation: 1e-6 of max |L|, as for FP32 products.  On random
    state in [-1, 1] the state split adds its error (x_lo rounded: below
    2^-17 of each |u - c|, the dropped A_mid x_lo below 2^-18, at most
    doubled by the mass correction): every output within 2^-15 of
    sum_k |L_ik| |u_k - c| <= 2 sum_k |L_ik|."""
    import torch
    say("P3 BF16X3 operator extraction")
    mesh, op, Lref, n = _bf16x3_case(dgd)
    R = (n + 15) // 16 * 16
    x = torch.zeros((n, R), dtype=torch.float32, device="cuda")
    x[:, :n] = torch.eye(n, dtype=torch.float32, device="cuda")
    y = torch.zeros_like(x)
    op.apply(x, y, R)
    torch.cuda.synchronize()
    Lg = y[:, :n].double().cpu().numpy()
    err = np.abs(Lg - Lref).max() / np.abs(Lref).max()
    say(f"  max |L_bf16x3 - L_oracle| / max|L| = {err:.2e}")
    assert err < 1e-6
    # random state, 32 columns
    rng = np.random.default_rng(5)
    xr = rng.uniform(-1.0, 1.0, size=(n, 32))
    xt = torch.tensor(xr, dtype=torch.float32, device="cuda")
    yt = torch.zeros_like(xt)
    op.apply(xt, yt, 32)
    torch.cuda.synchronize()
    yref = Lref @ xt.double().cpu().numpy()
    scale = np.abs(Lref) @ np.full((n, 1), 2.0)
    rel = (np.abs(yt.double().cpu().numpy() - yref) / scale).max()
    say(f"  random state: max |y - y_ref| / (|L| 2) = {rel:.2e} (bound {2.0 ** -15:.2e})")
    assert rel < 2.0 ** -15
    # the split needs blocks of 16 right-hand sides
    with pytest.raises(dgd.DGDError) as e:
        op.apply(xt, yt, 24)
    assert e.value.code == dgd.DGD_EINVAL


def test_bf16x3_solve_matches_oracle(dgd):
    """P3 RK3 with BF16 hi/lo split products (DGD_BF16X3) on a dense
    packing, 16 start points: Sigma within 1e-4 of the oracle and of the
    FP32 vector path; the FP64 mass correction keeps M0 to the stochastic
    rounding walk of the FP32 state (2.5e-6, as for the FP32 products)."""
    g, pts = _small_dense_case(nrhs=16, N=32, seed=21)
    deltas = [0.05, 0.1]
    prob = osolve.prepare(g.L, g.N, g.disks, 3, 2.0, 10.0)
    dt = prob.dt["dt_nom"]
    say(f"P3 BF16X3 solve: {prob.op.mesh.n_elements} elements, dt={dt:.3e}")
    ref = osolve.solve(prob, pts, 0.3, deltas, method="cheb")
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, 3, 2.0, 10.0, dgd.DGD_BF16X3, dt_max_ms=dt)
    run = dgd.Run(op, pts, 0.3)
    assert dgd.dgd_run_kernel(run.handle)[0] == "mfma_bf16x3"
    run.close()
    sig_b, mom_b = op.solve(pts, 0.3, deltas)
    op32 = dgd.Operator(mesh, 3, 2.0, 10.0, dgd.DGD_FP32, dt_max_ms=dt)
    dgd.dgd_set_option("p3_mfma", 0)
    try:
        sig_v, _ = op32.solve(pts, 0.3, deltas)
    finally:
        dgd.dgd_set_option("p3_mfma", 2)
    e_ref = omom.rel_err(sig_b, omom.sigma_a(ref)).max()
    e_valu = omom.rel_err(sig_b, sig_v).max()
    drift = np.abs(mom_b[..., 0] - 1).max()
    say(f"  bf16x3 vs oracle {e_ref:.2e}, vs fp32 valu {e_valu:.2e}, |M0-1| {drift:.2e}")
    assert e_ref < 1e-4 and e_valu < 1e-4
    assert drift < 2.5e-6
    # 8 start points are not a multiple of 16: refused
    with pytest.raises(dgd.DGDError) as e:
        op.solve(pts[:8], 0.3, deltas)
    assert e.value.code == dgd.DGD_EINVAL


@pytest.mark.parametrize("p", [1, 2, 3])
def test_expm_solve_matches_oracle_flow(dgd, p):
    """Chebyshev exponential on the GPU (FP64 state) against the oracle's
    Chebyshev exponential: both are the exact semi-discrete flow, so Sigma
    agrees to 1e-10 whatever the spectral bounds each side uses."""
    g, pts = _small_dense_case(nrhs=4, N=32, seed=31 + p)
    deltas = [0.2, 1.0, 3.0]
    prob = osolve.prepare(g.L, g.N, g.disks, p, 2.0, 10.0)
    ref = osolve.solve(prob, pts, 0.3, deltas, method="cheb")
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, p, 2.0, 10.0, dgd.DGD_FP32)
    sig, mom, napp = dgd.dgd_eap_solve_expm(op.handle, pts, 0.3, deltas)
    err = omom.rel_err(sig, omom.sigma_a(ref)).max()
    say(f"expm p={p}: {napp} applications, max rel err vs oracle {err:.2e}, |M0-1| "
        f"{np.abs(mom[..., 0] - 1).max():.1e}")
    assert err < 1e-10

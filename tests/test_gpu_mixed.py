"""GPU parity of the paper's mixed form on all pixels (eq. (6)-(7), fluxes of
section 3.2, k = 0 in axon cells) against the oracle's mixed form, through
the C-ABI:

* the dense operator (gradient pass + divergence pass, FP64 and FP32, one
  block of all columns and blocks of 8) after the change of basis;
* RK3 with a Gaussian pulse, FP64 state, same step schedule: moments 1e-10;
* point mass, FP32 state, against the oracle's exact flow;
* the device power iteration against the oracle's spectral radius;
* E(0) = M0 of the signal, and the error paths (axon start point, the
  exponential and batches reject the mixed form).
"""

import sys

import numpy as np
import pytest

from oracle import mixed, moments as omom, sipg, timeint
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


def _block_transform(mesh, m, Np_o, p, nodes, npn):
    """Library (element order, nodal) <- oracle (element order, monomials)."""
    ci, cj, ori = mesh.elements()
    key = {(int(a), int(b), int(c)): e for e, (a, b, c) in enumerate(zip(m.cell_i, m.cell_j, m.orient))}
    perm = np.array([key[(int(a), int(b), int(c))] for a, b, c in zip(ci, cj, ori)])
    mons = sipg.monomials(p)
    T = [np.stack([(nodes[o, :, 0] - 0.5) ** a * (nodes[o, :, 1] - 0.5) ** b for (a, b) in mons], axis=1)
         for o in (0, 1)]
    E = m.n_elements
    Tb = np.zeros((E * npn, E * npn))
    for e in range(E):
        Tb[e * npn:(e + 1) * npn, perm[e] * npn:(perm[e] + 1) * npn] = T[int(ori[e])]
    return Tb


DISKS = np.array([[1.5, 2.5, 0.7], [4.2, 4.4, 0.8], [5.6, 0.4, 0.6]])


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n_rhs", ["all", 8])
def test_mixed_operator_extraction(dgd, p, prec, n_rhs):
    import torch
    say(f"mixed-form operator extraction p={p} {prec} rhs={n_rhs}")
    L, N, D = 6.0, 6, 1.7
    mesh = dgd.Mesh(L, N, np.zeros((0, 3)))
    pr = dgd.DGD_FP64 if prec == "fp64" else dgd.DGD_FP32
    op = dgd.MixedOperator(mesh, DISKS, p, D, pr, dt_max_ms=1e-3)
    npn, nodes, _ = op.info()
    oo = mixed.assemble_mixed(L, N, DISKS, p, D)
    assert (~oo.extracellular).sum() > 0
    n = oo.mesh.n_elements * npn
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
    Tb = _block_transform(mesh, oo.mesh, oo.Np, p, nodes, npn)
    Lref = Tb @ oo.L.toarray() @ np.linalg.inv(Tb)
    scale = np.abs(Lref).max()
    # FP64: the test's monomial-to-nodal change of basis loses ~1e-11 at p = 3
    tol = (1e-12 if p < 3 else 1e-10) if prec == "fp64" else 2e-6
    err = np.abs(Lg - Lref).max() / scale
    say(f"  max |L_gpu - L_oracle| / max|L| = {err:.2e}")
    assert err < tol


def _case(nrhs, N, seed, phi=0.55):
    h = 100.0 / 512
    g = make_geometry(N * h, N, 19070619 + 1500 + seed, phi=phi)
    pts = start_points(g.disks, g.L, g.N, nrhs, np.random.default_rng(19070619 + 1501 + seed))
    return g, pts


def _dt(op_o, D, h):
    p = op_o.p
    return min(0.1 * h * h / (D * (p + 1) ** 2), mixed.step_rule(op_o)["dt_nom"])


@pytest.mark.parametrize("p", [1, 2, 3])
def test_mixed_rk3_fp64_matches_oracle(dgd, p):
    g, pts = _case(4, 24, p)
    D = 2.0
    deltas = [0.05, 0.2, 0.5]
    oo = mixed.assemble_mixed(g.L, g.N, g.disks, p, D)
    mesh = dgd.Mesh(g.L, g.N, np.zeros((0, 3)))
    op = dgd.MixedOperator(mesh, g.disks, p, D, dgd.DGD_FP64, dt_max_ms=_dt(oo, D, g.L / g.N))
    dt = op.dt                  # the same step on both sides
    say(f"mixed RK3 FP64 p={p}: {oo.mesh.n_elements} elements "
        f"({int((~oo.extracellular).sum())} in axons), dt={dt:.3e}")
    U0 = mixed.initial_block(oo, pts, 0.3)
    ref = np.stack(timeint.rk3(oo.L, U0, deltas, dt, on_delta=lambda k, U: omom.moments(oo, U, pts)),
                   axis=1)                                           # [R, nDelta, 6]
    sig, mom = op.solve(pts, 0.3, deltas)
    err = np.abs(mom - ref).max() / np.abs(ref).max()
    say(f"  max moment err {err:.2e}; |M0 - 1| {np.abs(mom[..., 0] - 1).max():.1e}")
    assert err < 1e-10
    assert np.abs(mom[..., 0] - 1).max() < 1e-12


def test_mixed_point_mass_fp32_vs_exact_flow(dgd):
    from scipy.sparse.linalg import expm_multiply
    g, pts = _case(8, 40, 11, phi=0.6)
    D, p = 2.0, 2
    deltas = [0.1, 0.4]
    oo = mixed.assemble_mixed(g.L, g.N, g.disks, p, D)
    dt = _dt(oo, D, g.L / g.N)
    say(f"mixed point mass FP32 P2: {oo.mesh.n_elements} elements, dt={dt:.3e}")
    U = mixed.initial_block(oo, pts, 0.0)
    ref, prev = [], 0.0
    for t in deltas:
        U = expm_multiply(oo.L * (t - prev), U)
        prev = t
        ref.append(omom.moments(oo, U, pts))
    ref = np.stack(ref, axis=1)
    mesh = dgd.Mesh(g.L, g.N, np.zeros((0, 3)))
    op = dgd.MixedOperator(mesh, g.disks, p, D, dgd.DGD_FP32, dt_max_ms=dt)
    sig, mom = op.solve(pts, 0.0, deltas)
    err = np.abs(mom - ref).max()
    say(f"  max |moments - oracle| = {err:.2e}; |M0 - 1| {np.abs(mom[..., 0] - 1).max():.1e}")
    assert err < 1e-5
    assert np.abs(mom[..., 0] - 1).max() < 1e-5


def test_mixed_auto_dt_and_signal(dgd):
    g, pts = _case(2, 24, 21)
    D, p = 2.0, 2
    oo = mixed.assemble_mixed(g.L, g.N, g.disks, p, D)
    rho = mixed.spectral_radius(oo)
    mesh = dgd.Mesh(g.L, g.N, np.zeros((0, 3)))
    op = dgd.MixedOperator(mesh, g.disks, p, D, dgd.DGD_FP64)
    dt, lam = dgd.dgd_operator_dt(op.handle)
    say(f"mixed auto dt: rho oracle {rho:.6e}, gpu {lam:.6e}, dt {dt:.4e}")
    assert abs(lam / rho - 1) < 0.02
    qs = np.array([[0.0, 0.0], [0.8, -0.3]])
    sig, mom = dgd.dgd_eap_solve_signal(op.handle, pts, 0.3, [0.05], qs)
    assert np.abs(sig[:, 0, 0].real - mom[:, 0, 0]).max() < 1e-14


def test_mixed_checkpoint_resume_bitwise(dgd):
    """FP32 run: state + step count saved and restored repeat the
    uninterrupted run bit for bit; set_state clears axon-cell blocks."""
    g, pts = _case(3, 20, 41)
    mesh = dgd.Mesh(g.L, g.N, np.zeros((0, 3)))
    op = dgd.MixedOperator(mesh, g.disks, 2, 2.0, dgd.DGD_FP32, dt_max_ms=1e-4)
    E = mesh.info()["n_active"]
    nval = E * 6 * 3
    a = dgd.Run(op, pts, 0.3)
    a.advance(40, 1e-4)
    st = dgd.dgd_run_get_state(a.handle, nval, np.float32)
    steps = dgd.dgd_run_step_count(a.handle)
    a.advance(50, 1e-4)
    ref = dgd.dgd_run_get_state(a.handle, nval, np.float32)
    b = dgd.Run(op, pts, 0.3)
    dirty = st.copy().reshape(E, -1)
    oo = mixed.assemble_mixed(g.L, g.N, g.disks, 2, 2.0)
    ci, cj, ori = mesh.elements()
    ax_cell = {(int(i), int(j)) for i, j, k in zip(oo.mesh.cell_i, oo.mesh.cell_j, oo.kel) if k == 0}
    axon = np.array([(int(i), int(j)) in ax_cell for i, j in zip(ci, cj)])
    assert axon.any() and np.abs(dirty[axon]).max() == 0.0
    dirty[axon] = 7.0
    dgd.dgd_run_set_state(b.handle, dirty.ravel())
    dgd.dgd_run_set_step_count(b.handle, steps)
    b.advance(50, 1e-4)
    got = dgd.dgd_run_get_state(b.handle, nval, np.float32)
    say(f"mixed checkpoint: {int(axon.sum())} axon elements; equal {np.array_equal(got, ref)}")
    assert np.array_equal(got, ref)
    a.close()
    b.close()


def test_mixed_tuned_shape_same_bits(dgd):
    """The autotuned launch shape of the two passes gives the same state,
    bit for bit, as the default shape (each element's arithmetic does not
    depend on which wave runs it)."""
    g, pts = _case(5, 24, 51)
    mesh = dgd.Mesh(g.L, g.N, np.zeros((0, 3)))
    op = dgd.MixedOperator(mesh, g.disks, 2, 2.0, dgd.DGD_FP32, dt_max_ms=1e-4)
    nval = mesh.info()["n_active"] * 6 * 5
    states = []
    for tuned in (1, 0):
        dgd.dgd_set_option("autotune", tuned)
        try:
            run = dgd.Run(op, pts, 0.3)
            shape = dgd.dgd_run_kernel(run.handle)[1]
            run.advance(60, 1e-4)
            states.append(dgd.dgd_run_get_state(run.handle, nval, np.float32))
            run.close()
        finally:
            dgd.dgd_set_option("autotune", 1)
        say(f"mixed shape (autotune={tuned}): {shape}")
    assert np.array_equal(states[0], states[1])


def test_mixed_errors(dgd):
    g, pts = _case(2, 16, 31)
    mesh = dgd.Mesh(g.L, g.N, np.zeros((0, 3)))
    op = dgd.MixedOperator(mesh, g.disks, 2, 2.0, dgd.DGD_FP64, dt_max_ms=1e-4)
    d = g.disks[np.argmax(g.disks[:, 2])]
    with pytest.raises(dgd.DGDError) as e:
        op.solve(np.array([[d[0], d[1]]]), 0.3, [0.01])
    assert e.value.code == dgd.DGD_ENOTFREE
    with pytest.raises(dgd.DGDError) as e:
        op.solve(np.array([[d[0], d[1]]]), 0.0, [0.01])
    assert e.value.code == dgd.DGD_ENOTFREE
    with pytest.raises(dgd.DGDError) as e:
        dgd.dgd_eap_solve_expm(op.handle, pts, 0.3, [0.01])
    assert e.value.code == dgd.DGD_EINVAL
    with pytest.raises(dgd.DGDError) as e:
        dgd.dgd_eap_solve_batch([op], pts[None], 0.3, [0.01])
    assert e.value.code == dgd.DGD_EINVAL

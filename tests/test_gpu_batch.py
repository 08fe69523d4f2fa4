"""GPU: the batched solve (several geometries of uneven size and mixed
degree in one launch sequence) against the plain per-geometry solve and the
FP64 oracle."""

import sys

import numpy as np
import pytest

from oracle import moments as omom
from oracle import solve as osolve
from workloads import make_geometry, start_points

pytestmark = pytest.mark.gpu

H = 100.0 / 512


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


def _geoms(n, R, seed0=4100):
    out = []
    rng = np.random.default_rng(seed0)
    for g in range(n):
        N = int(rng.integers(24, 61))
        phi = float(rng.uniform(0.4, 0.7))
        geo = make_geometry(N * H, N, seed0 + 17 * g, phi=phi, shape=float(rng.uniform(3, 6)),
                            mean=float(rng.uniform(0.4, 0.7)))
        pts = start_points(geo.disks, geo.L, geo.N, R, np.random.default_rng(seed0 + 17 * g + 1))
        p = 1 if g % 3 == 0 else 2
        out.append((geo, pts, p))
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_equals_plain_bitwise(dgd, prec):
    """Concatenated geometries run the same per-element arithmetic and the
    same block-aligned reductions as separate plain solves: equal bitwise."""
    R = 4
    cases = _geoms(5, R)
    pr = dgd.DGD_FP32 if prec == "fp32" else dgd.DGD_FP64
    dt = {1: 1.2e-4, 2: 2.3e-5}
    meshes = [dgd.Mesh(g.L, g.N, g.disks) for g, _, _ in cases]
    ops = [dgd.Operator(m, p, 2.0, 10.0, pr, dt_max_ms=dt[p]) for m, (_, _, p) in zip(meshes, cases)]
    pts = np.stack([c[1] for c in cases])
    deltas = [0.02, 0.05]
    say(f"batch {prec}: sizes {[m.info()['n_active'] for m in meshes]}")
    sig_b, mom_b = dgd.dgd_eap_solve_batch(ops, pts, 0.3, deltas)
    for g, op in enumerate(ops):
        sig_p, mom_p = op.solve(pts[g], 0.3, deltas)
        assert np.array_equal(mom_b[g], mom_p), g
        assert np.array_equal(sig_b[g], sig_p), g


def test_batch_vs_oracle_and_advance_api(dgd):
    """Batched FP32 against the FP64 oracle (Chebyshev flow) on two
    geometries, through the create / advance / moments entry points."""
    R = 4
    cases = _geoms(2, R, seed0=5200)
    cases = [(cases[0][0], cases[0][1], 1), (cases[1][0], cases[1][1], 2)]
    deltas = [0.3]
    ops, refs = [], []
    for geo, pts, p in cases:
        prob = osolve.prepare(geo.L, geo.N, geo.disks, p, 2.0, 10.0)
        refs.append(osolve.solve(prob, pts, 0.3, deltas, method="cheb"))
        m = dgd.Mesh(geo.L, geo.N, geo.disks)
        ops.append(dgd.Operator(m, p, 2.0, 10.0, dgd.DGD_FP32, dt_max_ms=prob.dt["dt_nom"]))
    pts = np.stack([c[1] for c in cases])
    b = dgd.Batch(ops, pts, 0.3)
    groups = b.groups()
    say(f"batch groups {groups}")
    assert sorted(gr["p"] for gr in groups) == [1, 2]
    for k, gr in enumerate(groups):
        n = int(np.ceil(deltas[0] / gr["dt"] - 1e-9))
        b.advance(k, n, deltas[0] / n)
    mom = b.moments()
    for g in range(2):
        err = omom.rel_err(omom.sigma_a(mom[g]), omom.sigma_a(refs[g][:, 0]))
        say(f"  geometry {g} p={cases[g][2]}: max rel err {err.max():.2e}")
        assert err.max() < 1e-4
    b.close()


def test_batch_persistent_grid_bitwise(dgd):
    """A persistent stage grid (fewer workgroups than blocks, each looping)
    gives the same bits as one workgroup per block."""
    R = 4
    cases = _geoms(3, R, seed0=6300)
    meshes = [dgd.Mesh(g.L, g.N, g.disks) for g, _, _ in cases]
    ops = [dgd.Operator(m, 2, 2.0, 10.0, dgd.DGD_FP32, dt_max_ms=2.3e-5) for m in meshes]
    pts = np.stack([c[1] for c in cases])
    say("persistent grid")
    a, _ = dgd.dgd_eap_solve_batch(ops, pts, 0.3, [0.01])
    dgd.dgd_set_option("stage_grid", 64)
    try:
        b, _ = dgd.dgd_eap_solve_batch(ops, pts, 0.3, [0.01])
    finally:
        dgd.dgd_set_option("stage_grid", 0)
    assert np.array_equal(a, b)


def test_sorted_tables(dgd):
    """With class-sorted element tables (option sort_classes = 1): batched ==
    plain bitwise; Sigma within 1e-5 of the mesh-order runs (the same
    arithmetic per lane; reductions sum in another order, which moves FP32
    states by an ulp and so the stochastic rounding); the host state is in
    mesh order (initial states agree with the mesh-order run's to 1e-6),
    and a checkpoint resumes bitwise."""
    R = 4
    cases = _geoms(3, R, seed0=7300)
    meshes = [dgd.Mesh(g.L, g.N, g.disks) for g, _, _ in cases]
    ops = [dgd.Operator(m, p, 2.0, 10.0, dgd.DGD_FP32, dt_max_ms={1: 1.2e-4, 2: 2.3e-5}[p])
           for m, (_, _, p) in zip(meshes, cases)]
    pts = np.stack([c[1] for c in cases])
    deltas = [0.02, 0.05]
    say("sorted element tables")
    ref = [op.solve(pts[g], 0.3, deltas)[0] for g, op in enumerate(ops)]
    init0 = dgd.Run(ops[0], pts[0], 0.3)
    s0 = dgd.dgd_run_get_state(init0.handle)
    init0.close()
    dgd.dgd_set_option("sort_classes", 1)
    try:
        sig_b, mom_b = dgd.dgd_eap_solve_batch(ops, pts, 0.3, deltas)
        for g, op in enumerate(ops):
            sig_p, mom_p = op.solve(pts[g], 0.3, deltas)
            assert np.array_equal(mom_b[g], mom_p), g
            err = omom.rel_err(sig_p, ref[g])
            assert err.max() < 1e-5, err.max()
        run = dgd.Run(ops[0], pts[0], 0.3)
        s1 = dgd.dgd_run_get_state(run.handle)
        assert s1.shape == s0.shape
        assert np.abs(s1 - s0).max() <= 1e-6 * np.abs(s0).max()
        dt = ops[0].dt
        run.advance(50, dt)
        ck = (dgd.dgd_run_get_state(run.handle), dgd.dgd_run_step_count(run.handle))
        run.advance(30, dt)
        want = dgd.dgd_run_get_state(run.handle)
        run.close()
        run2 = dgd.Run(ops[0], pts[0], 0.3)
        dgd.dgd_run_set_state(run2.handle, ck[0])
        dgd.dgd_run_set_step_count(run2.handle, ck[1])
        run2.advance(30, dt)
        assert np.array_equal(dgd.dgd_run_get_state(run2.handle), want)
        run2.close()
    finally:
        dgd.dgd_set_option("sort_classes", 0)

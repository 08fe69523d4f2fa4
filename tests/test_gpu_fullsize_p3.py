"""GPU parity at full size for the 256 x 256, phi = 0.65, P3, 128-start-point
workload against oracle values stored by tests/golden/make_full_golden.py
(the oracle's Chebyshev exponential on the full mesh, 8 sampled start
points, all 20 Delta).

* Chebyshev exponential (FP64 state): every Delta to 30 ms, 1e-8 on Sigma.
* RK3 on matrix cores (FP32 state, forced): the first Delta (about 150k
  steps), 1e-4 on Sigma.
* RK3 with BF16 hi/lo split products (DGD_BF16X3): the first two Delta,
  1e-4 on Sigma (all 20 Delta, about 4.7 million steps, with DGD_LONG=1).
"""

import json
import os
import sys

import numpy as np
import pytest

from oracle import moments as omom
from workloads import config, make_geometry, start_points

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "pack256-p3_oracle.json")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def case():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1907_06191_amd import dgd
    with open(GOLDEN) as f:
        gold = json.load(f)
    c = config(gold["workload"])
    g = make_geometry(c["L"], c["N"], c["geom_seed"], phi=c["phi"], n_disks=c["n_disks"])
    pts = start_points(g.disks, g.L, g.N, c["R"], np.random.default_rng(c["point_seed"]))
    idx = np.asarray(gold["sample_index"])
    assert g.disks.shape[0] == gold["n_disks"]
    assert np.array_equal(pts[idx], np.asarray(gold["points"]))
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    assert mesh.info()["n_active"] == gold["n_elements"]
    return dgd, c, gold, mesh, pts, idx


def test_fullsize_p3_expm_all_deltas(case):
    dgd, c, gold, mesh, pts, idx = case
    say(f"full-size P3 Chebyshev exponential: {gold['n_elements']} elements, "
        f"{len(gold['deltas'])} Delta to {gold['deltas'][-1]:.0f} ms")
    op = dgd.Operator(mesh, 3, c["D"], c["eta"], dgd.DGD_FP32, dt_max_ms=gold["dt_nom"])
    sig, mom, napp = dgd.dgd_eap_solve_expm(op.handle, pts, c["sigma0"], gold["deltas"])
    err = omom.rel_err(sig[idx], omom.sigma_a(np.asarray(gold["moments"])))
    say(f"  {napp} operator applications; max rel err vs oracle {err.max():.2e}")
    assert err.max() < 1e-8
    op.close()


def test_fullsize_p3_rk3_matrix_cores_first_delta(case):
    """The matrix-core kernel (an option: the vector kernel is faster) over
    the first Delta, on the 8 stored start points and the 8 following ones
    (16 right-hand sides: one 64-column chunk per element)."""
    dgd, c, gold, mesh, pts, idx = case
    sel = np.sort(np.concatenate([idx, idx + 1]))
    pos = np.searchsorted(sel, idx)
    say(f"full-size P3 RK3 on matrix cores: dt {gold['dt_nom']:.4e} ms to Delta "
        f"{gold['deltas'][0]} ms, 16 right-hand sides")
    op = dgd.Operator(mesh, 3, c["D"], c["eta"], dgd.DGD_FP32, dt_max_ms=gold["dt_nom"])
    dgd.dgd_set_option("p3_mfma", 1)
    try:
        run = dgd.Run(op, pts[sel], c["sigma0"])
        assert dgd.dgd_run_kernel(run.handle)[0] == "mfma"
        run.close()
        sig, mom = op.solve(pts[sel], c["sigma0"], gold["deltas"][:1])
    finally:
        dgd.dgd_set_option("p3_mfma", 2)
    err = omom.rel_err(sig[pos], omom.sigma_a(np.asarray(gold["moments"])[:, :1]))
    drift = np.abs(mom[..., 0] - 1).max()
    say(f"  max rel err vs oracle {err.max():.2e}; |M0-1| {drift:.2e}")
    assert err.max() < 1e-4
    assert drift < 1e-5
    op.close()


def test_fullsize_p3_rk3_valu_first_delta(case):
    """The kernel the P3 benchmark runs when the autotuner prefers the FP64
    vector path: k_stage<float, 10> at 128 right-hand sides (two 64-column
    chunks per element), RK3 over the first Delta."""
    dgd, c, gold, mesh, pts, idx = case
    say(f"full-size P3 RK3 on the vector kernel: dt {gold['dt_nom']:.4e} ms to Delta "
        f"{gold['deltas'][0]} ms, {pts.shape[0]} right-hand sides")
    op = dgd.Operator(mesh, 3, c["D"], c["eta"], dgd.DGD_FP32, dt_max_ms=gold["dt_nom"])
    dgd.dgd_set_option("p3_mfma", 0)
    try:
        run = dgd.Run(op, pts, c["sigma0"])
        assert dgd.dgd_run_kernel(run.handle)[0] == "valu"
        run.close()
        sig, mom = op.solve(pts, c["sigma0"], gold["deltas"][:1])
    finally:
        dgd.dgd_set_option("p3_mfma", 2)
    err = omom.rel_err(sig[idx], omom.sigma_a(np.asarray(gold["moments"])[:, :1]))
    drift = np.abs(mom[..., 0] - 1).max()
    say(f"  max rel err vs oracle {err.max():.2e}; |M0-1| {drift:.2e}")
    assert err.max() < 1e-4
    assert drift < 1e-5
    op.close()


def _bf16x3_deltas(case, nd):
    import torch
    dgd, c, gold, mesh, pts, idx = case
    sel = np.sort(np.concatenate([idx, idx + 1]))
    pos = np.searchsorted(sel, idx)
    op = dgd.Operator(mesh, 3, c["D"], c["eta"], dgd.DGD_BF16X3, dt_max_ms=gold["dt_nom"])
    run = dgd.Run(op, pts[sel], c["sigma0"])
    assert dgd.dgd_run_kernel(run.handle)[0] == "mfma_bf16x3"
    dt, prev, mom = gold["dt_nom"], 0.0, []
    ref = np.asarray(gold["moments"])
    for k, d in enumerate(gold["deltas"][:nd]):
        n = int(np.ceil((d - prev) / dt - 1e-9))
        # the library's landing step for this interval, advanced in pieces
        # (same steps, a progress line at least every 100k)
        for a in range(0, n, 100000):
            run.advance(min(100000, n - a), (d - prev) / n)
            if n > 100000:
                torch.cuda.synchronize()
                say(f"    {min(a + 100000, n)} / {n} steps")
        mom.append(run.moments())
        prev = d
        e = omom.rel_err(omom.sigma_a(mom[-1][pos][:, None]), omom.sigma_a(ref[:, k:k + 1])).max()
        say(f"  Delta {d:.3f} ms ({n} steps): rel err {e:.2e}, |M0-1| {np.abs(mom[-1][:, 0] - 1).max():.1e}")
    run.close()
    mom = np.stack(mom, axis=1)
    err = omom.rel_err(omom.sigma_a(mom[pos]), omom.sigma_a(ref[:, :nd]))
    drift = np.abs(mom[..., 0] - 1).max()
    say(f"  max rel err vs oracle {err.max():.2e}; |M0-1| {drift:.2e}")
    op.close()
    return err, drift


def test_fullsize_p3_rk3_bf16x3_first_deltas(case):
    """DGD_BF16X3 (every stage on matrix cores as BF16 hi/lo split products)
    over the first two Delta on the 8 stored start points and the 8
    following ones (16 right-hand sides)."""
    say("full-size P3 RK3, BF16 hi/lo split products, first two Delta")
    err, drift = _bf16x3_deltas(case, 2)
    assert err.max() < 1e-4
    assert drift < 1e-5


@pytest.mark.skipif(os.environ.get("DGD_LONG") != "1",
                    reason="about 15 minutes of GPU time: run with DGD_LONG=1")
def test_fullsize_p3_rk3_bf16x3_all_deltas(case):
    say("full-size P3 RK3, BF16 hi/lo split products, all Delta to 30 ms")
    err, drift = _bf16x3_deltas(case, 20)
    assert err.max() < 1e-4
    assert drift < 1e-5

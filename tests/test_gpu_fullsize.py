"""GPU parity at full size: the 512 x 512, phi = 0.6, P2, 64-start-point
workload, in the launch configuration the benchmark times, against oracle
values stored by tests/golden/make_full_golden.py (the oracle's Chebyshev
exponential on the full mesh, 8 sampled start points, all 20 Delta).

* RK3 (FP32 state): every Delta up to 5.19 ms (the first nine, about 226k
  steps, a tenth of the 50 ms schedule), 1e-4 on Sigma; mass within 1e-5.
* Chebyshev exponential (FP64 state): every Delta to 50 ms, 1e-8 on Sigma.
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
                      "pack512-p2_oracle.json")


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


def test_fullsize_rk3_fp32_first_deltas(case):
    dgd, c, gold, mesh, pts, idx = case
    nd = int(np.sum(np.asarray(gold["deltas"]) <= 5.2))
    assert nd == 9
    say(f"full-size RK3 P{gold['p']} FP32: {gold['n_elements']} elements, {pts.shape[0]} points, "
        f"dt {gold['dt_nom']:.4e} ms, Delta {gold['deltas'][:nd]}")
    op = dgd.Operator(mesh, gold["p"], c["D"], c["eta"], dgd.DGD_FP32, dt_max_ms=gold["dt_nom"])
    # with the q-space signal at every Delta: E(0) = M0 and the small-q
    # expansion E(eps u) = M0 + i eps u.m1 - eps^2 u^T M2 u / 2 + O(eps^3)
    # hold against the FP64 moment kernel at any size
    eps = 1e-3
    dirs = np.array([[1.0, 0.0], [0.0, 1.0], [0.6, 0.8]])
    qs = np.concatenate([np.zeros((1, 2)), eps * dirs, [[1.0, 0.5]]])
    E, mom = dgd.dgd_eap_solve_signal(op.handle, pts, c["sigma0"], gold["deltas"][:nd], qs)
    sig = omom.sigma_a(mom)
    ref = omom.sigma_a(np.asarray(gold["moments"])[:, :nd])
    err = omom.rel_err(sig[idx], ref)
    drift = np.abs(mom[..., 0] - 1).max()
    say(f"  max rel err vs oracle {err.max():.2e}; |M0-1| {drift:.2e}")
    assert err.max() < 1e-4
    assert drift < 1e-5
    assert np.abs(E[..., 0] - mom[..., 0]).max() < 1e-12
    m1 = mom[..., 1:3]
    M2 = np.stack([np.stack([mom[..., 3], mom[..., 4]], -1), np.stack([mom[..., 4], mom[..., 5]], -1)], -2)
    for k, u in enumerate(dirs):
        first = eps * (m1 @ u)
        second = 0.5 * eps ** 2 * np.einsum("...i,...ij,j->...", np.broadcast_to(u, m1.shape), M2, u)
        assert np.abs(E[..., 1 + k].imag - first).max() < 1e-4 * np.abs(first).max()
        assert np.abs((mom[..., 0] - E[..., 1 + k].real) - second).max() < 1e-3 * np.abs(second).max()
    op.close()


def test_fullsize_expm_all_deltas(case):
    dgd, c, gold, mesh, pts, idx = case
    say(f"full-size Chebyshev exponential P{gold['p']}: {len(gold['deltas'])} Delta to "
        f"{gold['deltas'][-1]:.0f} ms")
    op = dgd.Operator(mesh, gold["p"], c["D"], c["eta"], dgd.DGD_FP32, dt_max_ms=gold["dt_nom"])
    sig, mom, napp = dgd.dgd_eap_solve_expm(op.handle, pts, c["sigma0"], gold["deltas"])
    ref = omom.sigma_a(np.asarray(gold["moments"]))
    err = omom.rel_err(sig[idx], ref)
    say(f"  {napp} operator applications; max rel err vs oracle {err.max():.2e}")
    assert err.max() < 1e-8
    op.close()


@pytest.mark.skipif(os.environ.get("DGD_LONG") != "1",
                    reason="about 6 minutes of GPU time: run with DGD_LONG=1")
def test_fullsize_rk3_fp32_all_deltas_r16(case):
    """The whole 50 ms schedule of the 512^2 P2 workload by RK3 (about 2.26
    million steps): the 8 stored start points and the 8 following ones as
    16 right-hand sides (the packed stage kernel), every Delta against the
    oracle's exact flow; 1e-4 on Sigma, mass within 1e-5."""
    dgd, c, gold, mesh, pts, idx = case
    sel = np.sort(np.concatenate([idx, idx + 1]))
    pos = np.searchsorted(sel, idx)
    say(f"full-size RK3 P2 FP32, 16 right-hand sides, {len(gold['deltas'])} Delta to "
        f"{gold['deltas'][-1]:.0f} ms, dt {gold['dt_nom']:.4e} ms")
    op = dgd.Operator(mesh, gold["p"], c["D"], c["eta"], dgd.DGD_FP32, dt_max_ms=gold["dt_nom"])
    # the library's landing schedule, one Delta at a time (progress per Delta)
    run = dgd.Run(op, pts[sel], c["sigma0"])
    dt, prev, mom = gold["dt_nom"], 0.0, []
    for k, d in enumerate(gold["deltas"]):
        n = int(np.ceil((d - prev) / dt - 1e-9))
        run.advance(n, (d - prev) / n)
        mom.append(run.moments())
        prev = d
        say(f"  Delta {d:.3f} ms reached ({n} steps), |M0-1| {np.abs(mom[-1][:, 0] - 1).max():.1e}")
    run.close()
    mom = np.stack(mom, axis=1)
    sig = omom.sigma_a(mom)
    ref = omom.sigma_a(np.asarray(gold["moments"]))
    err = omom.rel_err(sig[pos], ref)
    drift = np.abs(mom[..., 0] - 1).max()
    say(f"  max rel err vs oracle {err.max():.2e} (per Delta {np.round(err.max(axis=0), 8).tolist()}); "
        f"|M0-1| {drift:.2e}")
    assert err.max() < 1e-4
    assert drift < 1e-5
    op.close()

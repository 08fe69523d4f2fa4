"""GPU parity at full size for P1: the 512 x 512, phi = 0.6 geometry of the
plain workload run at p = 1 with its 64 start points as right-hand sides
(the kernel the P1 roofline figure measures, k_stage<float, 3> in its RK3
mode), against oracle values stored by
`tests/golden/make_full_golden.py pack512-p2 --p 1` (the oracle's Chebyshev
exponential on the full mesh, 8 sampled start points, all 20 Delta).

RK3 (FP32 state) over the whole Delta list to 50 ms (about 290k steps):
1e-4 on Sigma at every Delta, mass within 1e-5.
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
                      "pack512-p2_p1_oracle.json")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_fullsize_p1_rk3_all_deltas():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1907_06191_amd import dgd
    with open(GOLDEN) as f:
        gold = json.load(f)
    assert gold["p"] == 1
    c = config(gold["workload"])
    g = make_geometry(c["L"], c["N"], c["geom_seed"], phi=c["phi"], n_disks=c["n_disks"])
    pts = start_points(g.disks, g.L, g.N, c["R"], np.random.default_rng(c["point_seed"]))
    idx = np.asarray(gold["sample_index"])
    assert np.array_equal(pts[idx], np.asarray(gold["points"]))
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    assert mesh.info()["n_active"] == gold["n_elements"]
    say(f"full-size RK3 P1 FP32: {gold['n_elements']} elements, {pts.shape[0]} points, "
        f"dt {gold['dt_nom']:.4e} ms, {len(gold['deltas'])} Delta to {gold['deltas'][-1]:.0f} ms")
    op = dgd.Operator(mesh, 1, c["D"], c["eta"], dgd.DGD_FP32, dt_max_ms=gold["dt_nom"])
    run = dgd.Run(op, pts, c["sigma0"])
    assert dgd.dgd_run_kernel(run.handle)[0] == "valu"
    run.close()
    sig, mom = op.solve(pts, c["sigma0"], gold["deltas"])
    ref = omom.sigma_a(np.asarray(gold["moments"]))
    err = omom.rel_err(sig[idx], ref)
    drift = np.abs(mom[..., 0] - 1).max()
    say(f"  max rel err vs oracle {err.max():.2e} (per Delta {np.round(err.max(axis=0), 8).tolist()}); "
        f"|M0-1| {drift:.2e}")
    assert err.max() < 1e-4
    assert drift < 1e-5
    op.close()
    mesh.close()

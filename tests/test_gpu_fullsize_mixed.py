"""The mixed form (the paper's own formulation, every pixel kept, k = 0 in
axon cells) at full size: the 512 x 512, phi = 0.6, P2 workload in the
launch configuration the benchmark's mixed-form leg times (FP32 state,
autotuned shape, its own step rule), on the 8 start points sampled by the
stored oracle values, over the first two Delta.

The oracle's mixed form is too slow at this size, so the checks are the
properties that hold at any size: unit mass (zero-flux walls and box),
axon cells exactly zero, Sigma symmetric positive definite and below the
free-space value sigma0^2 + 2 D Delta (walls only hinder), and agreement
with the stored primal-form oracle values within the difference of the two
discretisations (5e-2 relative on Sigma).
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


def test_fullsize_mixed_form_properties():
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
    assert np.array_equal(pts[idx], np.asarray(gold["points"]))
    sel = pts[idx]
    deltas = gold["deltas"][:2]
    mesh = dgd.Mesh(g.L, g.N, np.zeros((0, 3)))
    op = dgd.MixedOperator(mesh, g.disks, 2, c["D"], dgd.DGD_FP32)
    dt, rho = dgd.dgd_operator_dt(op.handle)
    E = mesh.info()["n_active"]
    say(f"full-size mixed form: {E} triangles, dt {dt:.4e} ms, spectral radius {rho:.4e}/ms, "
        f"Delta {deltas}")
    R = sel.shape[0]
    run = dgd.Run(op, sel, c["sigma0"])
    sig = []
    prev = 0.0
    for d in deltas:
        n = int(np.ceil((d - prev) / dt - 1e-9))
        run.advance(n, (d - prev) / n)
        prev = d
        mom = run.moments()
        sig.append(omom.sigma_a(mom))
        say(f"  Delta {d:.4f} ms after {n} steps: |M0 - 1| {np.abs(mom[:, 0] - 1).max():.2e}")
        assert np.abs(mom[:, 0] - 1).max() < 1e-5
    st = dgd.dgd_run_get_state(run.handle, E * 6 * R, np.float32).reshape(E, 6 * R)
    run.close()
    # axon cells: the cells the primal mesh removes
    removed = dgd.Mesh(g.L, g.N, g.disks)
    act = np.ones((g.N, g.N), dtype=bool)
    ci_a, cj_a, _ = removed.elements()
    act[:] = False
    act[cj_a, ci_a] = True
    ci, cj, _ = mesh.elements()
    axon = ~act[cj, ci]
    say(f"  {int(axon.sum())} axon elements, max |u| there {np.abs(st[axon]).max():.1e}")
    assert axon.sum() > 0 and np.abs(st[axon]).max() == 0.0
    sig = np.stack(sig, axis=1)                                   # [R, 2, 3]
    ref = omom.sigma_a(np.asarray(gold["moments"])[:, :2])
    for k, d in enumerate(deltas):
        S = sig[:, k]
        assert (S[:, 0] > 0).all() and (S[:, 0] * S[:, 2] - S[:, 1] ** 2 > 0).all()
        free = c["sigma0"] ** 2 + 2 * c["D"] * d
        assert (S[:, 0] < free).all() and (S[:, 2] < free).all()
    diff = omom.rel_err(sig, ref)
    say(f"  Sigma vs the primal form's oracle values: max rel diff {diff.max():.2e}")
    assert diff.max() < 5e-2
    op.close()

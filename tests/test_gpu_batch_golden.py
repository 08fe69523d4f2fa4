"""GPU parity of the batched workload on its own geometries: 16 of the 256
seeded members (8 at P1, 8 at P2, spread over grid edges 128..512 at
h = 100/512 um and packing fractions 0.4..0.7), all 16 start points of
each, solved together through dgd_eap_solve_batch (one persistent run per
degree group, autotuned shapes, library step rule), against oracle values
stored by tests/golden/make_batch_golden.py (the oracle's Chebyshev
exponential on each full mesh).  1e-4 on Sigma at the first two Delta,
mass within 1e-5.
"""

import json
import os
import sys

import numpy as np
import pytest

from oracle import moments as omom
from workloads.configs import _batch_one

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "batch256-p12_oracle.json")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_batch_members_against_oracle():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1907_06191_amd import dgd
    with open(GOLDEN) as f:
        gold = json.load(f)
    nd = 2
    deltas = gold["deltas"][:nd]
    members = gold["members"]
    assert len(members) >= 16 and {m["p"] for m in members} == {1, 2}
    meshes, ops, pts = [], [], []
    for rec in members:
        geo, p_pts, p = _batch_one(rec["index"])
        assert p == rec["p"] and geo.N == rec["N"]
        assert np.array_equal(p_pts, np.asarray(rec["points"]))
        m = dgd.Mesh(geo.L, geo.N, geo.disks)
        assert m.info()["n_active"] == rec["n_elements"]
        meshes.append(m)
        ops.append(dgd.Operator(m, p, gold["D"], gold["eta"], dgd.DGD_FP32))
        pts.append(p_pts)
    pts = np.stack(pts)
    say(f"batch golden: {len(members)} geometries (N {[m['N'] for m in members]}), "
        f"{pts.shape[1]} start points each, Delta {deltas}")
    sig, mom = dgd.dgd_eap_solve_batch(ops, pts, gold["sigma0"], deltas)
    worst = 0.0
    for g, rec in enumerate(members):
        ref = omom.sigma_a(np.asarray(rec["moments"])[:, :nd])
        err = omom.rel_err(sig[g], ref)
        worst = max(worst, float(err.max()))
        assert err.max() < 1e-4, (rec["index"], err.max())
    drift = np.abs(mom[..., 0] - 1).max()
    say(f"  max rel err vs oracle {worst:.2e}; |M0-1| {drift:.2e}")
    assert drift < 1e-5
    for o in ops:
        o.close()
    for m in meshes:
        m.close()

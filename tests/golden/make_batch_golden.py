"""Write oracle values for parity of the batched workload on sampled members.

    python tests/golden/make_batch_golden.py --geoms 16 --deltas 3 --workers 8

The batched workload has 256 seeded geometries (grid edge 128..512 at
h = 100/512 um, packing fraction 0.4..0.7, P1 or P2, 16 start points each).
This script samples ``--geoms`` of them spread over grid size and degree
(half P1, half P2, each half taken at evenly spaced ranks of the grid edge),
assembles the FP64 oracle on each full mesh, and carries all 16 start points
of each through the first ``--deltas`` diffusion times with the oracle's
Chebyshev exponential (the exact semi-discrete flow).  It stores, per
sampled geometry, its index, degree, mesh size, the oracle's nominal step
and the six moments per (start point, Delta).  Calls nothing but oracle/ and
the seeded input generator.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import solve as osolve  # noqa: E402
from workloads import CONFIGS, batch_geometry_params  # noqa: E402
from workloads.configs import _batch_one  # noqa: E402


def sample_members(n_geoms: int, n_total: int) -> list:
    """Indices of n_geoms members: n_geoms/2 per degree, at evenly spaced
    ranks of the grid edge within that degree."""
    prm = [batch_geometry_params(g) for g in range(n_total)]
    out = []
    for p in (1, 2):
        idx = sorted((g for g in range(n_total) if prm[g]["p"] == p), key=lambda g: prm[g]["N"])
        k = n_geoms // 2 if p == 1 else n_geoms - n_geoms // 2
        pos = np.linspace(0, len(idx) - 1, k).round().astype(int)
        out.extend(idx[i] for i in pos)
    return sorted(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--geoms", type=int, default=16)
    ap.add_argument("--deltas", type=int, default=3)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    c = CONFIGS["batch256-p12"]
    members = sample_members(args.geoms, c["n_geoms"])
    deltas = list(c["deltas"][: args.deltas])
    recs = []
    t_all = time.time()
    for g in members:
        geo, pts, p = _batch_one(g)
        t0 = time.time()
        prob = osolve.prepare(geo.L, geo.N, geo.disks, p, c["D"], c["eta"])
        mom = osolve.solve(prob, pts, c["sigma0"], deltas, method="cheb", workers=args.workers)
        el = time.time() - t0
        print(f"geometry {g}: N {geo.N}, p {p}, {prob.op.mesh.n_elements} elements, "
              f"{el:.0f}s", flush=True)
        recs.append(dict(index=int(g), N=int(geo.N), L=float(geo.L), p=int(p),
                         n_disks=int(geo.disks.shape[0]),
                         n_elements=int(prob.op.mesh.n_elements),
                         dt_nom=prob.dt["dt_nom"], lambda_max=prob.dt["lambda_max"],
                         points=pts.tolist(), moments=mom.tolist(), oracle_seconds=el))
    out = dict(workload="batch256-p12", D=c["D"], eta=c["eta"], sigma0=c["sigma0"],
               deltas=deltas, method="chebyshev", oracle_workers=args.workers,
               oracle_seconds=time.time() - t_all, members=recs)
    path = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                    "batch256-p12_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()

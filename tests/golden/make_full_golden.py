"""Write oracle values for parity at a workload's full size.

    python tests/golden/make_full_golden.py pack512-p2 --sample 8 --workers 8

Builds the workload's seeded geometry and start points, assembles the FP64
oracle on the full mesh, and carries a sample of the start points (every
R/sample-th one) through the whole Delta list with the oracle's Chebyshev
exponential (the exact semi-discrete flow).  Stores the oracle's nominal
step (so the GPU run uses the same step rule), its largest eigenvalue, and
the six moments per (sampled start point, Delta).  Calls nothing but
oracle/ and the seeded input generator.
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
from workloads import config, make_geometry, start_points  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--sample", type=int, default=8)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--p", type=int, default=None)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    c = config(args.workload)
    p = args.p or c["p"]
    g = make_geometry(c["L"], c["N"], c["geom_seed"], phi=c["phi"], n_disks=c["n_disks"])
    pts = start_points(g.disks, g.L, g.N, c["R"], np.random.default_rng(c["point_seed"]))
    idx = np.arange(0, c["R"], max(1, c["R"] // args.sample))[: args.sample]
    t0 = time.time()
    prob = osolve.prepare(g.L, g.N, g.disks, p, c["D"], c["eta"])
    print(f"assembled {prob.op.ndof} dofs, lambda_max {prob.dt['lambda_max']:.6e} "
          f"in {time.time() - t0:.0f}s", flush=True)
    t0 = time.time()
    mom = osolve.solve(prob, pts[idx], c["sigma0"], c["deltas"], method="cheb", workers=args.workers)
    el = time.time() - t0
    print(f"solved {len(idx)} start points in {el:.0f}s", flush=True)
    out = dict(
        workload=args.workload, p=p, D=c["D"], eta=c["eta"], sigma0=c["sigma0"],
        geom_seed=c["geom_seed"], point_seed=c["point_seed"], n_disks=int(g.disks.shape[0]),
        n_elements=int(prob.op.mesh.n_elements), dt_nom=prob.dt["dt_nom"],
        lambda_max=prob.dt["lambda_max"], dt_rule=prob.dt["rule"], method="chebyshev",
        sample_index=[int(i) for i in idx], points=pts[idx].tolist(), deltas=list(c["deltas"]),
        moments=mom.tolist(), oracle_seconds=el, oracle_workers=args.workers,
    )
    name = args.workload if args.p is None else f"{args.workload}_p{p}"
    path = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                    f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()

"""The synthetic workloads (sizes, seeds and Delta lists).

  box20-p1      20 um box, 64^2 grid, 8 disks, P1, FP64, 1 start point
  pack512-p2    100 um box, 512^2 grid, phi = 0.6, P2, FP32, 64 start points
  batch256-p12  256 geometries, grid edge 128..512 at h = 100/512 um, P1/P2
  pack256-p3    50 um box, 256^2 grid, phi = 0.65, P3, FP32, 128 start points

Seeds: base s = 19070619.  Workload with seed index k draws its geometry
with seed s + 100*k and its start points with s + 100*k + 1.  Batched geometry g
uses s + 300 + 1000*g and s + 301 + 1000*g; surrogate data reuse that rule
for g >= 256.

The paper's dense substrate (section 2.2, 1901 circles in a 50 um square) is
unpublished; these seeded packings stand in for it.  Where a workload gives
both a disk count and a packing fraction that disagree (a Gamma(4, mean 0.5)
radius has E[r^2] = 0.3125 um^2, so 300 disks cover ~3% of a 100 um square,
not 60%), the packing fraction controls and the count follows.
"""

from __future__ import annotations

import numpy as np

BASE_SEED = 19070619


def _logspace(lo, hi, n):
    k = np.arange(n)
    return lo * (hi / lo) ** (k / (n - 1))


CONFIGS = {
    # Plain FP64 P1, one solve, 64^2 grid on a 20 um box, 8 disks.
    "box20-p1": dict(seed_index=1, L=20.0, N=64, n_disks=8, phi=None, shape=4.0, mean=0.5,
                     p=1, R=1, precision="fp64", D=2.0, eta=10.0, sigma0=0.3,
                     deltas=[1.0, 2.0, 5.0]),
    # Plain FP32 P2 at scale: 512^2 grid on a 100 um box, phi = 0.6, 64 RHS.
    "pack512-p2": dict(seed_index=2, L=100.0, N=512, n_disks=None, phi=0.6, shape=4.0,
                       mean=0.5, p=2, R=64, precision="fp32", D=2.0, eta=10.0, sigma0=0.3,
                       deltas=list(_logspace(1.0, 50.0, 20))),
    # Batched: 256 uneven geometries, h = 100/512, P1/P2 mixed, 16 RHS each.
    "batch256-p12": dict(seed_index=3, n_geoms=256, h=100.0 / 512, R=16, precision="fp32",
                         D=2.0, eta=10.0, sigma0=0.3, deltas=list(_logspace(1.0, 50.0, 20))),
    # High order: P3 on a 256^2 grid over a 50 um box, phi = 0.65, 128 RHS.
    "pack256-p3": dict(seed_index=4, L=50.0, N=256, n_disks=None, phi=0.65, shape=4.0,
                       mean=0.5, p=3, R=128, precision="fp32", D=2.0, eta=10.0, sigma0=0.3,
                       deltas=list(_logspace(1.0, 30.0, 20))),
}


def config(name: str) -> dict:
    c = dict(CONFIGS[name])
    k = c.pop("seed_index")
    c["geom_seed"] = BASE_SEED + 100 * k
    c["point_seed"] = BASE_SEED + 100 * k + 1
    return c


def batch_geometry_params(g: int) -> dict:
    """Parameters of batched geometry g (grid edge, phi, Gamma law, p)."""
    rng = np.random.default_rng(BASE_SEED + 300 + 1000 * g)
    N = int(rng.integers(128, 513))
    phi = float(rng.uniform(0.4, 0.7))
    shape = float(rng.uniform(3.0, 6.0))
    mean = float(rng.uniform(0.4, 0.7))
    p = 1 if rng.random() < 0.5 else 2
    h = CONFIGS["batch256-p12"]["h"]
    return dict(N=N, L=N * h, phi=phi, shape=shape, mean=mean, p=p,
                geom_seed=BASE_SEED + 300 + 1000 * g + 7,
                point_seed=BASE_SEED + 301 + 1000 * g)


def _batch_one(g):
    from .geometry import make_geometry, start_points
    prm = batch_geometry_params(g)
    # proposals drawn 2048 at a time: the densest of these packings jam
    geo = make_geometry(prm["L"], prm["N"], prm["geom_seed"], phi=prm["phi"],
                        shape=prm["shape"], mean=prm["mean"], batch=2048)
    pts = start_points(geo.disks, geo.L, geo.N, CONFIGS["batch256-p12"]["R"],
                       np.random.default_rng(prm["point_seed"]))
    return geo, pts, prm["p"]


def batch_workload(n_geoms: int | None = None, workers: int = 1):
    """[(Geometry, start points [16, 2], p)] for the batched workload's
    geometries 0 .. n_geoms-1 (all 256 by default), drawn in parallel."""
    n = CONFIGS["batch256-p12"]["n_geoms"] if n_geoms is None else n_geoms
    if workers <= 1:
        return [_batch_one(g) for g in range(n)]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_batch_one, range(n), chunksize=1)

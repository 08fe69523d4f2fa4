"""Surrogate driver: DG-generated training data, ensemble training, and
prediction with DG fallback -- all arithmetic in libdgd's kernels.

    python -m paper_1907_06191_amd.surrogate --train-geoms 512 --test-geoms 128

Data recipe.  Geometries follow the batched workload's recipe (packing
fraction ~ U(0.4, 0.7), Gamma shape ~ U(3, 6), mean ~ U(0.4, 0.7) um,
16 start points, the 20 log-spaced Delta in [1, 50] ms, h = 100/512 um) on
a fixed 64 x 64 grid, so the 64 x 64 occupancy image is exactly the
removed-cell mask and the DG cost of thousands of solves stays affordable.
DG solves use P1 (the coarser half of the workload's degree mix; P2 needs
7x more steps).  Target per (geometry, Delta): the start-point mean of
Sigma about the start point, divided by 2 D Delta, entries (xx, xy, yy).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1907_06191_amd import dgd  # noqa: E402

GRID = 64
H = 100.0 / 512
D = 2.0
SIGMA0 = 0.3
ETA = 10.0


def deltas_default():
    k = np.arange(20)
    return 1.0 * 50.0 ** (k / 19)


def geometry(g: int, grid: int = GRID):
    """Geometry g of the surrogate recipe (seeded; g counts from 256 so the
    batched workload's own geometries 0..255 are never reused)."""
    from workloads import make_geometry, start_points
    from workloads.configs import BASE_SEED
    rng = np.random.default_rng(BASE_SEED + 300 + 1000 * (256 + g))
    phi = float(rng.uniform(0.4, 0.7))
    shape = float(rng.uniform(3.0, 6.0))
    mean = float(rng.uniform(0.4, 0.7))
    geo = make_geometry(grid * H, grid, BASE_SEED + 300 + 1000 * (256 + g) + 7, phi=phi,
                        shape=shape, mean=mean, batch=2048)
    pts = start_points(geo.disks, geo.L, geo.N, 16,
                       np.random.default_rng(BASE_SEED + 301 + 1000 * (256 + g)))
    return geo, pts


def geometries(ids, workers=8, grid=GRID):
    if workers <= 1:
        return [geometry(g, grid) for g in ids]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.starmap(geometry, [(g, grid) for g in ids], chunksize=1)


def dg_targets(geos, deltas, p=1, dt_max=0.0, chunk=64, label="DG"):
    """Batched DG solves of the geometries, `chunk` per batch; returns
    (images [G][64][64], targets [G][nDelta][3], seconds of the solves)."""
    meshes = [dgd.Mesh(g.L, g.N, g.disks) for g, _ in geos]
    ops = [dgd.Operator(m, p, D, ETA, dgd.DGD_FP32, dt_max_ms=dt_max) for m in meshes]
    pts = np.stack([pp for _, pp in geos])
    sig = []
    el = 0.0
    for i in range(0, len(ops), chunk):
        t0 = time.perf_counter()
        s, _ = dgd.dgd_eap_solve_batch(ops[i:i + chunk], pts[i:i + chunk], SIGMA0, deltas)
        el += time.perf_counter() - t0
        sig.append(s)
        print(f"{label}: {min(i + chunk, len(ops))}/{len(ops)} geometries solved, {el:.0f}s",
              flush=True)
    sig = np.concatenate(sig)
    scale = 2.0 * D * np.asarray(deltas)[None, :, None]
    targets = sig.mean(axis=1) / scale                       # [G][nDelta][3]
    images = np.stack([dgd.dgd_mesh_occupancy(m.handle, GRID) for m in meshes])
    return images, targets, el


def flatten(images, targets, deltas):
    G, nd = targets.shape[:2]
    im = np.repeat(images, nd, axis=0)
    ld = np.tile(np.log(np.asarray(deltas)), G)
    return im, ld, targets.reshape(G * nd, 3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-geoms", type=int, default=512)
    ap.add_argument("--test-geoms", type=int, default=128)
    ap.add_argument("--members", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--threshold", type=float, default=1e-3)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    deltas = deltas_default()
    rep = {"grid": GRID, "p": 1, "deltas_ms": list(deltas)}
    t0 = time.time()
    train = geometries(range(args.train_geoms), args.workers)
    test = geometries(range(args.train_geoms, args.train_geoms + args.test_geoms), args.workers)
    rep["geometry_seconds"] = time.time() - t0
    print(f"geometries: {len(train)} train, {len(test)} test in {rep['geometry_seconds']:.0f}s", flush=True)
    im_tr, tg_tr, t_tr = dg_targets(train, deltas, label="DG train")
    im_te, tg_te, t_te = dg_targets(test, deltas, label="DG test")
    rep["dg_seconds_train"] = t_tr
    rep["dg_seconds_test"] = t_te
    print(f"DG data: train {t_tr:.0f}s, test {t_te:.0f}s", flush=True)
    X, L, Y = flatten(im_tr, tg_tr, deltas)
    s = dgd.Surrogate(n_members=args.members, channels=32, hidden=256, seed=1907)
    t0 = time.perf_counter()
    losses = s.train(X, L, Y, epochs=args.epochs, batch=args.batch, lr=args.lr, shuffle_seed=619)
    rep["train_seconds"] = time.perf_counter() - t0
    rep["final_train_loss"] = losses[:, -1].tolist()
    print(f"trained {args.members} members in {rep['train_seconds']:.0f}s, loss {losses[:, -1]}", flush=True)
    Xt, Lt, Yt = flatten(im_te, tg_te, deltas)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mean, spread, fb = s.predict(Xt, Lt, threshold=args.threshold)
    t_pred = time.perf_counter() - t0
    err = np.sqrt(((mean - Yt) ** 2).sum(1) + (mean[:, 1] - Yt[:, 1]) ** 2) / \
        np.sqrt((Yt ** 2).sum(1) + Yt[:, 1] ** 2)
    n = Yt.shape[0]
    frac_fb = float(fb.mean())
    # time per query: DG-only = the test set's batched DG time per (geometry, Delta)
    dg_per_query = t_te / n
    sur_per_query = t_pred / n + frac_fb * dg_per_query
    rep.update(
        n_test_queries=n, predict_seconds=t_pred, fallback_rate=frac_fb,
        rel_err_all_median=float(np.median(err)), rel_err_all_p95=float(np.percentile(err, 95)),
        rel_err_accepted_max=float(err[~fb].max()) if (~fb).any() else None,
        rel_err_accepted_median=float(np.median(err[~fb])) if (~fb).any() else None,
        spread_median=float(np.median(spread)),
        dg_queries_per_s=1.0 / dg_per_query, surrogate_queries_per_s=1.0 / sur_per_query,
        gain=dg_per_query / sur_per_query)
    print(json.dumps(rep), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()

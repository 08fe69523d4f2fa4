"""Surrogate driver: DG-generated training data, ensemble training, and
prediction with DG fallback -- all arithmetic in libdgd's kernels.

    python -m paper_1907_06191_amd.surrogate --train-geoms 1250 --test-geoms 128 \
        --epochs 20 --weights surrogate_weights.npz --out report.json

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
    """Batched DG solves of the geometries, `chunk` per batch.  Returns
    (images [G][64][64], targets [G][nDelta][3], halves [2][G][nDelta][3],
    seconds of the solves): the target is the mean over the 16 start points
    of Sigma / (2 D Delta) as (xx, xy, yy); `halves` are the same means over
    start points 0..7 and 8..15 (their half-difference measures the
    sampling noise of the 16-point target)."""
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
    sig = np.concatenate(sig)                                  # [G][16][nDelta][3]
    scale = 2.0 * D * np.asarray(deltas)[None, :, None]
    targets = sig.mean(axis=1) / scale
    halves = np.stack([sig[:, :8].mean(axis=1) / scale, sig[:, 8:].mean(axis=1) / scale])
    images = np.stack([dgd.dgd_mesh_occupancy(m.handle, GRID) for m in meshes])
    for o in ops:
        o.close()
    for m in meshes:
        m.close()
    return images, targets, halves, el


def augment(images, targets):
    """The mesh's exact symmetries: the transpose (x, y) -> (y, x) maps the
    pixel triangulation to itself (its diagonals run along x = y) and swaps
    Sigma_xx and Sigma_yy; the half turn (x, y) -> (L - x, L - y) maps it to
    itself (T0 <-> T1) and leaves Sigma unchanged.  Transposed or rotated
    start points give exactly these Sigma, so the four images of a geometry
    under {identity, transpose, half turn, both} are exact DG samples."""
    t_sw = targets[..., ::-1]
    tr = np.swapaxes(images, 1, 2)
    rot = images[:, ::-1, ::-1]
    both = np.swapaxes(rot, 1, 2)
    return (np.concatenate([images, tr, rot, both]),
            np.concatenate([targets, t_sw, targets, t_sw]))


def flatten(images, targets, deltas):
    G, nd = targets.shape[:2]
    im = np.repeat(images, nd, axis=0)
    ld = np.tile(np.log(np.asarray(deltas)), G)
    return im, ld, targets.reshape(G * nd, 3)


def rel_err(a, b):
    """Frobenius norm of the symmetric 2 x 2 difference over that of b, per
    row of (xx, xy, yy)."""
    num = np.sqrt(((a - b) ** 2).sum(-1) + (a[..., 1] - b[..., 1]) ** 2)
    den = np.sqrt((b ** 2).sum(-1) + b[..., 1] ** 2)
    return num / den


def evaluate(s, images, targets, halves, deltas, dg_seconds, thresholds):
    """Surrogate against the DG solve on held-out geometries: error of the
    ensemble mean, the 16-point target's sampling noise (half the distance
    between the two 8-point halves), and per spread threshold the fallback
    rate, the error of the accepted answers and the gain in queries per
    second over answering every query with the DG solve."""
    import torch
    X, Lq, Y = flatten(images, targets, deltas)
    n = Y.shape[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mean, spread, _ = s.predict(X, Lq, threshold=thresholds[0])
    t_pred = time.perf_counter() - t0
    err = rel_err(mean, Y)
    noise = rel_err(0.5 * (halves[0] - halves[1]).reshape(n, 3) + Y, Y)
    G, nd = targets.shape[:2]
    # a fallback needs its geometry's DG solve up to that Delta: the time of
    # a solve grows linearly with the last Delta it reaches (fixed step)
    t_geo = dg_seconds / G
    dl = np.asarray(deltas)
    rep = {"n_queries": n, "predict_seconds": t_pred, "dg_seconds": dg_seconds,
           "dg_queries_per_s": n / dg_seconds, "surrogate_only_queries_per_s": n / t_pred,
           "rel_err_median": float(np.median(err)), "rel_err_p95": float(np.percentile(err, 95)),
           "noise_floor_median": float(np.median(noise)),
           "noise_floor_p95": float(np.percentile(noise, 95)),
           "spread_median": float(np.median(spread)), "by_threshold": []}
    for thr in thresholds:
        fb = spread > thr
        frac = float(fb.mean())
        need = np.where(fb.reshape(G, nd), dl[None, :], 0.0).max(axis=1) / dl[-1]
        t_total = t_pred + t_geo * float(need.sum())
        acc = ~fb
        rep["by_threshold"].append({
            "threshold": thr, "fallback_rate": frac, "gain": dg_seconds / t_total,
            "geometries_solved": int((need > 0).sum()),
            "accepted": int(acc.sum()),
            "accepted_rel_err_median": float(np.median(err[acc])) if acc.any() else None,
            "accepted_rel_err_max": float(err[acc].max()) if acc.any() else None,
            "answer_rel_err_median": float(np.median(np.where(fb, 0.0, err)))})
    return rep, mean, spread


def speed(members=4, n=8192):
    """Throughput of the training and inference kernels on synthetic data:
    one epoch over n random occupancy images (after a warm-up epoch on 512),
    then prediction of 2n queries in batches of 4096."""
    import torch
    rng = np.random.default_rng(5)
    imgs = (rng.random((n, GRID, GRID)) < 0.5).astype(np.uint8)
    ld = rng.uniform(0, np.log(50), n)
    tg = rng.uniform(0.2, 0.8, (n, 3))
    s = dgd.Surrogate(n_members=members, channels=32, hidden=256, seed=1)
    s.train(imgs[:512], ld[:512], tg[:512], epochs=1, batch=256)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.train(imgs, ld, tg, epochs=1, batch=256)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    print(f"train: {members * n / t:.0f} sample-passes/s ({t:.2f}s for {members} members x {n})",
          flush=True)
    big, bl = np.repeat(imgs, 2, axis=0), np.repeat(ld, 2)
    s.predict(big[:4096], bl[:4096])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.predict(big, bl)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    print(f"predict: {big.shape[0] / t:.0f} queries/s ({members} members, batches of 4096)", flush=True)
    s.close()


THRESHOLDS = [1e-3, 3e-3, 1e-2, 3e-2, 1e-1]
TEST_FIRST = 1250       # held-out geometries are numbered from here


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-geoms", type=int, default=1250)
    ap.add_argument("--test-geoms", type=int, default=128)
    ap.add_argument("--members", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--no-augment", dest="augment", action="store_false")
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--save-data", default=None, help="write the DG data set here (.npz) and stop")
    ap.add_argument("--load-data", default=None, help="read the DG data set from here (.npz)")
    ap.add_argument("--weights", default=None, help="write the trained members here (.npz)")
    ap.add_argument("--out", default=None, help="write the report here (.json)")
    ap.add_argument("--speed", action="store_true",
                    help="only time training and prediction on synthetic data and stop")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    if args.speed:
        speed(args.members)
        return
    deltas = deltas_default()
    rep = {"grid": GRID, "p": 1, "deltas_ms": list(deltas), "augment": args.augment,
           "train_geoms": args.train_geoms, "test_geoms": args.test_geoms, "epochs": args.epochs}
    if args.load_data:
        z = np.load(args.load_data)
        im_tr, tg_tr, hv_tr, im_te, tg_te, hv_te = (z[k] for k in
                                                     ("im_tr", "tg_tr", "hv_tr", "im_te", "tg_te", "hv_te"))
        t_tr, t_te = float(z["t_tr"]), float(z["t_te"])
        rep["train_geoms"], rep["test_geoms"] = int(im_tr.shape[0]), int(im_te.shape[0])
    else:
        t0 = time.time()
        train = geometries(range(args.train_geoms), args.workers)
        test = geometries(range(TEST_FIRST, TEST_FIRST + args.test_geoms), args.workers)
        rep["geometry_seconds"] = time.time() - t0
        print(f"geometries: {len(train)} train, {len(test)} test in {rep['geometry_seconds']:.0f}s",
              flush=True)
        im_tr, tg_tr, hv_tr, t_tr = dg_targets(train, deltas, label="DG train")
        im_te, tg_te, hv_te, t_te = dg_targets(test, deltas, label="DG test")
        if args.save_data:
            np.savez_compressed(args.save_data, im_tr=im_tr, tg_tr=tg_tr, hv_tr=hv_tr, im_te=im_te,
                                tg_te=tg_te, hv_te=hv_te, t_tr=t_tr, t_te=t_te)
            print(f"wrote {args.save_data}", flush=True)
            return
    rep["dg_seconds_train"] = t_tr
    rep["dg_seconds_test"] = t_te
    noise_tr = rel_err(0.5 * (hv_tr[0] - hv_tr[1]) + tg_tr, tg_tr)
    rep["train_noise_floor_median"] = float(np.median(noise_tr))
    if args.augment:
        im_tr, tg_tr = augment(im_tr, tg_tr)
    X, L, Y = flatten(im_tr, tg_tr, deltas)
    rep["train_samples"] = int(Y.shape[0])
    s = dgd.Surrogate(n_members=args.members, channels=32, hidden=256, seed=1907)
    t0 = time.perf_counter()
    # one epoch per call (the optimizer state persists in the surrogate), a
    # cosine-decayed step size, a fresh shuffle each epoch
    for e in range(args.epochs):
        lr = args.lr * max(0.5 * (1.0 + np.cos(np.pi * e / args.epochs)), 0.05)
        losses = s.train(X, L, Y, epochs=1, batch=args.batch, lr=lr, shuffle_seed=619 + 7919 * e)
        print(f"epoch {e + 1}/{args.epochs}: lr {lr:.2e}, train loss {losses[:, -1]}, "
              f"{time.perf_counter() - t0:.0f}s", flush=True)
    rep["train_seconds"] = time.perf_counter() - t0
    rep["train_loss"] = losses[:, -1].tolist()
    print(f"trained {args.members} members on {Y.shape[0]} samples in {rep['train_seconds']:.0f}s, "
          f"loss {losses[:, -1]}", flush=True)
    ev, _, _ = evaluate(s, im_te, tg_te, hv_te, deltas, t_te, THRESHOLDS)
    rep["test"] = ev
    print(json.dumps(rep), flush=True)
    if args.weights:
        np.savez(args.weights, **{f"member{k}": dgd.dgd_surrogate_get_params(s.handle, k)
                                  for k in range(args.members)})
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()

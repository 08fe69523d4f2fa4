"""Throughput of the DG diffusion hot path on one MI355X.

Default workload: the plain solve at scale -- a 100 um box on a 512 x 512
pixel grid (h = 0.1953 um), seeded random-sequential-addition disks of
Gamma(4, mean 0.5 um) radius at packing fraction 0.6 removed as zero-flux
axons, P2 SIPG (6 nodes per triangle), 64 start points carried together as
64 right-hand sides, FP32 state with FP64 element arithmetic, FP64 moments.

A "step" is one SSP-RK3 time step of the whole state (three fused stage
launches: volume + face + lift + stage combine over every active triangle
and every right-hand side).  The timed region advances K steps from a state
already resident in HBM.  value = GDoF-updates/s, one update advancing one
DoF of one right-hand side by one RK3 step.

Also reported:
  * Sigma-solves/s of the RK3 path, projected from the measured step time
    and the full Delta-landing schedule;
  * Sigma-solves/s measured end to end (initial projection, the whole
    Delta list, moments) with the Chebyshev exponential integrator
    (--no-expm skips it);
  * --workload batch256-p12: the batched solve (256 uneven geometries, P1/P2
    groups, 16 start points each); --workload pack256-p3: P3, 128 start
    points (FP64 vector kernel, or with --precision bf16x3 BF16 hi/lo split
    products on matrix cores).

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes (FETCH_SIZE calibrated x 2.000, WRITE_SIZE x 1.000 by a
# plain 1 GiB copy), keyed by (workload, kernel, sha256 prefix of
# csrc/kernels.hip when the counters were taken, launch shape as elements
# per wave, waves, XCD order, workgroups): a changed kernel source or
# another tuned shape reports traffic null.  Summaries: profiles/.
MEASURED_TRAFFIC = {
    ("pack512-p2", "k_stage<float,6>", "b1461cb9119fe11a", (2, 4, 0, 26674)): 1129.6e6,
    ("pack512-p2", "k_stage<float,3>", "b1461cb9119fe11a", (2, 4, 0, 26674)): 566.5e6,
    ("pack256-p3", "k_stage<float,10>", "b1461cb9119fe11a", (1, 1, 1, 47872)): 660.0e6,
    ("pack256-p3", "k_stage_p3_mfma<true>", "b1461cb9119fe11a", (4, 1, 1, 11968)): 752.7e6,
}


def kernel_source_tag():
    import hashlib
    path = os.path.join(ROOT, "paper_1907_06191_amd", "csrc", "kernels.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def schedule_steps(deltas, dt):
    prev, n = 0.0, 0
    for d in deltas:
        n += max(int(np.ceil((d - prev) / dt - 1e-9)), 1)
        prev = d
    return n


def usable_cpus():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def host_workers():
    """Worker processes for the oracle: every CPU this process may use, up to
    the host's per-GPU share when the environment states one
    (OMP_NUM_THREADS)."""
    n = usable_cpus()
    share = os.environ.get("OMP_NUM_THREADS")
    if share and share.isdigit() and int(share) > 0:
        n = min(n, int(share))
    return max(1, n)


def cpu_baseline(g, pts, p, D, eta, sigma0, dt, lam, budget_s=20.0):
    """The FP64 oracle's SSP-RK3 on the same mesh, on a bounded sample:
    a few start points (one per worker process) for a fixed number of steps."""
    from oracle import solve as osolve
    t0 = time.time()
    prob = osolve.prepare(g.L, g.N, g.disks, p, D, eta, lam=lam)
    setup = time.time() - t0
    workers = host_workers()
    sample = pts[:workers]
    t0 = time.time()
    osolve.solve(prob, sample[:1], sigma0, [3 * dt], method="rk3", dt_nom=dt, workers=1)
    per_step = (time.time() - t0) / 3
    steps = max(3, int(budget_s / max(per_step, 1e-6)))
    t0 = time.time()
    osolve.solve(prob, sample, sigma0, [steps * dt], method="rk3", dt_nom=dt, workers=workers)
    el = time.time() - t0
    v = prob.op.ndof * sample.shape[0] * steps / el / 1e9
    return {"value": v, "unit": "GDoF-updates/s", "cores": workers, "kind": "oracle",
            "host_cpu_count": os.cpu_count(), "host_cpus_usable": usable_cpus(),
            "sample": f"oracle SSP-RK3 (scipy CSR, FP64) on the same mesh: {sample.shape[0]} start "
                      f"points x {steps} steps, one worker process per start point, {el:.1f} s "
                      f"(+{setup:.1f} s assembly, not timed)"}


def time_steps(advance, steps, stream):
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    advance(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1)


def copy_bandwidth(stream, nbytes=1 << 30, reps=10):
    """A plain device-to-device copy of nbytes timed with HIP events:
    (read + written bytes) / time, the bandwidth a streaming kernel reaches
    on this machine (context for the 8 TB/s peak)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    with torch.cuda.stream(stream):
        b.copy_(a)
        ms = time_steps(lambda k: [b.copy_(a) for _ in range(k)], reps, stream)
    del a, b
    gbs = 2.0 * nbytes * reps / (ms * 1e-3) / 1e9
    return {"gbs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "note": f"torch copy_ of {nbytes >> 20} MiB, {reps} repetitions, read + write bytes"}


def base_record(args, value, ms_per_step, dtype, config):
    return {
        "metric": "DG GDoF-updates/s (and Sigma-solves/s) at 1e-4 rel err vs FP64 oracle",
        "value": round(value, 4), "unit": "GDoF-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic (seeded RSA disk packing and start points)", "config": config,
    }


def plain(args):
    import torch
    from paper_1907_06191_amd import dgd
    from workloads import config, make_geometry, start_points

    c = config(args.workload)
    p = args.p or c["p"]
    t0 = time.time()
    g = make_geometry(c["L"], c["N"], c["geom_seed"], phi=c["phi"], n_disks=c["n_disks"])
    pts = start_points(g.disks, g.L, g.N, c["R"], np.random.default_rng(c["point_seed"]))
    log(f"geometry: {g.disks.shape[0]} disks in {time.time() - t0:.1f}s")
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    info = mesh.info()
    prec_name = args.precision or c["precision"]
    prec = {"fp64": dgd.DGD_FP64, "fp32": dgd.DGD_FP32, "bf16x3": dgd.DGD_BF16X3}[prec_name]
    t0 = time.time()
    op = dgd.Operator(mesh, p, c["D"], c["eta"], prec)
    dt, lam = dgd.dgd_operator_dt(op.handle)
    log(f"operator p={p}: {info['n_active']} triangles, lambda_max {lam:.4e}/ms, dt {dt:.4e} ms "
        f"({time.time() - t0:.1f}s)")
    R = pts.shape[0]
    npn = (p + 1) * (p + 2) // 2
    dof = info["n_active"] * npn * R
    stream = torch.cuda.Stream()
    ws = torch.empty(op.workspace_size(R), dtype=torch.uint8, device="cuda")
    run = dgd.Run(op, pts, c["sigma0"], workspace=ws, stream=stream)   # tunes the stage shape
    run.advance(args.warmup, dt)
    gpu_ms = time_steps(lambda k: run.advance(k, dt), args.steps, stream)
    ms_per_step = gpu_ms / args.steps
    value = dof * args.steps / (gpu_ms * 1e-3) / 1e9
    torch.cuda.synchronize()
    tm = time.perf_counter()
    mom = run.moments(check=False)
    mom_ms = (time.perf_counter() - tm) * 1e3
    nsteps = schedule_steps(c["deltas"], dt)
    solve_s = nsteps * ms_per_step * 1e-3 + len(c["deltas"]) * mom_ms * 1e-3
    launch_ms = gpu_ms / (3 * args.steps)
    sbytes = 8 if prec == dgd.DGD_FP64 else 4
    bytes_per_launch = 8.0 * sbytes / 3.0 * dof
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    kind, shape = dgd.dgd_run_kernel(run.handle)
    ts = "double" if sbytes == 8 else "float"
    kernel = {"mfma": "k_stage_p3_mfma<false>", "mfma_bf16x3": "k_stage_p3_mfma<true>",
              "packed": f"k_stage_packed<{ts},{npn},{4 if R <= 16 else 2}>",
              "valu": f"k_stage<{ts},{npn}>"}[kind]
    dtype = {"mfma": "f32 MFMA contraction + f64 mass correction, f32 state",
             "mfma_bf16x3": "bf16 hi/lo split MFMA contraction (4 products, f32 accumulate) "
                            "+ f64 mass correction, f32 state"}.get(
        kind, "f64 arithmetic, f32 state" if sbytes == 4 else "f64")
    out = base_record(args, value, ms_per_step, dtype, {
        "workload": f"{args.workload}: plain solve, {g.N}x{g.N} grid on [0,{g.L:g}]^2 um, "
                    f"phi={c['phi'] if c['phi'] is not None else str(c['n_disks']) + ' disks'}, "
                    f"P{p}, {R} start points as RHS",
        "active_triangles": info["n_active"], "dof_per_rhs": info["n_active"] * npn, "rhs": R,
        "p": p, "dt_ms": dt, "lambda_max_per_ms": lam, "steps_full_solve": nsteps,
        "deltas_ms": [round(x, 4) for x in c["deltas"]]})
    out["sigma_solves_per_s"] = round(R / solve_s, 6)
    out["sigma_solves_note"] = ("RK3 path, projected: measured ms/step x the full Delta-landing "
                                "schedule + measured moment reduction per Delta")
    out["mass_after_timed"] = float(np.abs(mom[:, 0] - 1).max())
    shape_key = (shape["epw"], shape["waves"], shape["xcd_remap"], shape["grid"])
    traffic = MEASURED_TRAFFIC.get((args.workload, kernel, kernel_source_tag(), shape_key))
    out["roofline"] = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
        "bytes_per_launch": bytes_per_launch, "launch_ms": round(launch_ms, 5), "launch_shape": shape,
        "traffic_note": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated), "
                        "null unless measured on this kernel source and launch shape"}
    if kind in ("mfma", "mfma_bf16x3"):
        # the method's flops per element and right-hand side: the 10 x 10
        # self block and one 10 x 10 block per present face (2 Np^2 (1 + faces));
        # interior faces count twice, once from each side.  The BF16 split
        # does the contraction four times (A_lo x_hi, A_mid x_hi, A_hi x_lo,
        # A_hi x_hi).
        method = 2.0 * npn * npn * (info["n_active"] + 2 * info["n_faces"]) * R
        nprod = 4 if kind == "mfma_bf16x3" else 1
        peak = 2500.0 if kind == "mfma_bf16x3" else 157.3
        issued = (2 * 4 * 16 * 16 * 32 * 2 if nprod == 4 else 10 * 16 * 16 * 4 * 2) * info["n_active"] * R / 16
        rate = method * nprod / (launch_ms * 1e-3) / 1e12
        out["roofline_mfma"] = {
            "bound": "mfma", "achieved": round(rate, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(rate / peak, 5), "flops_per_launch": method * nprod,
            "issued_flops_per_launch": issued,
            "dtype": ("bf16 MFMA (v_mfma_f32_16x16x32_bf16), 4 split products" if nprod == 4 else
                      "fp32 MFMA (v_mfma_f32_16x16x4_f32)"),
            "note": "method flops 2 Np^2 (1 + present faces) per element and right-hand side, "
                    "times the products the split needs; issued counts the padded 16 x 16 tiles"}
    run.close()
    if args.full_solve:
        out["full_solve"] = full_solve_leg(args, dgd, op, pts, c, dt, ws, stream, p)
    if args.expm:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sig, mom_e, napp = dgd.dgd_eap_solve_expm(op.handle, pts, c["sigma0"], c["deltas"])
        el = time.perf_counter() - t0
        out["expm"] = {"sigma_solves_per_s": round(R / el, 5), "seconds": round(el, 3),
                       "operator_applications": napp,
                       "gdof_applications_per_s": round(dof * napp / el / 1e9, 3),
                       "note": "measured end to end: projection, whole Delta list (Chebyshev "
                               "exponential, FP64 state), moments",
                       "max_mass_drift": float(np.abs(mom_e[..., 0] - 1).max())}
    if args.mixed:
        out["mixed_form"] = mixed_leg(args, dgd, g, pts, p, c, prec, R, out["sigma_solves_per_s"],
                                      info["n_active"])
    out["stage_shape_table"] = dgd.dgd_tune_export().strip().split("\n")
    out["hbm_copy"] = copy_bandwidth(stream)
    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = {"read": a.numel() * 4, "write": b.numel() * 4}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(g, pts, p, c["D"], c["eta"], c["sigma0"], dt, lam,
                                           args.cpu_budget)
    return out


def full_solve_leg(args, dgd, op, pts, c, dt, ws, stream, p):
    """The whole RK3 solve timed end to end: projection of the 64 pulses,
    every step of the Delta-landing schedule (each interval in ceil(span /
    dt) equal steps), the moments at every Delta.  Sigma about the start
    point (M2 / M0) is compared at the sampled start points with the values
    the oracle stored in tests/golden (its exact semi-discrete flow)."""
    import torch
    golden = os.path.join(ROOT, "tests", "golden", f"{args.workload}_oracle.json")
    gold = None
    if os.path.exists(golden) and p == c["p"]:
        with open(golden) as f:
            gold = json.load(f)
    R = pts.shape[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run = dgd.Run(op, pts, c["sigma0"], workspace=ws, stream=stream)
    prev, total, mom = 0.0, 0, []
    for d in c["deltas"]:
        n = max(int(np.ceil((d - prev) / dt - 1e-9)), 1)
        for a in range(0, n, 100000):
            run.advance(min(100000, n - a), (d - prev) / n)
            stream.synchronize()
            log(f"full solve: Delta {d:.4f} ms, {min(a + 100000, n)} / {n} steps, "
                f"{time.perf_counter() - t0:.0f} s")
        mom.append(run.moments(check=False))
        total += n
        prev = d
    el = time.perf_counter() - t0
    run.close()
    mom = np.stack(mom, axis=1)                   # [R][n_delta][6]
    res = {"sigma_solves_per_s": round(R / el, 6), "seconds": round(el, 2), "steps": total,
           "max_mass_drift": float(np.abs(mom[..., 0] - 1).max()),
           "note": "measured end to end: projection, every RK3 step of the Delta list, "
                   "moments at each Delta"}
    if gold is not None:
        idx = np.asarray(gold["sample_index"])
        ref = np.asarray(gold["moments"])
        s = mom[idx][..., 3:6] / mom[idx][..., 0:1]
        r = ref[..., 3:6] / ref[..., 0:1]
        fro = lambda v: np.sqrt(v[..., 0] ** 2 + 2.0 * v[..., 1] ** 2 + v[..., 2] ** 2)
        res["max_rel_err_sigma_vs_oracle"] = float((fro(s - r) / fro(r)).max())
        res["oracle_sample"] = (f"{len(idx)} of the {R} start points, all {len(c['deltas'])} Delta "
                                f"(tests/golden/{args.workload}_oracle.json)")
    return res


def mixed_leg(args, dgd, g, pts, p, c, prec, R, primal_sigma_per_s, n_ext):
    """The paper's own formulation on the same geometry and start points:
    every pixel kept, k = 0 in axon cells, two kernels per RK stage, its own
    (larger) stable step.  Timed like the primal run."""
    import torch
    t0 = time.time()
    mesh = dgd.Mesh(g.L, g.N, np.zeros((0, 3)))
    op = dgd.MixedOperator(mesh, g.disks, p, c["D"], prec)
    dt, rho = dgd.dgd_operator_dt(op.handle)
    E = mesh.info()["n_active"]
    npn = (p + 1) * (p + 2) // 2
    log(f"mixed form p={p}: {E} triangles (all pixels), spectral radius {rho:.4e}/ms, dt {dt:.4e} ms "
        f"({time.time() - t0:.1f}s)")
    stream = torch.cuda.Stream()
    ws = torch.empty(op.workspace_size(R), dtype=torch.uint8, device="cuda")
    run = dgd.Run(op, pts, c["sigma0"], workspace=ws, stream=stream)
    run.advance(args.warmup, dt)
    gpu_ms = time_steps(lambda k: run.advance(k, dt), args.steps, stream)
    ms_per_step = gpu_ms / args.steps
    mom = run.moments(check=False)
    run.close()
    nsteps = schedule_steps(c["deltas"], dt)
    solve_s = nsteps * ms_per_step * 1e-3
    out = {"dt_ms": dt, "spectral_radius_per_ms": rho, "triangles": E, "ms_per_step": round(ms_per_step, 5),
           "gdof_updates_per_s_extracellular": round(n_ext * npn * R * args.steps / (gpu_ms * 1e-3) / 1e9, 3),
           "extracellular_triangles": n_ext,
           "steps_full_solve": nsteps, "sigma_solves_per_s": round(R / solve_s, 6),
           "vs_primal_sigma_solves": round(R / solve_s / primal_sigma_per_s, 3),
           "mass_after_timed": float(np.abs(mom[:, 0] - 1).max()),
           "kernels": "k_mixed_grad + k_mixed_div per RK stage (axon elements skipped)",
           "note": "projected like the primal figure (ms/step x Delta-landing schedule); a different "
                   "discretisation of the same problem, checked against its own oracle; its Sigma "
                   "differs from the primal form's by up to 2.4% at this h (Delta = 1 ms)"}
    op.close()
    return out


def batched(args):
    import torch
    from paper_1907_06191_amd import dgd
    from workloads import batch_workload, config

    c = config("batch256-p12")
    n = args.geoms or c["n_geoms"]
    t0 = time.time()
    work = batch_workload(n, workers=args.workers)
    log(f"{n} geometries in {time.time() - t0:.0f}s")
    meshes = [dgd.Mesh(g.L, g.N, g.disks) for g, _, _ in work]
    ops = [dgd.Operator(m, p, c["D"], c["eta"], dgd.DGD_FP32) for m, (_, _, p) in zip(meshes, work)]
    pts = np.stack([pp for _, pp, _ in work])
    stream = torch.cuda.Stream()
    b = dgd.Batch(ops, pts, c["sigma0"], stream=stream)
    groups = b.groups()
    R = pts.shape[1]
    total_ms, total_updates, solve_s = 0.0, 0.0, 0.0
    per_group = []
    for k, gr in enumerate(groups):
        b.advance(k, args.warmup, gr["dt"])
        ms = time_steps(lambda s: b.advance(k, s, gr["dt"]), args.steps, stream)
        total_ms += ms
        total_updates += gr["dof"] * R * args.steps
        nsteps = schedule_steps(c["deltas"], gr["dt"])
        solve_s += nsteps * ms / args.steps * 1e-3
        per_group.append({"p": gr["p"], "geometries": gr["size"], "dof_per_rhs": gr["dof"],
                          "dt_ms": gr["dt"], "ms_per_step": round(ms / args.steps, 4),
                          "gdof_updates_per_s": round(gr["dof"] * R * args.steps / (ms * 1e-3) / 1e9, 2),
                          "steps_full_solve": nsteps})
    mom = b.moments(check=False)
    value = total_updates / (total_ms * 1e-3) / 1e9
    # algorithmic bytes per launch: 32 B per DoF-update / 3 launches per step
    for gr, pg in zip(groups, per_group):
        launch_ms = pg["ms_per_step"] / 3
        byts = 32.0 / 3.0 * gr["dof"] * R
        pg["roofline"] = {"bound": "hbm", "achieved": round(byts / (launch_ms * 1e-3) / 1e9, 1),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(byts / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "bytes_per_launch": byts, "launch_ms": round(launch_ms, 5)}
    out = base_record(args, value, total_ms / args.steps, "f64 arithmetic, f32 state", {
        "workload": f"batch256-p12: batched solve, {n} geometries (grid edge 128..512 at h=100/512 um, "
                    f"phi 0.4..0.7), P1/P2 groups, {R} start points each",
        "groups": per_group})
    # the dominant kernel: the group with the longest step
    top = max(range(len(groups)), key=lambda k: per_group[k]["ms_per_step"])
    npn = (groups[top]["p"] + 1) * (groups[top]["p"] + 2) // 2
    kern = (f"k_stage_packed<float,{npn},{4 if R <= 16 else 2}>" if R <= 32 else f"k_stage<float,{npn}>")
    out["roofline"] = dict(per_group[top]["roofline"], kernel=kern, traffic=None,
                           group=f"P{groups[top]['p']}",
                           traffic_note="HBM counters of this kernel on the batched workload: "
                                        "profiles/k_stage_packed_batch256-p12.md (taken on an earlier "
                                        "source with the same kernel body); null here")
    out["stage_shape_table"] = dgd.dgd_tune_export().strip().split("\n")
    out["sigma_solves_per_s"] = round(n * R / solve_s, 6)
    out["sigma_solves_note"] = "projected: measured ms/step per group x its full schedule"
    out["mass_after_timed"] = float(np.abs(mom[..., 0] - 1).max())
    out["ms_per_step_note"] = "sum over groups of one RK3 step of every geometry in the group"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="pack512-p2",
                    choices=["box20-p1", "pack512-p2", "batch256-p12", "pack256-p3"])
    ap.add_argument("--p", type=int, default=None, help="override polynomial degree")
    ap.add_argument("--geoms", type=int, default=0, help="batch256-p12: number of geometries (default all)")
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-expm", dest="expm", action="store_false")
    ap.add_argument("--full-solve", action="store_true",
                    help="also run the whole RK3 solve (every step of the Delta list) timed end to "
                         "end, checked at the sampled start points against the stored oracle values")
    ap.add_argument("--no-mixed", dest="mixed", action="store_false",
                    help="skip the mixed-form leg (the paper's own formulation on all pixels)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32", "bf16x3"],
                    help="operator precision (default: the workload's); bf16x3 = P3 stages as "
                         "BF16 hi/lo split products on matrix cores")
    ap.add_argument("--p3-mfma", type=int, default=2, choices=[0, 1, 2],
                    help="P3 FP32 stage kernel: 0 VALU, 1 matrix cores, 2 the faster (tuned)")
    ap.add_argument("--tune-file", default=None,
                    help="stage launch-shape table: merged in before the runs if the file "
                         "exists, written back after them (a run with a warm file does no tuning)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed region, copy 1 GiB device-to-device once (a plain "
                         "copy kernel of known size, to calibrate HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    from paper_1907_06191_amd import dgd
    dgd.dgd_set_option("p3_mfma", args.p3_mfma)
    if args.tune_file and os.path.exists(args.tune_file):
        with open(args.tune_file) as f:
            dgd.dgd_tune_import(f.read())
    out = batched(args) if args.workload == "batch256-p12" else plain(args)
    if args.tune_file:
        with open(args.tune_file, "w") as f:
            f.write(dgd.dgd_tune_export())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

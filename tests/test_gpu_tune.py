"""GPU: the stage-kernel autotuner.  Tuned shapes are valid, land in the
table under their key, and change no bit of a solve (every launch shape
computes each element and right-hand side in the same lane order)."""

import sys

import numpy as np
import pytest

from workloads import make_geometry, start_points

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dgd():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1907_06191_amd import dgd as d
    return d


def _case(nrhs, N=64, seed=41):
    h = 100.0 / 512
    g = make_geometry(N * h, N, 19070619 + 900 + seed, phi=0.6)
    pts = start_points(g.disks, g.L, g.N, nrhs, np.random.default_rng(19070619 + 901 + seed))
    return g, pts


@pytest.mark.parametrize("p,R,kernel", [(2, 64, "valu"), (1, 16, "packed"), (2, 32, "packed"),
                                        (3, 16, "mfma"), (3, 64, "mfma")])
def test_autotune_shape_valid_and_bit_invariant(dgd, p, R, kernel):
    g, pts = _case(R)
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, p, 2.0, 10.0, dgd.DGD_FP32)   # stable step from the auto rule
    E = mesh.info()["n_active"]
    say(f"autotune p={p} R={R} ({kernel}), {E} elements")
    # the kernel under test throughout (for P3 the autotuner may otherwise
    # pick the other kernel kind, whose arithmetic differs)
    dgd.dgd_set_option("p3_mfma", 1 if kernel == "mfma" else 0)
    try:
        dgd.dgd_tune_clear()
        shape, ms = dgd.dgd_autotune(op.handle, R)
        say(f"  best {shape}, {ms * 1e3:.1f} us per stage launch")
        assert shape["epw"] in (1, 2, 4) and shape["waves"] in (1, 2, 4)
        assert shape["xcd_remap"] in (0, 1) and shape["grid_per_cu"] in (0, 4, 8, 16)
        assert 0 < ms < 100
        table = dgd.dgd_tune_export()
        key = f"|np{(p + 1) * (p + 2) // 2}|fp32|{kernel}|R{R}|E2^{int(np.floor(np.log2(E)))} "
        assert key in table, table
        deltas = [0.002, 0.004]
        sig_t, mom_t = op.solve(pts, 0.3, deltas)
        dgd.dgd_set_option("autotune", 0)
        for epw, waves, grid in ((1, 4, 0), (2, 1, 512)):
            dgd.dgd_set_option("stage_epw", epw)
            dgd.dgd_set_option("stage_waves", waves)
            dgd.dgd_set_option("stage_grid", grid)
            sig_o, mom_o = op.solve(pts, 0.3, deltas)
            assert np.array_equal(mom_t, mom_o), (epw, waves, grid)
    finally:
        dgd.dgd_set_option("p3_mfma", 2)
        dgd.dgd_set_option("autotune", 1)
        dgd.dgd_set_option("stage_epw", 1)
        dgd.dgd_set_option("stage_waves", 4)
        dgd.dgd_set_option("stage_grid", 0)
    op.close()
    mesh.close()


def test_run_log_and_tune_cache(dgd, tmp_path):
    """DGD_RUN_LOG: a solve appends one JSON line with its configuration,
    step count, status, mass drift and the start-point mean of Sigma (equal
    to the returned Sigma's).  DGD_TUNE_CACHE: a newly tuned key is written
    to the file, and a fresh process that finds the file takes its shape
    without tuning."""
    import json
    import os
    import subprocess
    g, pts = _case(16, N=32, seed=43)
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, 1, 2.0, 10.0, dgd.DGD_FP32)
    log = tmp_path / "runs.jsonl"
    cache = tmp_path / "tune.txt"
    os.environ["DGD_RUN_LOG"] = str(log)
    os.environ["DGD_TUNE_CACHE"] = str(cache)
    try:
        dgd.dgd_tune_clear()
        say("run log and tune cache")
        sig, mom = op.solve(pts, 0.3, [0.01, 0.02])
    finally:
        del os.environ["DGD_RUN_LOG"]
        del os.environ["DGD_TUNE_CACHE"]
    rec = [json.loads(line) for line in log.read_text().splitlines()]
    assert len(rec) == 1 and rec[0]["entry"] == "dgd_eap_solve" and rec[0]["status"] == 0
    assert rec[0]["p"] == 1 and rec[0]["n_points"] == 16 and rec[0]["kernel"] == "packed"
    assert rec[0]["dt_rule"] == "stability" and rec[0]["steps"] > 0
    assert rec[0]["max_mass_drift"] == pytest.approx(np.abs(mom[..., 0] - 1).max())
    assert np.allclose(rec[0]["sigma_mean"], sig.mean(axis=0), rtol=1e-9, atol=0)
    table = cache.read_text()
    assert "|np3|fp32|packed|R16|" in table
    # a fresh process reads the cache: give the key an unusual shape and
    # check that the run takes it
    key = [line.split()[0] for line in table.splitlines() if "|packed|R16|" in line][0]
    cache.write_text(f"{key} 1 1 0 4 0.5\n")
    code = (
        "import sys, numpy as np; sys.path.insert(0, '.');"
        "from paper_1907_06191_amd import dgd; from workloads import make_geometry, start_points;"
        f"g = make_geometry({g.L!r}, {g.N}, 19070619 + 943, phi=0.6);"
        f"pts = start_points(g.disks, g.L, g.N, 16, np.random.default_rng(19070619 + 944));"
        "m = dgd.Mesh(g.L, g.N, g.disks); op = dgd.Operator(m, 1, 2.0, 10.0, dgd.DGD_FP32);"
        "r = dgd.Run(op, pts, 0.3); print(dgd.dgd_run_kernel(r.handle)[1])")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                         timeout=240, env=dict(os.environ, DGD_TUNE_CACHE=str(cache)))
    assert out.returncode == 0, out.stderr[-2000:]
    shape = eval(out.stdout.strip().splitlines()[-1])
    say(f"  shape from the cache in a fresh process: {shape}")
    assert (shape["epw"], shape["waves"], shape["xcd_remap"]) == (1, 1, 0)
    op.close()
    mesh.close()

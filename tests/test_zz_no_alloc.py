"""The allocation-free solve (dgd_eap_solve_noalloc) against dgd_eap_solve.

Both entry points run the same kernels on the same data (P2 FP64, P1 FP32
and P3 with BF16 hi/lo split products); the allocation-free
one keeps its buffers in the library's fixed device scratch, launches its
steps eagerly and uses the option's launch shape unless a tuned one exists.
The stage kernels give the same bits for every launch shape, so the two
solves must agree bit for bit.  Two calls in a row, the second on a smaller
mesh with fewer start points (the scratch keeps the first call's contents),
then the error paths: a run beyond the 64 MiB scratch (ENOMEM) and
point-mass data (EINVAL).
"""

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


CASES = [
    # (L, N, n_disks, p, precision, start points, Delta list): the second is smaller
    (10.0, 32, 5, 2, "fp64", 5, [0.01, 0.025]),
    (7.5, 24, 3, 2, "fp64", 2, [0.01, 0.025]),
    (10.0, 32, 5, 1, "fp32", 16, [0.02, 0.05]),
    (7.5, 24, 3, 1, "fp32", 3, [0.02, 0.05]),
    # P3 with BF16 hi/lo split products on matrix cores (multiples of 16 points)
    (10.0, 32, 5, 3, "bf16x3", 32, [0.005, 0.01]),
    (7.5, 24, 3, 3, "bf16x3", 16, [0.005, 0.01]),
]


def test_noalloc_matches_solve(dgd):
    for k, (L, N, nd, p, prec, R, deltas) in enumerate(CASES):
        say(f"noalloc case {k}: {N}^2 grid, {nd} disks, P{p} {prec}, {R} start points, Delta {deltas}")
        g = make_geometry(L, N, 19070619 + 40 + k, n_disks=nd)
        pts = start_points(g.disks, g.L, g.N, R, np.random.default_rng(19070619 + 50 + k))
        mesh = dgd.Mesh(g.L, g.N, g.disks)
        pr = {"fp64": dgd.DGD_FP64, "fp32": dgd.DGD_FP32, "bf16x3": dgd.DGD_BF16X3}[prec]
        op = dgd.Operator(mesh, p, 2.0, 10.0, pr)
        sig_a, mom_a = dgd.dgd_eap_solve(op.handle, pts, 0.3, deltas)
        sig_b, mom_b = dgd.dgd_eap_solve_noalloc(op.handle, pts, 0.3, deltas)
        say(f"  max |moment difference| = {np.abs(mom_a - mom_b).max():.3e}, "
            f"mass {np.abs(mom_b[..., 0] - 1).max():.2e}")
        assert np.array_equal(mom_a, mom_b)
        assert np.array_equal(sig_a, sig_b)
        op.close()
        mesh.close()


def test_noalloc_limits(dgd):
    say("noalloc limits: a run beyond the scratch, point-mass data")
    mesh = dgd.Mesh(25.0, 128, np.zeros((0, 3)))
    op = dgd.Operator(mesh, 1, 2.0, 10.0, dgd.DGD_FP64, dt_max_ms=1e-4)
    # 32768 triangles x 3 nodes x 64 right-hand sides x 8 B x 3 buffers = 151 MB
    pts = np.column_stack([np.linspace(10.0, 15.0, 64), np.full(64, 12.5)])
    with pytest.raises(dgd.DGDError) as e:
        dgd.dgd_eap_solve_noalloc(op.handle, pts, 0.3, [1e-3])
    assert e.value.code == dgd.DGD_ENOMEM and "64 MiB" in str(e.value)
    with pytest.raises(dgd.DGDError) as e:
        dgd.dgd_eap_solve_noalloc(op.handle, pts[:2], 0.0, [1e-3])
    assert e.value.code == dgd.DGD_EINVAL
    # the scratch still serves a run that fits after the refusals
    sig_a, mom_a = dgd.dgd_eap_solve(op.handle, pts[:4], 0.3, [2e-3])
    sig_b, mom_b = dgd.dgd_eap_solve_noalloc(op.handle, pts[:4], 0.3, [2e-3])
    assert np.array_equal(mom_a, mom_b)
    op.close()
    mesh.close()

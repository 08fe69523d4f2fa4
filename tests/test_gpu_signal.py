"""GPU parity of the q-space signal E(q) = int u exp(i q.(x - x0)) dx
against the oracle's signal on the same step schedule (FP64), against the
oracle's exact flow (FP32 state), and the properties that hold at any size
(E(0) = M0, the small-q expansion against the GPU's own FP64 moments)."""

import sys

import numpy as np
import pytest

from oracle import signal as osig
from oracle import solve as osolve
from oracle import timeint
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


def _qs(mags, n_dir, seed):
    ang = np.random.default_rng(seed).uniform(0, 2 * np.pi, n_dir)
    return np.array([[a * np.cos(t), a * np.sin(t)] for a in mags for t in ang])


def _case(nrhs, N, seed):
    h = 100.0 / 512
    g = make_geometry(N * h, N, 19070619 + 900 + seed, phi=0.6)
    pts = start_points(g.disks, g.L, g.N, nrhs, np.random.default_rng(19070619 + 901 + seed))
    return g, pts


@pytest.mark.parametrize("p", [1, 2, 3])
def test_signal_fp64_matches_oracle_rk3(dgd, p):
    g, pts = _case(3, 32, 61 + p)
    deltas = [0.02, 0.05]
    qs = np.concatenate([np.zeros((1, 2)), _qs([0.3, 1.0, 3.0], 5, p)])
    prob = osolve.prepare(g.L, g.N, g.disks, p, 2.0, 10.0)
    dt = prob.dt["dt_nom"]
    say(f"signal FP64 p={p}: {prob.op.mesh.n_elements} elements, {qs.shape[0]} wave vectors")
    U0 = osolve.initial_block(prob.op, pts, 0.3)
    ref = timeint.rk3(prob.op.L, U0, deltas, dt,
                      on_delta=lambda k, U: osig.signal(prob.op, U, pts, qs))
    ref = np.stack(ref, axis=1)                                      # [R, nDelta, nq]
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, p, 2.0, 10.0, dgd.DGD_FP64, dt_max_ms=dt)
    sig, mom = dgd.dgd_eap_solve_signal(op.handle, pts, 0.3, deltas, qs)
    err = np.abs(sig - ref).max()
    say(f"  max |E_gpu - E_oracle| = {err:.2e}")
    assert err < 1e-10            # the FP64 bar of the solve (|E| <= 1)
    assert np.abs(sig[..., 0].real - mom[..., 0]).max() < 1e-14


def test_signal_fp32_dense_packing_vs_exact_flow(dgd):
    g, pts = _case(8, 64, 71)
    deltas = [0.2, 0.5]
    qs = _qs([0.5, 1.5, 4.0], 6, 9)
    prob = osolve.prepare(g.L, g.N, g.disks, 2, 2.0, 10.0)
    dt = prob.dt["dt_nom"]
    say(f"signal FP32 P2: {prob.op.mesh.n_elements} elements, dt={dt:.3e}")
    U0 = osolve.initial_block(prob.op, pts, 0.3)
    ref = timeint.expm_deltas(prob.op.L, U0, deltas, prob.dt["b"],
                              on_delta=lambda k, U: osig.signal(prob.op, U, pts, qs))
    ref = np.stack(ref, axis=1)
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, 2, 2.0, 10.0, dgd.DGD_FP32, dt_max_ms=dt)
    sig, _ = dgd.dgd_eap_solve_signal(op.handle, pts, 0.3, deltas, qs)
    err = np.abs(sig - ref).max()
    say(f"  max |E_gpu - E_oracle| = {err:.2e}")
    assert err < 1e-5


def test_signal_rejects_bad_arguments(dgd):
    g, pts = _case(2, 16, 73)
    mesh = dgd.Mesh(g.L, g.N, g.disks)
    op = dgd.Operator(mesh, 1, 2.0, 10.0, dgd.DGD_FP64, dt_max_ms=1e-4)
    h = g.L / g.N
    with pytest.raises(dgd.DGDError) as e:
        dgd.dgd_eap_solve_signal(op.handle, pts, 0.3, [0.01], [[4.01 / h, 0.0]])
    assert e.value.code == dgd.DGD_EINVAL
    with pytest.raises(dgd.DGDError) as e:
        dgd.dgd_eap_solve_signal(op.handle, pts, 0.3, [0.01], [[np.nan, 0.0]])
    assert e.value.code == dgd.DGD_EINVAL

"""The whole oracle pipeline for one geometry and many start points.

Section 4.1 of the paper: for each start point x_i, solve the diffusion
problem from a pulse at x_i up to each diffusion time, normalise, and
estimate the covariance by quadrature.  ``solve`` returns the six moments
per (start point, Delta) from which every covariance reading follows
(``moments``).  Start points are split across worker processes in column
blocks when ``workers > 1``.
"""

from __future__ import annotations

import dataclasses
import os

import numpy as np

from . import bounds, initial, mesh as meshmod, moments as mom, sipg, timeint


@dataclasses.dataclass
class Problem:
    op: sipg.Operator
    dt: dict


def prepare(L, N, disks, p, D, eta, lam=None, outer="reflect") -> Problem:
    m = meshmod.build_mesh(L, N, disks)
    op = sipg.assemble(m, p, D, eta, outer=outer)
    return Problem(op=op, dt=bounds.dt_rule(op, lam))


def initial_block(op, points, sigma0):
    return np.stack([initial.project_gaussian(op, np.asarray(x), sigma0) for x in points], axis=1)


def _solve_block(args):
    op, points, sigma0, deltas, dt_nom, b, method = args
    U0 = initial_block(op, points, sigma0)

    def cb(k, U):
        return mom.moments(op, U, points)

    if method == "rk3":
        res = timeint.rk3(op.L, U0, deltas, dt_nom, on_delta=cb)
    else:
        res = timeint.expm_deltas(op.L, U0, deltas, b, on_delta=cb)
    return np.stack(res, axis=1)            # [R, nDelta, 6]


def solve(prob: Problem, points, sigma0, deltas, method="rk3", dt_nom=None,
          workers: int = 1) -> np.ndarray:
    """Moments [R, nDelta, 6] for every start point (row) and Delta."""
    points = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    dt_nom = prob.dt["dt_nom"] if dt_nom is None else dt_nom
    b = prob.dt["b"]
    if workers <= 1 or points.shape[0] == 1:
        return _solve_block((prob.op, points, sigma0, deltas, dt_nom, b, method))
    import multiprocessing as mp
    chunks = np.array_split(np.arange(points.shape[0]), min(workers, points.shape[0]))
    args = [(prob.op, points[c], sigma0, deltas, dt_nom, b, method) for c in chunks]
    ctx = mp.get_context("fork")
    with ctx.Pool(len(chunks)) as pool:
        parts = pool.map(_solve_block, args)
    return np.concatenate(parts, axis=0)


def default_workers() -> int:
    return max(1, (os.cpu_count() or 1))

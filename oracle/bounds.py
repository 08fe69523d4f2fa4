"""Spectral bound of M^-1 A and the time-step rule (oracle).

The paper advances in time "by a Runge-Kutta method" without naming the
scheme or the step (section 3.1).  Readings taken here:

* the scheme is SSP-RK3 (Shu-Osher form), whose stability polynomial
  R(z) = 1 + z + z^2/2 + z^3/6 satisfies |R(-x)| <= 1 on the real interval
  [0, X_RK3], X_RK3 ~= 2.5127 the real root of R(-x) = -1;
* the nominal step is dt_nom = min(0.1 h^2 / (D (p+1)^2), 0.9 X_RK3 / b),
  with b = 1.01 * lambda_max(M^-1 A): the first term is the workload's
  formula, which on its own is unstable at penalty eta = 10 for every p;
* the step lands on each requested time: for each interval
  (Delta_{k-1}, Delta_k], n_k = ceil((Delta_k - Delta_{k-1})/dt_nom - 1e-9)
  steps of dt_k = (Delta_k - Delta_{k-1})/n_k, with Delta_0 = 0.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import eigsh

from .sipg import Operator


def rk3_real_stability_limit() -> float:
    """Real root of x^3/6 - x^2/2 + x - 2 = 0, i.e. R(-x) = -1 for SSP-RK3."""
    roots = np.roots([1.0 / 6.0, -0.5, 1.0, -2.0])
    real = [r.real for r in roots if abs(r.imag) < 1e-12]
    x = max(real)
    # one Newton polish
    f = x ** 3 / 6 - x * x / 2 + x - 2
    df = x * x / 2 - x + 1
    return float(x - f / df)


X_RK3 = rk3_real_stability_limit()


def symmetric_operator(op: Operator) -> sp.csr_matrix:
    """B = C^-1 A C^-T with M = C C^T blockwise: symmetric and similar to M^-1 A."""
    mesh = op.mesh
    Np = op.Np
    E = mesh.n_elements
    blocks = []
    for e_o in (0, 1):
        Mo = op.mesh.h ** 2 * op.loc.Mhat[e_o]
        C = np.linalg.cholesky(Mo)
        blocks.append(np.linalg.inv(C))
    Cinv = np.zeros((E, Np, Np))
    for o in (0, 1):
        Cinv[mesh.orient == o] = blocks[o]
    Ci = sp.block_diag(list(Cinv), format="csr")
    return (Ci @ op.A @ Ci.T).tocsr()


def lambda_max(op: Operator, tol: float = 1e-10) -> float:
    """Largest eigenvalue of M^-1 A (Lanczos on the symmetric form, fixed start)."""
    B = symmetric_operator(op)
    n = B.shape[0]
    if n <= 1500:
        return float(np.linalg.eigvalsh(B.toarray())[-1])
    rng = np.random.default_rng(12345)
    v0 = rng.standard_normal(n)
    w = eigsh(B, k=1, which="LA", v0=v0, tol=tol, return_eigenvectors=False,
              ncv=64, maxiter=100000)
    return float(w[0])


def dt_rule(op: Operator, lam: float | None = None) -> dict:
    """Nominal step: min(workload formula, 0.9 X_RK3 / (1.01 lambda_max))."""
    h = op.mesh.h
    lam = lambda_max(op) if lam is None else lam
    b = 1.01 * lam
    dt_formula = 0.1 * h * h / (op.D * (op.p + 1) ** 2)
    dt_stab = 0.9 * X_RK3 / b
    return dict(dt_nom=min(dt_formula, dt_stab), dt_formula=dt_formula,
                dt_stab=dt_stab, lambda_max=lam, b=b,
                rule="stability" if dt_stab < dt_formula else "formula")


def schedule(deltas, dt_nom: float):
    """[(n_k, dt_k)] landing exactly on each Delta_k."""
    out = []
    prev = 0.0
    for d in deltas:
        span = float(d) - prev
        if not span > 0:
            raise ValueError("Delta list must be strictly increasing and positive")
        n = int(math.ceil(span / dt_nom - 1e-9))
        n = max(n, 1)
        out.append((n, span / n))
        prev = float(d)
    return out

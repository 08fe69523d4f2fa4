"""Time integration of du/dt = L u, L = -M^-1 A (oracle).

* ``rk3``: SSP-RK3 in Shu-Osher form with the Delta-landing schedule of
  ``bounds.schedule`` (the paper's "Runge-Kutta method", section 3.1, read
  as SSP-RK3):
      u1 = u + dt L u
      u2 = 3/4 u + 1/4 (u1 + dt L u1)
      u' = 1/3 u + 2/3 (u2 + dt L u2)
* ``expm_cheb``: u(t) = exp(t L) u0 by a Chebyshev expansion on the
  spectrum [-b, 0] (Tal-Ezer and Kosloff, 1984).  With X = I + (2/b) L and
  z = t b / 2,
      exp(t L) = sum_k c_k e^{-z} I_k(z) T_k(X),   c_0 = 1, c_k = 2,
  using exponentially scaled Bessel functions; the series is cut where the
  remaining coefficients sum below ``tol`` (T_k(X) has M-norm <= 1 because
  L is M-self-adjoint with spectrum in [-b, 0]).  This is the exact
  semi-discrete flow, used where the RK3 run would take days on the host.
"""

from __future__ import annotations

import numpy as np
from scipy.special import ive

from .bounds import schedule


def rk3(L, U0: np.ndarray, deltas, dt_nom: float, on_delta=None):
    """SSP-RK3 from U0 through the Delta list; returns [U(Delta_k)] (or the
    values of on_delta(k, U) when given)."""
    U = np.array(U0, dtype=np.float64, copy=True)
    out = []
    for k, (n, dt) in enumerate(schedule(deltas, dt_nom)):
        for _ in range(n):
            U1 = U + dt * (L @ U)
            U2 = 0.75 * U + 0.25 * (U1 + dt * (L @ U1))
            U = U / 3.0 + (2.0 / 3.0) * (U2 + dt * (L @ U2))
        out.append(on_delta(k, U) if on_delta else U.copy())
    return out


def cheb_coefficients(z: float, tol: float = 1e-17):
    """c_k e^{-z} I_k(z) until the tail is negligible."""
    kmax = int(12.0 * np.sqrt(z) + 60)
    while True:
        c = ive(np.arange(kmax + 1), z)
        if 2.0 * c[-1] < 1e-3 * tol:
            break
        kmax *= 2
    c[1:] *= 2.0
    tail = np.cumsum(c[::-1])[::-1]
    keep = np.flatnonzero(tail > tol)   # the c_k sum to exactly 1
    K = int(keep[-1]) + 1 if keep.size else 1
    return c[:max(K, 2)]


def expm_cheb(L, U: np.ndarray, t: float, b: float, tol: float = 1e-17) -> np.ndarray:
    """exp(t L) U for L with spectrum in [-b, 0]."""
    z = 0.5 * t * b
    c = cheb_coefficients(z, tol)
    alpha = 2.0 / b

    def X(V):
        return V + alpha * (L @ V)

    T0 = np.array(U, dtype=np.float64, copy=True)
    out = c[0] * T0
    T1 = X(T0)
    out += c[1] * T1
    for k in range(2, c.size):
        T2 = 2.0 * X(T1) - T0
        out += c[k] * T2
        T0, T1 = T1, T2
    return out


def expm_deltas(L, U0: np.ndarray, deltas, b: float, on_delta=None, tol: float = 1e-17):
    """Chebyshev exponential through the Delta list (one expansion per interval)."""
    U = np.array(U0, dtype=np.float64, copy=True)
    prev = 0.0
    out = []
    for k, d in enumerate(deltas):
        U = expm_cheb(L, U, float(d) - prev, b, tol)
        prev = float(d)
        out.append(on_delta(k, U) if on_delta else U.copy())
    return out

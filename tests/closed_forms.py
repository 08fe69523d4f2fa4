"""Closed-form reference results for the oracle pins (test helpers).

Free diffusion in the plane from a Gaussian of variance s0^2 keeps a
Gaussian of variance s0^2 + 2 D t in each axis (the paper's free-diffusion
check, section 4.2: Sigma = 2 T k I for a Dirac start).

Reflecting walls: on [0, w] with zero Neumann data the solution from a
Gaussian N(y0, s0^2) whose tails beyond the walls are negligible is the
method-of-images sum
    u(y, t) = sum_n [ phi(y - y0 - 2 n w) + phi(y + y0 - 2 n w) ],
phi the N(0, s0^2 + 2 D t) density (Carslaw and Jaeger).  Its moments over
[0, w] follow from truncated Gaussian integrals in closed form.  In a square
box the 2D solution is the product of two such 1D solutions.
"""

from __future__ import annotations

import math


def _trunc_moments(a, b, c, s, y0):
    """int_a^b (y - y0)^k phi(y - c; s^2) dy for k = 0, 1, 2."""
    A = (a - c) / s
    B = (b - c) / s
    pdf = lambda z: math.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)  # noqa: E731
    j0 = 0.5 * (math.erf(B / math.sqrt(2)) - math.erf(A / math.sqrt(2)))
    j1 = s * (pdf(A) - pdf(B))                        # int z phi, z in original units
    j2 = s * s * (j0 + A * pdf(A) - B * pdf(B))       # int z^2 phi
    e = c - y0                                        # y - y0 = z + e
    return (j0, j1 + e * j0, j2 + 2 * e * j1 + e * e * j0)


def neumann_1d_moments(w, y0, s0, D, t, n_images=40):
    """(m0, m1, m2) of the 1D Neumann solution about y0 at time t."""
    s = math.sqrt(s0 * s0 + 2.0 * D * t)
    m = [0.0, 0.0, 0.0]
    for n in range(-n_images, n_images + 1):
        for c in (y0 + 2 * n * w, -y0 + 2 * n * w):
            t3 = _trunc_moments(0.0, w, c, s, y0)
            for k in range(3):
                m[k] += t3[k]
    return tuple(m)


def box_moments(w, x0, s0, D, t):
    """Six moments (M0, mx, my, Mxx, Mxy, Myy) about x0 in the box [0, w]^2."""
    ax = neumann_1d_moments(w, x0[0], s0, D, t)
    ay = neumann_1d_moments(w, x0[1], s0, D, t)
    return (ax[0] * ay[0], ax[1] * ay[0], ax[0] * ay[1],
            ax[2] * ay[0], ax[1] * ay[1], ax[0] * ay[2])

"""Exact polynomial arithmetic and integration (oracle, test infrastructure).

A bivariate polynomial is a dict {(a, b): coefficient} meaning
sum c * x**a * y**b.  Coefficients may be Python floats or
``fractions.Fraction`` (the latter gives exact rational integrals for the
brute-force checks on tiny meshes).

Integrals over a triangle use the affine map from the unit triangle
{r, s >= 0, r + s <= 1} and the closed form
    integral of r**m * s**n over the unit triangle = m! n! / (m + n + 2)!.
Integrals along an edge reduce to integral_0^1 t**k dt = 1 / (k + 1).
These are the integrals of the weak form, eq. (7) of the paper.
"""

from __future__ import annotations

from fractions import Fraction
from math import comb, factorial


def padd(p, q, scale=1):
    out = dict(p)
    for k, v in q.items():
        out[k] = out.get(k, 0) + scale * v
    return out


def pmul(p, q):
    out = {}
    for (a, b), u in p.items():
        for (c, d), v in q.items():
            k = (a + c, b + d)
            out[k] = out.get(k, 0) + u * v
    return out


def pscale(p, s):
    return {k: v * s for k, v in p.items()}


def dx(p):
    return {(a - 1, b): a * v for (a, b), v in p.items() if a > 0}


def dy(p):
    return {(a, b - 1): b * v for (a, b), v in p.items() if b > 0}


def shift(p, sx, sy):
    """q(x, y) = p(x + sx, y + sy), expanded binomially."""
    out = {}
    for (a, b), v in p.items():
        for i in range(a + 1):
            for j in range(b + 1):
                c = v * comb(a, i) * comb(b, j) * (sx ** (a - i)) * (sy ** (b - j))
                out[(i, j)] = out.get((i, j), 0) + c
    return out


def _affine_pow(c0, c1, c2, n):
    """(c0 + c1 r + c2 s)**n as a polynomial in (r, s)."""
    base = {(0, 0): c0, (1, 0): c1, (0, 1): c2}
    out = {(0, 0): 1}
    for _ in range(n):
        out = pmul(out, base)
    return out


def _to_rs(p, v0, v1, v2):
    """Substitute x = v0 + r (v1 - v0) + s (v2 - v0)."""
    ex = (v1[0] - v0[0], v2[0] - v0[0])
    ey = (v1[1] - v0[1], v2[1] - v0[1])
    out = {}
    for (a, b), v in p.items():
        term = pmul(_affine_pow(v0[0], ex[0], ex[1], a), _affine_pow(v0[1], ey[0], ey[1], b))
        out = padd(out, term, v)
    return out, ex[0] * ey[1] - ex[1] * ey[0]


def integrate_triangle(p, v0, v1, v2, exact=False):
    """Integral of p over the triangle (v0, v1, v2)."""
    q, det = _to_rs(p, v0, v1, v2)
    total = 0
    for (m, n), v in q.items():
        if exact:
            w = Fraction(factorial(m) * factorial(n), factorial(m + n + 2))
        else:
            w = factorial(m) * factorial(n) / factorial(m + n + 2)
        total += v * w
    return total * abs(det)


def restrict_edge(p, p0, p1):
    """p(p0 + t (p1 - p0)) as a dict {k: coefficient of t**k}."""
    q, _ = _to_rs(p, p0, p1, p0)  # second direction unused (zero vector)
    out = {}
    for (m, n), v in q.items():
        if n == 0:
            out[m] = out.get(m, 0) + v
        elif v != 0:
            # the s-direction is the zero vector, so s-terms carry zero
            # coefficients; anything else is a bug
            raise AssertionError("non-zero s-term on an edge restriction")
    return out


def integrate_edge_param(p, p0, p1, exact=False):
    """Integral over t in [0, 1] of p(p0 + t (p1 - p0)) dt (no length factor)."""
    q = restrict_edge(p, p0, p1)
    total = 0
    for k, v in q.items():
        total += v * (Fraction(1, k + 1) if exact else 1.0 / (k + 1))
    return total

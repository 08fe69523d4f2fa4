"""Seeded disk packings and start points (inputs only, no method arithmetic).

The paper's substrate (section 2.2) is a square of side L holding
non-overlapping circles (axons) whose radii follow a Gamma law, clipped to
the square.  Its coordinates were never published, so these generators
produce seeded stand-ins:

* ``rsa_disks``: random sequential addition.  Radii are drawn i.i.d. from
  Gamma(shape k, scale mean/k) -- either a fixed count, or until the summed
  disk area reaches phi * L**2 -- and placed largest first.  Each disk gets at
  most ``max_tries`` uniform centre proposals in [0, L]^2 and is accepted at
  the first proposal whose gap to every placed disk is at least ``gap``;
  a disk that finds no place is dropped, and after ``max_fail_run``
  consecutive dropped disks the packing counts as jammed and placement
  stops.  Disks may cross the box edge.
* ``start_points``: points uniform over the extracellular part of the
  centred box of side ``box_frac*L`` (section 4.1 draws the pulses uniformly
  in the extracellular space; section 4.2 keeps them in a centred 20 um box
  of a 50 um square).  On the pixel grid the extracellular space is the set
  of cells whose centroid lies outside every disk, so a uniform proposal in
  the box is kept iff the cell holding it is such a cell: the accepted
  points are uniform over the kept cells' area, right up to the staircase
  walls.  ``law="pore_interior"`` keeps the earlier, narrower law (points at
  least r + sqrt(2) h from every disk centre) for comparison.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Geometry:
    """A square box [0, L]^2 on an N x N cell grid with a list of disks."""

    L: float
    N: int
    disks: np.ndarray          # float64 [n, 3] = (cx, cy, r) in um
    params: dict               # how it was drawn (for reports)

    @property
    def h(self) -> float:
        return self.L / self.N


def _draw_radii(rng, L, phi, n_disks, shape, mean):
    scale = mean / shape
    if n_disks is not None:
        radii = rng.gamma(shape, scale, size=int(n_disks))
    else:
        target = phi * L * L
        chunks = []
        total = 0.0
        while total < target:
            c = rng.gamma(shape, scale, size=1024)
            area = np.cumsum(np.pi * c * c) + total
            k = int(np.searchsorted(area, target)) + 1
            if k <= c.size:
                chunks.append(c[:k])
                total = float(area[k - 1])
                break
            chunks.append(c)
            total = float(area[-1])
        radii = np.concatenate(chunks) if chunks else np.zeros(0)
    return np.sort(radii)[::-1].copy()


def rsa_disks(L: float, rng: np.random.Generator, *, phi: float | None = None,
              n_disks: int | None = None, shape: float = 4.0, mean: float = 0.5,
              gap: float = 0.1, max_tries: int = 20000, batch: int = 256,
              max_fail_run: int = 64) -> np.ndarray:
    """Random sequential addition of Gamma-radius disks in [0, L]^2.

    Exactly one of ``phi`` (target summed disk area / L^2) and ``n_disks``
    must be given.  Returns float64 [n_placed, 3] = (cx, cy, r).
    """
    if (phi is None) == (n_disks is None):
        raise ValueError("give exactly one of phi and n_disks")
    radii = _draw_radii(rng, L, phi, n_disks, shape, mean)
    if radii.size == 0:
        return np.zeros((0, 3))
    # Exclusion lookup on a fine grid: disk j is registered in every cell its
    # zone of radius 2 r_j + gap touches.  Radii are placed in decreasing
    # order, so a later disk of radius r <= r_j clashes with j only at
    # proposal points inside that zone: one cell lookup finds every clash.
    cell = max(0.25, float(np.mean(radii)))
    ng = max(1, int(math.ceil(L / cell)))
    cap = 16
    grid = -np.ones((ng, ng, cap), dtype=np.int64)
    count = np.zeros((ng, ng), dtype=np.int64)
    placed = np.zeros((radii.size, 3))
    n = 0
    fail_run = 0
    for r in radii:
        if fail_run >= max_fail_run:
            break
        tries = 0
        done = False
        while tries < max_tries and not done:
            k = min(batch, max_tries - tries)
            prop = rng.uniform(0.0, L, size=(k, 2))
            tries += k
            gx = np.minimum((prop[:, 0] / cell).astype(np.int64), ng - 1)
            gy = np.minimum((prop[:, 1] / cell).astype(np.int64), ng - 1)
            cand = grid[gx, gy]                      # [k, cap]
            valid = cand >= 0
            ok = np.ones(k, dtype=bool)
            if valid.any():
                ci = np.where(valid, cand, 0)
                dx = placed[ci, 0] - prop[:, 0, None]
                dy = placed[ci, 1] - prop[:, 1, None]
                need = placed[ci, 2] + r + gap
                ok = ~(valid & (dx * dx + dy * dy < need * need)).any(axis=1)
            idx = np.flatnonzero(ok)
            if idx.size:
                j = int(idx[0])
                x, y = float(prop[j, 0]), float(prop[j, 1])
                placed[n] = (x, y, r)
                zr = 2.0 * r + gap
                i0, i1 = max(0, int((x - zr) / cell)), min(ng - 1, int((x + zr) / cell))
                j0, j1 = max(0, int((y - zr) / cell)), min(ng - 1, int((y + zr) / cell))
                ii, jj = np.meshgrid(np.arange(i0, i1 + 1), np.arange(j0, j1 + 1), indexing="ij")
                # distance from the centre to each cell rectangle
                ddx = np.maximum(np.maximum(ii * cell - x, x - (ii + 1) * cell), 0.0)
                ddy = np.maximum(np.maximum(jj * cell - y, y - (jj + 1) * cell), 0.0)
                hit = ddx * ddx + ddy * ddy < zr * zr
                ii, jj = ii[hit], jj[hit]
                if ii.size and count[ii, jj].max() >= cap:
                    grid = np.concatenate([grid, -np.ones_like(grid)], axis=2)
                    cap *= 2
                grid[ii, jj, count[ii, jj]] = n
                count[ii, jj] += 1
                n += 1
                done = True
        fail_run = 0 if done else fail_run + 1
    return placed[:n].copy()


def coverage_fraction(disks: np.ndarray, L: float, samples: int = 1024) -> float:
    """Area fraction of [0, L]^2 covered by the (clipped) disks, estimated on a
    samples x samples midpoint raster.  Reporting only."""
    t = (np.arange(samples) + 0.5) * (L / samples)
    covered = np.zeros((samples, samples), dtype=bool)
    for cx, cy, r in disks:
        i0 = max(0, int((cx - r) / L * samples) - 1)
        i1 = min(samples, int((cx + r) / L * samples) + 2)
        j0 = max(0, int((cy - r) / L * samples) - 1)
        j1 = min(samples, int((cy + r) / L * samples) + 2)
        if i0 >= i1 or j0 >= j1:
            continue
        xx = t[i0:i1, None] - cx
        yy = t[None, j0:j1] - cy
        covered[i0:i1, j0:j1] |= xx * xx + yy * yy < r * r
    return float(covered.mean())


def _cell_kept(p: np.ndarray, disks: np.ndarray, L: float, N: int) -> np.ndarray:
    """Whether the grid cell holding each point [k, 2] has its centroid
    outside every disk (strict test, as the mesh builders read it; a point on
    the far box edge belongs to the last cell)."""
    h = L / N
    ij = np.minimum(np.floor(p / h).astype(np.int64), N - 1)
    c = (ij + 0.5) * h
    if disks.shape[0] == 0:
        return np.ones(p.shape[0], dtype=bool)
    dx = c[:, 0, None] - disks[None, :, 0]
    dy = c[:, 1, None] - disks[None, :, 1]
    r = disks[None, :, 2]
    return ~(dx * dx + dy * dy < r * r).any(axis=1)


def start_points(disks: np.ndarray, L: float, N: int, m: int,
                 rng: np.random.Generator, box_frac: float = 0.4,
                 center: tuple | None = None, law: str = "extracellular") -> np.ndarray:
    """m start points in the centred box of side box_frac*L, float64 [m, 2].

    law = "extracellular" (default): uniform over the box area covered by
    cells whose centroid is outside every disk (section 4.1).
    law = "pore_interior": uniform in the box, each at least r + sqrt(2)*h
    from every disk centre (a narrower law, kept for comparison)."""
    if law not in ("extracellular", "pore_interior"):
        raise ValueError("law must be 'extracellular' or 'pore_interior'")
    h = L / N
    cx0, cy0 = (0.5 * L, 0.5 * L) if center is None else center
    half = 0.5 * box_frac * L
    margin = math.sqrt(2.0) * h
    out = np.zeros((m, 2))
    n = 0
    guard = 0
    while n < m:
        guard += 1
        if guard > 100000:
            raise RuntimeError("could not place start points")
        p = rng.uniform(-half, half, size=(256, 2)) + np.array([cx0, cy0])
        if law == "extracellular":
            ok = _cell_kept(p, disks, L, N)
        elif disks.shape[0]:
            dx = p[:, 0, None] - disks[None, :, 0]
            dy = p[:, 1, None] - disks[None, :, 1]
            lim = disks[None, :, 2] + margin
            ok = ~(dx * dx + dy * dy < lim * lim).any(axis=1)
        else:
            ok = np.ones(p.shape[0], dtype=bool)
        good = p[ok]
        take = min(m - n, good.shape[0])
        out[n:n + take] = good[:take]
        n += take
    return out


def make_geometry(L: float, N: int, seed: int, *, phi=None, n_disks=None,
                  shape=4.0, mean=0.5, gap=0.1, batch=256) -> Geometry:
    """Seeded disk packing on an N x N grid over [0, L]^2."""
    rng = np.random.default_rng(seed)
    if phi is None and n_disks is None:
        disks = np.zeros((0, 3))
    else:
        disks = rsa_disks(L, rng, phi=phi, n_disks=n_disks, shape=shape,
                          mean=mean, gap=gap, batch=batch)
    params = dict(L=L, N=N, seed=seed, phi_target=phi, n_disks_target=n_disks,
                  gamma_shape=shape, gamma_mean=mean, gap=gap,
                  n_disks=int(disks.shape[0]))
    return Geometry(L=float(L), N=int(N), disks=disks, params=params)

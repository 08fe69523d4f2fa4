"""The seeded start-point law (section 4.1: pulses placed uniformly in the
extracellular space, here the centred box of side 0.4 L).

On the pixel grid the extracellular space is the union of the cells whose
centroid lies outside every disk.  These checks use their own cell test
(plain loops over the disks), not the generator's.
"""

import math

import numpy as np

from workloads import make_geometry, start_points


def _kept_cells(g):
    """Boolean [N, N] (indexed [i, j]) of cells with centroid outside every disk."""
    h = g.L / g.N
    c = (np.arange(g.N) + 0.5) * h
    X, Y = np.meshgrid(c, c, indexing="ij")
    kept = np.ones((g.N, g.N), dtype=bool)
    for cx, cy, r in g.disks:
        kept &= ~((X - cx) ** 2 + (Y - cy) ** 2 < r * r)
    return kept


def _geometry():
    return make_geometry(20.0, 100, 19070619 + 77, phi=0.6, shape=4.0, mean=0.5)


def test_points_lie_in_kept_cells_of_the_centred_box():
    g = _geometry()
    kept = _kept_cells(g)
    pts = start_points(g.disks, g.L, g.N, 400, np.random.default_rng(5))
    h = g.L / g.N
    assert np.all(np.abs(pts - 0.5 * g.L) <= 0.2 * g.L)
    ij = np.floor(pts / h).astype(int)
    assert kept[ij[:, 0], ij[:, 1]].all()


def test_points_are_uniform_over_kept_area_including_wall_cells():
    """The share of points in kept cells that touch a removed cell (4-
    neighbour) matches that share of the kept area in the box, within five
    binomial standard deviations; the earlier pore-interior law puts far
    fewer points there."""
    g = _geometry()
    kept = _kept_cells(g)
    N = g.N
    wall = np.zeros_like(kept)
    for di, dj in [(1, 0), (-1, 0), (0, 1), (0, -1)]:
        sh = np.ones_like(kept)
        src = kept[max(0, di):N + min(0, di), max(0, dj):N + min(0, dj)]
        sh[max(0, -di):N + min(0, -di), max(0, -dj):N + min(0, -dj)] = src
        wall |= ~sh
    wall &= kept
    h = g.L / N
    lo, hi = int(math.floor(0.3 * g.L / h)), int(math.ceil(0.7 * g.L / h))
    # expected share over the box: cells fully inside [0.3 L, 0.7 L] (the
    # box edges fall on cell boundaries here: 0.3 * 100 = 30)
    box_kept = kept[lo:hi, lo:hi]
    share = wall[lo:hi, lo:hi].sum() / box_kept.sum()
    n = 4000
    pts = start_points(g.disks, g.L, N, n, np.random.default_rng(11))
    ij = np.floor(pts / h).astype(int)
    got = wall[ij[:, 0], ij[:, 1]].mean()
    sd = math.sqrt(share * (1 - share) / n)
    assert abs(got - share) < 5 * sd, (got, share)
    old = start_points(g.disks, g.L, N, n, np.random.default_rng(11), law="pore_interior")
    ij = np.floor(old / h).astype(int)
    assert wall[ij[:, 0], ij[:, 1]].mean() < 0.5 * share
    d = np.sqrt(((old[:, None, :] - g.disks[None, :, :2]) ** 2).sum(-1))
    assert (d >= g.disks[None, :, 2] + math.sqrt(2.0) * h).all()

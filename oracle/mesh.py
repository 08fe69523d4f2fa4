"""Pixel-triangle mesh of the extracellular region (oracle, test infrastructure).

Section 3.3 of the paper splits each square pixel by a diagonal into two
triangles.  Readings taken where the paper is silent (its meshing figure is
missing):

* the diagonal runs from the cell's lower-left to its upper-right corner;
  triangle T0 of cell (i, j) is {(i,j), (i+1,j), (i+1,j+1)} * h (lower right)
  and T1 is {(i,j), (i+1,j+1), (i,j+1)} * h (upper left);
* a cell is removed iff its centroid lies strictly inside a disk
  (|c - c_d|^2 < r_d^2, FP64, centroid ((i+1/2) h, (j+1/2) h)); both of its
  triangles go with it.  Removing the axon cells is the zero-flux reading of
  eq. (3) with k = 0 in the axons (eq. (5));
* a face is interior iff the triangles on both sides are active.  Faces on a
  removed cell or on the box edge carry no flux (zero Neumann data, eq. (3);
  the box uses zero flux too).

Elements are numbered 2 * rank(cell) + o, o = 0 for T0 and 1 for T1, with
active cells ranked in row-major order (j slow, i fast).
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


# Local faces, per orientation: (name, neighbour cell offset).  The
# neighbour is always the other orientation.
#   T0: f0 bottom edge -> T1 of cell (i, j-1); f1 right edge -> T1 of (i+1, j);
#       f2 diagonal -> T1 of the same cell.
#   T1: f0 top edge -> T0 of cell (i, j+1); f1 left edge -> T0 of (i-1, j);
#       f2 diagonal -> T0 of the same cell.
FACE_OFFSETS = {0: [(0, -1), (1, 0), (0, 0)], 1: [(0, 1), (-1, 0), (0, 0)]}


@dataclasses.dataclass
class Mesh:
    L: float
    N: int
    h: float
    active_cell: np.ndarray      # bool [N, N] indexed [i, j]
    cell_i: np.ndarray           # int64 [E] cell index of element e
    cell_j: np.ndarray
    orient: np.ndarray           # int8 [E]
    nbr: np.ndarray              # int64 [E, 3], -1 where the face has no flux

    @property
    def n_elements(self) -> int:
        return int(self.orient.size)

    def n_components(self) -> int:
        """Connected components of the element graph joined by interior faces."""
        E = self.n_elements
        rows, cols = [], []
        for f in range(3):
            m = self.nbr[:, f] >= 0
            rows.append(np.flatnonzero(m))
            cols.append(self.nbr[m, f])
        r = np.concatenate(rows)
        c = np.concatenate(cols)
        g = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(E, E)).tocsr()
        n, _ = connected_components(g, directed=False)
        return int(n)

    def n_interior_faces(self) -> int:
        return int((self.nbr >= 0).sum() // 2)

    def removed_fraction(self) -> float:
        return 1.0 - float(self.active_cell.mean())


def build_mesh(L: float, N: int, disks: np.ndarray) -> Mesh:
    """Mesh of [0, L]^2 on an N x N grid with the disk cells removed."""
    h = L / N
    centers = (np.arange(N) + 0.5) * h
    active = np.ones((N, N), dtype=bool)
    X = centers[:, None]
    Y = centers[None, :]
    for cx, cy, r in np.asarray(disks, dtype=np.float64).reshape(-1, 3):
        active &= ~((X - cx) ** 2 + (Y - cy) ** 2 < r * r)
    # rank active cells in row-major order: j slow, i fast
    jj, ii = np.nonzero(active.T)
    rank = -np.ones((N, N), dtype=np.int64)
    rank[ii, jj] = np.arange(ii.size)
    E = 2 * ii.size
    cell_i = np.repeat(ii, 2)
    cell_j = np.repeat(jj, 2)
    orient = np.tile(np.array([0, 1], dtype=np.int8), ii.size)
    nbr = -np.ones((E, 3), dtype=np.int64)
    for o in (0, 1):
        sel = np.flatnonzero(orient == o)
        ci, cj = cell_i[sel], cell_j[sel]
        for f, (oi, oj) in enumerate(FACE_OFFSETS[o]):
            ni, nj = ci + oi, cj + oj
            inside = (ni >= 0) & (ni < N) & (nj >= 0) & (nj < N)
            r = -np.ones(sel.size, dtype=np.int64)
            r[inside] = rank[ni[inside], nj[inside]]
            ok = r >= 0
            nbr[sel[ok], f] = 2 * r[ok] + (1 - o)
    return Mesh(L=float(L), N=int(N), h=h, active_cell=active, cell_i=cell_i,
                cell_j=cell_j, orient=orient, nbr=nbr)

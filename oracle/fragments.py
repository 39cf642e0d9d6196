"""Fragment delineation -- oracle.

Fragments are the connected sets of material cells (Section 4.2/4.3 delineate
fragments at the 0.5 void-fraction contour; with a surrounding gas the
material cell test is on the solid's own volume fraction, phi_s > cut).
Connectivity is through cell faces (4 neighbours in 2D, 6 in 3D; the paper
does not state it).  Each fragment is labelled with the smallest linear cell
index it contains (x fastest), its mass is the correctly rounded sum of
phi_s rho_s over its cells times the cell volume, and it is flagged when it
touches the domain boundary.  A breadth-first flood fill written out in
plain Python: slow, for small grids.
"""
import math
from collections import deque

import numpy as np


def label(solid_phi, cut=0.5):
    """Labels (nz, ny, nx) int64, -1 for non-material cells."""
    nz, ny, nx = solid_phi.shape
    mat = solid_phi > cut
    lab = np.full(mat.shape, -1, dtype=np.int64)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if not mat[z, y, x] or lab[z, y, x] >= 0:
                    continue
                root = (z * ny + y) * nx + x
                lab[z, y, x] = root
                dq = deque([(z, y, x)])
                while dq:
                    cz, cy, cx = dq.popleft()
                    for dz, dy, dx in ((1, 0, 0), (-1, 0, 0), (0, 1, 0),
                                       (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                        qz, qy, qx = cz + dz, cy + dy, cx + dx
                        if (0 <= qz < nz and 0 <= qy < ny and 0 <= qx < nx
                                and mat[qz, qy, qx] and lab[qz, qy, qx] < 0):
                            lab[qz, qy, qx] = root
                            dq.append((qz, qy, qx))
    # breadth-first from the first cell in scan order yields the minimum
    # linear index of the component as its root
    return lab


def fragments(solid_phi, solid_mass, cell_volume, cut=0.5):
    """List of (label, n_cells, mass, touches_boundary) sorted by label."""
    lab = label(solid_phi, cut)
    nz, ny, nx = lab.shape
    out = []
    for root in np.unique(lab[lab >= 0]):
        cells = lab == root
        vals = solid_mass[cells].ravel().tolist()
        zz, yy, xx = np.nonzero(cells)
        touch = bool(
            (nx > 1 and (xx.min() == 0 or xx.max() == nx - 1))
            or (ny > 1 and (yy.min() == 0 or yy.max() == ny - 1))
            or (nz > 1 and (zz.min() == 0 or zz.max() == nz - 1)))
        out.append((int(root), int(cells.sum()),
                    math.fsum(vals) * cell_volume, touch))
    return out


def mass_histogram(frags, edges):
    """Cumulative fragment count against fragment mass, the form in which
    Sections 4.2 and 4.3 present fragment distributions (fragment mass
    against cumulative fragment number): entry k is the number of fragments
    whose mass is at least edges[k]."""
    masses = [f[2] for f in frags]
    return [sum(1 for m in masses if m >= e) for e in edges]

"""Conservation totals -- oracle.

Each total is the correctly rounded sum (math.fsum) of the cell values of a
conserved field, times the cell volume: the exact value of the sum rounded
once, then one IEEE multiplication.  Boundary outflows are summed the same
way per boundary side and multiplied by that side's face area.  The totals
cover the conservation-form equations of Section 2.1 (phasic mass, momentum,
total energy).
"""
import math


def total_rows(layout):
    return layout.mass + layout.mom + [layout.energy]


def interior_totals(U, layout, cell_volume):
    return [math.fsum(U[r].ravel().tolist()) * cell_volume
            for r in total_rows(layout)]


def flux_total_rows(layout):
    """Positions of the totals' variables in the conserved-flux vector."""
    L = layout
    nh = 2 * len(L.solids)
    return (list(range(L.nm))
            + [L.nm + nh + k for k in range(L.dim)] + [L.nm + nh + L.dim])


def boundary_totals(bacc, layout, face_areas):
    """bacc[(k, side)]: accumulated outward flux per boundary face, shaped
    (n_flux, ...).  Returns the outflow per totals variable."""
    rows = flux_total_rows(layout)
    out = []
    for r in rows:
        parts = []
        for (k, side), arr in sorted(bacc.items()):
            parts.append(math.fsum(arr[r].ravel().tolist()) * face_areas[k])
        out.append(math.fsum(parts))
    return out

"""Field order of the conserved state.

Follows the order of the evolution equations of Section 2.1: volume
fractions, phasic masses, phasic history densities (equivalent plastic strain
and damage of each solid), momentum, total energy, the stored components of
the unimodular stretch, and the Lagrangian coordinates of Section 2.4
(perturbation field).  The void fraction is not stored: it is 1 minus the sum
of the material volume fractions.
"""


def vbar_comps(dim):
    if dim == 1:
        return [(0, 0), (1, 1), (2, 2)]
    if dim == 2:
        return [(0, 0), (0, 1), (1, 0), (1, 1), (2, 2)]
    return [(i, j) for i in range(3) for j in range(3)]


def hencky_comps(dim):
    """Independent components of the symmetric Hencky strain that can be
    non-zero in each dimension."""
    if dim == 1:
        return [(0, 0), (1, 1), (2, 2)]
    if dim == 2:
        return [(0, 0), (0, 1), (1, 1), (2, 2)]
    return [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


class Layout:
    def __init__(self, dim, mats):
        self.dim = dim
        self.mats = mats
        self.nm = len(mats)
        self.solids = [l for l, m in enumerate(mats) if m["kind"] == "solid"]
        k = 0
        self.phi = list(range(k, k + self.nm)); k += self.nm
        self.mass = list(range(k, k + self.nm)); k += self.nm
        self.eps = {}
        self.dmg = {}
        for l in self.solids:
            self.eps[l] = k
            self.dmg[l] = k + 1
            k += 2
        self.mom = list(range(k, k + dim)); k += dim
        self.energy = k; k += 1
        self.vcomps = vbar_comps(dim)
        self.vbar = list(range(k, k + len(self.vcomps))); k += len(self.vcomps)
        self.X = list(range(k, k + dim)); k += dim
        self.S = k
        # conserved-flux vector: masses, histories, momenta, energy
        self.flux_rows = (self.mass
                          + [r for l in self.solids
                             for r in (self.eps[l], self.dmg[l])]
                          + self.mom + [self.energy])

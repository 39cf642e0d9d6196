"""Pins of the oracle's conservation totals and fragment labelling (CPU):
exact summation against cancellation-heavy data, labels against
scipy.ndimage.label with face connectivity, and the workload constants that
come from the paper's material tables (tests/golden/paper_tables.json)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.ndimage

import fvinputs as F
from oracle import fragments as Fr
from oracle.layout import Layout
from oracle.totals import interior_totals

HERE = os.path.dirname(os.path.abspath(__file__))


def test_totals_are_correctly_rounded():
    L = Layout(1, [F.COPPER])
    U = np.zeros((L.S, 1, 1, 6))
    U[L.mass[0], 0, 0] = [1e16, 1.0, -1e16, 3.0, 1e-3, -1e-3]
    tot = interior_totals(U, L, 0.5)
    assert tot[0] == 2.0            # naive left-to-right summation gives 0
    rng = np.random.default_rng(5)
    vals = rng.standard_normal(1000) * 10.0 ** rng.integers(-8, 8, 1000)
    U2 = np.zeros((L.S, 1, 1, 1000))
    U2[L.energy, 0, 0] = vals
    from fractions import Fraction
    exact = sum(Fraction(float(v)) for v in vals)
    assert interior_totals(U2, L, 1.0)[-1] == float(exact)


@pytest.mark.parametrize("shape", [(1, 23, 31), (7, 9, 11)])
def test_labels_match_scipy(shape):
    rng = np.random.default_rng(11)
    phi = scipy.ndimage.gaussian_filter(rng.random(shape), 1.0)
    phi = (phi - phi.min()) / (phi.max() - phi.min())
    lab = Fr.label(phi, 0.5)
    ref, n = scipy.ndimage.label(phi > 0.5)
    assert len(np.unique(lab[lab >= 0])) == n
    for k in range(1, n + 1):
        cells = ref == k
        vals = np.unique(lab[cells])
        assert len(vals) == 1
        # canonical label: smallest linear index of the component
        assert vals[0] == np.flatnonzero(cells.ravel()).min()
    assert np.all((lab >= 0) == (phi > 0.5))


def test_fragment_masses_and_boundary_flags():
    phi = np.zeros((1, 6, 8))
    phi[0, 1:3, 1:3] = 1.0        # interior block
    phi[0, 4:6, 5:8] = 0.8        # touches the boundary
    mass = phi * 8930.0
    frags = Fr.fragments(phi, mass, 2.0, 0.5)
    assert len(frags) == 2
    (l0, n0, m0, t0), (l1, n1, m1, t1) = frags
    assert (l0, n0, t0) == (1 * 8 + 1, 4, False)
    assert (l1, n1, t1) == (4 * 8 + 5, 6, True)
    assert m0 == math.fsum([8930.0] * 4) * 2.0
    assert m1 == math.fsum([0.8 * 8930.0] * 6) * 2.0


def test_mass_histogram_counts_fragments_at_or_above_each_edge():
    """Cumulative count against mass (Sections 4.2, 4.3), on a list whose
    counts follow by inspection: ties count at their own edge."""
    frags = [(0, 1, 1.0, False), (5, 2, 2.0, True), (9, 2, 2.0, False),
             (12, 5, 5.0, False)]
    edges = [0.5, 1.0, 2.0, math.nextafter(2.0, 3.0), 5.0, 6.0]
    assert Fr.mass_histogram(frags, edges) == [4, 4, 3, 1, 1, 0]
    assert Fr.mass_histogram([], edges) == [0] * len(edges)
    # the first edge at or below the lightest fragment counts them all, and
    # the count never rises with the edge
    rng = np.random.default_rng(3)
    frags = [(i, 1, float(m), False) for i, m in enumerate(rng.lognormal(0, 2, 50))]
    edges = sorted(rng.lognormal(0, 2, 20).tolist())
    h = Fr.mass_histogram(frags, [0.0] + edges)
    assert h[0] == 50 and all(a >= b for a, b in zip(h, h[1:]))


def test_workload_constants_from_paper_tables():
    g = json.load(open(os.path.join(HERE, "golden", "paper_tables.json")))
    cu = F.COPPER
    assert cu["alpha"] == g["romenskii_cube"]["alpha"]
    assert cu["beta"] == g["romenskii_cube"]["beta"]
    assert cu["Gamma0"] == g["romenskii_cube"]["Gamma0"]
    assert cu["n_hard"] == g["johnson_cook_cube"]["n"]
    assert cu["eps_th"] == g["bonora_cube"]["eps_thresh"]
    assert cu["eps_c"] == g["bonora_cube"]["eps_crit"]
    assert cu["bonora_alpha"] == g["bonora_cube"]["alpha"]

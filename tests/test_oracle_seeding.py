"""Pins of the oracle's Lagrangian seeding into void (Section 3.2.1
seeding routine) and of the expanding-disk workload's constants (CPU only).

The routine extrapolates X into a void cell c from the point p it probes on
the material side: X_new = X(p) - (p - c).  For coordinates linear in space
(a body in rigid translation, X = x - d) this is exact whatever the normal,
the probe distance or the interpolation weights, so a linear field must come
back unchanged; a slip in the sign or the offset of the extrapolation moves
it by a multiple of the probe distance."""
import json
import os

import numpy as np
import pytest

import fvinputs as F
from oracle.layout import Layout
from oracle.mixture import Options, prim_to_cons
from oracle.scheme import Geometry
from oracle.seeding import seed_void

HERE = os.path.dirname(os.path.abspath(__file__))


def _body_case(n=24, shift=(-3.0e-4, 2.0e-4)):
    """A square block of steel in void on an n x n grid of 1 mm cells, with
    Lagrangian coordinates X = x - shift in every cell."""
    c = F.uniform_case(2, (n, n, 1), [F.STEEL_304L], [1.0], [8000.0], [0.0, 0.0],
                       0.0, bc="transmissive", lo=(0.0, 0.0, 0.0),
                       hi=(n * 1e-3, n * 1e-3, 1.0))
    L = Layout(2, c.mats)
    y, x = np.indices((n, n))
    body = (x >= 8) & (x < 16) & (y >= 6) & (y < 18)
    c.prim[L.phi[0]][0] = np.where(body, 1.0, 0.0)
    for k in range(2):
        c.prim[L.X[k]][0] -= shift[k]
    return c, L, body


def _seed(c, L, thresh=0.99):
    opts = Options(cfl=c.cfl)
    U = prim_to_cons(c.prim.copy(), L, opts)
    geom = Geometry(c.dim, c.n, c.lo, c.hi, c.bc)
    X0 = U[L.X].copy()
    U1 = seed_void(U.copy(), geom, L, thresh)
    return X0, U1[L.X]


def test_linear_coordinates_are_reproduced():
    c, L, body = _body_case()
    X0, X1 = _seed(c, L)
    assert np.max(np.abs(X1 - X0)) <= 1e-15 * 0.03


def test_first_void_layer_takes_the_body_coordinates():
    """Void cells next to the block's straight sides get X = x - d from the
    block alone (their probe lands 1.5 cells inside it), whatever their own
    coordinates held; void cells away from any material keep theirs."""
    c, L, body = _body_case()
    rng = np.random.default_rng(3)
    n = c.n[0]
    X_true = [c.prim[L.X[k]][0].copy() for k in range(2)]
    for k in range(2):
        junk = X_true[k] + 1e-3 * rng.standard_normal((n, n))
        c.prim[L.X[k]][0] = np.where(body, X_true[k], junk)
    X0, X1 = _seed(c, L)
    y, x = np.indices((n, n))
    side = (((x == 7) | (x == 16)) & (y >= 7) & (y < 17)) | \
           (((y == 5) | (y == 18)) & (x >= 9) & (x < 15))
    for k in range(2):
        assert np.max(np.abs(X1[k][0][side] - X_true[k][side])) < 1e-15 * 0.03
    far = (np.abs(x - 11.5) > 9) | (np.abs(y - 11.5) > 10)
    for k in range(2):
        assert np.array_equal(X1[k][0][far], X0[k][0][far])
    # material cells are never reseeded
    for k in range(2):
        assert np.array_equal(X1[k][0][body], X0[k][0][body])


def test_threshold_spares_partially_filled_cells():
    c, L, body = _body_case()
    n = c.n[0]
    y, x = np.indices((n, n))
    half = (x == 16) & (y >= 6) & (y < 18)            # a half-filled column
    c.prim[L.phi[0]][0] = np.where(half, 0.5, c.prim[L.phi[0]][0])
    c.prim[L.X[0]][0] = np.where(half, 123.0, c.prim[L.X[0]][0])
    X0, X1 = _seed(c, L)
    assert np.all(X1[0][0][half] == 123.0)


def test_disk_constants_from_paper_tables():
    g = json.load(open(os.path.join(HERE, "golden", "paper_tables.json")))
    s = F.STEEL_304L
    r, jc, b = g["romenskii_304l"], g["johnson_cook_304l"], g["bonora_304l_disk"]
    assert s["rho0"] == r["rho0"] and s["K0"] == r["K0_GPa"] * 1e9
    assert s["G0"] == r["G0_GPa"] * 1e9
    assert (s["alpha"], s["beta"], s["Gamma0"]) == (r["alpha"], r["beta"], r["Gamma0"])
    assert s["yield_stress"] == pytest.approx(jc["c1_GPa"] * 1e9, rel=1e-15)
    assert s["n_hard"] == jc["n"]
    assert (s["D_crit"], s["eps_th"], s["eps_c"], s["bonora_alpha"]) == (
        b["D_crit"], b["eps_thresh"], b["eps_crit"], b["alpha"])
    c = F.expanding_disk(64)
    assert c.seed_nu == 0.99 and c.cfl == 0.4 and c.t_end == 200e-6
    L = Layout(2, c.mats)
    # the initial radial velocity 2000 r inside the disk
    xc = c.prim[L.X[0]][0]
    solid = c.prim[L.phi[0]][0] == 1.0
    assert np.allclose(c.prim[L.mom[0]][0][solid], 2000.0 * xc[solid], rtol=1e-12)


@pytest.mark.slow
def test_disk_with_seeding_stays_physical():
    """The disk at 48^2 through critical damage (about 400 steps): no
    negative mass, finite state, seeded coordinates next to the expanding
    edge within a cell of the material's."""
    from oracle import Solver
    c = F.expanding_disk(48)
    s = Solver(c)
    for _ in range(300):
        s.step()
    L = s.layout
    assert np.isfinite(s.U).all()
    assert np.min(s.U[L.mass[0]]) > 0
    D = s.U[L.dmg[0]] / s.U[L.mass[0]]
    assert np.max(D) >= 0.3 * (1 - 1e-9)


def _film_state(phi, rho_l, u, e, n=6):
    """A 1D row of one-solid cells (steel, volume fraction phi at phasic
    density rho_l, velocity u, undistorted, undamaged) with the specific
    internal energy set to e directly in the conserved state."""
    c = F.uniform_case(1, (n, 1, 1), [F.STEEL_304L], [phi], [rho_l], [u], 0.0,
                       bc="transmissive")
    L = Layout(1, c.mats)
    U = prim_to_cons(c.prim.copy(), L, Options(cfl=c.cfl))
    m = U[L.mass[0]]
    U[L.energy] = m * e + 0.5 * m * u * u
    geom = Geometry(c.dim, c.n, c.lo, c.hi, c.bc)
    return U, L, geom


def test_relaxed_cold_film_takes_the_reference_density():
    """Special case of the void relaxation: with no internal energy, no
    distortion and no damage the steel's pressure vanishes at its reference
    density rho0 (the cold curve's zero, where the film is unloaded), so a
    void cell's volume fraction becomes mass / rho0, from either side of
    rho0; mass, momentum and energy are untouched."""
    from oracle.seeding import relax_void
    rho0 = F.STEEL_304L["rho0"]
    for rho_l in (0.6 * rho0, 1.7 * rho0):
        U, L, geom = _film_state(0.004, rho_l, 120.0, 0.0)
        out = relax_void(U, geom, L, 0.99, 1e-8)
        m = U[L.mass[0]]
        assert np.allclose(out[L.phi[0]] * rho0 / m, 1.0, rtol=1e-13, atol=0)
        keep = [r for r in range(L.S) if r != L.phi[0]]
        assert np.array_equal(out[keep], U[keep])


def test_relaxed_film_has_zero_pressure_at_its_own_energy():
    """The film density solves p_l(rho, e) = 0 for the cell's specific
    internal energy: take e from the energy of the steel at zero pressure at
    a chosen density rho* < rho0 (the inverse equation of state), relax, and
    the film density mass / phi returns rho* (the bisection's rounding).
    Above rho0 the cold pressure alone is positive, so an energy below the
    cold curve (the zero-temperature bound the pressure inversion floors
    the thermal energy at) leaves the film at rho0."""
    from oracle.seeding import relax_void
    from oracle.mixture import energy_from_pressure, material_terms
    rho0 = F.STEEL_304L["rho0"]
    for rs in (0.93 * rho0, 0.985 * rho0):
        one = np.ones((1, 1))
        terms = material_terms(np.full((1, 1), rs), np.zeros((1, 1)), np.zeros(1),
                               [F.STEEL_304L], one)
        e = float(energy_from_pressure(one, terms, np.zeros(1), [F.STEEL_304L])[0]) / rs
        U, L, geom = _film_state(0.003, 0.8 * rho0, -40.0, e)
        out = relax_void(U, geom, L, 0.99, 1e-8)
        film = U[L.mass[0]] / out[L.phi[0]]
        assert np.allclose(film, rs, rtol=1e-12, atol=0)
    U, L, geom = _film_state(0.003, 1.2 * rho0, 5.0, -3.0e5)
    out = relax_void(U, geom, L, 0.99, 1e-8)
    assert np.allclose(U[L.mass[0]] / out[L.phi[0]], rho0, rtol=1e-13, atol=0)


def test_relaxation_spares_filled_cells_and_mixtures():
    """Only cells past the seeding threshold relax: a cell with 2% material
    keeps its volume fraction at a threshold of 0.99, and a run with two
    materials is left alone."""
    from oracle.seeding import relax_void
    rho0 = F.STEEL_304L["rho0"]
    U, L, geom = _film_state(0.02, 1.3 * rho0, 10.0, 0.0)
    assert np.array_equal(relax_void(U, geom, L, 0.99, 1e-8), U)
    c = F.uniform_case(1, (4, 1, 1), [F.STEEL_304L, F.STEEL_304L], [0.002, 0.003],
                       [rho0, rho0], [0.0], 0.0, bc="transmissive")
    L2 = Layout(1, c.mats)
    U2 = prim_to_cons(c.prim.copy(), L2, Options(cfl=c.cfl))
    g2 = Geometry(c.dim, c.n, c.lo, c.hi, c.bc)
    assert np.array_equal(relax_void(U2, g2, L2, 0.99, 1e-8), U2)

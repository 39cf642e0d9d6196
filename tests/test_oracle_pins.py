"""Further pins of the oracle against what the paper and the mathematics fix
(CPU only):

  * the Pirondi-Bonora gate of Section 2.2 inside the source step: no damage
    unless p < p_gate, eps_p above the triaxiality-dependent threshold and a
    plastic increment; where the gate is open the step's damage equals the
    exact integral of the Bonora rate over the step's plastic strain;
  * the threshold strain of Section 2.2 at R_t = 2, where the quotient of
    differences factors exactly, and its power law for large R_t;
  * the free surface (Section 3.1 void boundary): an elastic compression
    wave reflected at it leaves the surface moving at twice the particle
    velocity behind the incident wave, with zero normal stress;
  * the shear part of the flux: a tangential-velocity jump splits into two
    shear waves moving at sqrt(G/rho), with the contact at the
    impedance-weighted mean velocity and shear stress rho c_s |jump| / 2.
"""
import math

import numpy as np
import pytest

import fvinputs as F
from oracle import Solver
from oracle import closures as C
from oracle.layout import Layout
from oracle.mixture import Options, prim_to_cons, cons_to_prim
from oracle.scheme import Geometry
from oracle.source import source_step

CU = F.COPPER


# ---------------------------------------------------------------------------
# Pirondi-Bonora gate and the Bonora integral inside the source step
# ---------------------------------------------------------------------------
def _yielding_cell(rho_ratio, p, eps_n, D_n, p_gate, h=(2e-3, -1e-3, -1e-3)):
    """A two-cell periodic 1D copper state: phasic density rho_ratio * rho0,
    pressure p, plastic strain eps_n, damage D_n, and a stretch whose
    deviatoric Hencky strain has eigenvalue logs h (yielding: J > J_max)."""
    m = dict(CU, p_gate=p_gate)
    case = F.uniform_case(1, (2, 1, 1), [m], [1.0], [rho_ratio * CU["rho0"]],
                          [0.0], p, bc="periodic",
                          vbar=np.diag(np.exp(h)).tolist())
    L = Layout(1, case.mats)
    case.prim[L.eps[0]] = eps_n
    case.prim[L.dmg[0]] = D_n
    return case, L


def _source(case, L):
    opts = Options(cfl=case.cfl)
    U = prim_to_cons(case.prim.copy(), L, opts)
    P0 = cons_to_prim(U, L)
    geom = Geometry(case.dim, case.n, case.lo, case.hi, case.bc)
    U1 = source_step(U.copy(), case.phi0, geom, L, opts)
    P1 = cons_to_prim(U1, L)
    return P0, P1


def _J(h):
    h = np.asarray(h) - np.mean(h)
    return float(np.sqrt(np.sum(h * h)))


def test_gate_open_damage_is_the_exact_integral():
    """p = -80 MPa < p_gate = 0, eps_p = 0.1 above the threshold, yielding:
    the Bonora rate dD/deps = A R (Dc - D)^((a-1)/a) / eps at constant R
    integrates exactly to (Dc - D)^(1/a) falling linearly in ln(eps) with
    slope R (Dc - D0)^(1/a) / ln(eps_c/eps_th); the step's damage is that
    integral over [eps_n, eps_n + deps] to RK4 accuracy."""
    h = (2e-3, -1e-3, -1e-3)
    case, L = _yielding_cell(0.999, -8.0e7, 0.1, 0.2, 0.0, h)
    P0, P1 = _source(case, L)
    m = case.mats[0]
    rho = P0.rho_l[0]
    p = P0.p
    Gt = C.solid_shear_modulus(rho, m)
    Jmax = m["yield_stress"] / (math.sqrt(6.0) * Gt)
    deps = math.sqrt(2.0 / 3.0) * (_J(h) - Jmax)
    assert np.allclose(P1.eps[0], 0.1 + deps, rtol=1e-12)
    seq = (1.0 - 0.2) * m["yield_stress"]
    R = C.triaxiality(p, seq, rho, m)
    assert np.all(R > 1.5) and np.all(R < 2.5)      # a moderate triaxiality
    assert np.all(0.1 > C.eps_threshold(R, m))      # above the threshold
    a, Dc, D0 = m["bonora_alpha"], m["D_crit"], m["D0"]
    y0 = (Dc - 0.2) ** (1.0 / a)
    y1 = y0 - R * (Dc - D0) ** (1.0 / a) * np.log((0.1 + deps) / 0.1) / math.log(
        m["eps_c"] / m["eps_th"])
    D_exact = Dc - y1 ** a
    assert np.all(D_exact - 0.2 > 1e-3)              # damage really grew
    assert np.allclose(P1.D[0], D_exact, rtol=1e-9, atol=0)


@pytest.mark.parametrize("what", ["pressure_above_gate", "below_threshold",
                                  "no_plastic_increment", "critical"])
def test_gate_closed_leaves_damage_unchanged(what):
    """Each condition of the gate alone closes it: p >= p_gate, eps_p at or
    below the threshold, no plastic increment in the step, or damage already
    critical.  Plastic strain still accrues where the cell yields."""
    rho_ratio, p, eps_n, D_n, p_gate = 0.999, -8.0e7, 0.1, 0.2, 0.0
    h = (2e-3, -1e-3, -1e-3)
    if what == "pressure_above_gate":
        p_gate = -1.0e8
    elif what == "below_threshold":
        eps_n = 0.02
    elif what == "no_plastic_increment":
        h = (4e-4, -2e-4, -2e-4)                     # J < J_max: elastic
    else:
        D_n = CU["D_crit"]
    case, L = _yielding_cell(rho_ratio, p, eps_n, D_n, p_gate, h)
    P0, P1 = _source(case, L)
    if what == "below_threshold":
        R = C.triaxiality(P0.p, (1.0 - D_n) * CU["yield_stress"],
                          P0.rho_l[0], case.mats[0])
        assert np.all(eps_n <= C.eps_threshold(R, case.mats[0]))
    assert np.array_equal(P1.D[0], P0.D[0])
    if what == "no_plastic_increment":
        assert np.array_equal(P1.eps[0], P0.eps[0])
    elif what != "critical":
        assert np.all(P1.eps[0] > P0.eps[0])


# ---------------------------------------------------------------------------
# threshold strain: exact value at R_t = 2 and the large-R_t power law
# ---------------------------------------------------------------------------
def test_threshold_strain_at_triaxiality_two():
    """At R_t = 2 the quotient (ec^2n - et^2n) / (ec^n - et^n) is exactly
    ec^n + et^n, so eps_thresh = sqrt(et) / 2^(1/n) (ec^n + et^n)^(1/2n)."""
    for et, ec, n in ((0.08, 0.16, 0.31), (0.002, 0.5, 0.313), (0.5, 1.2, 0.22)):
        m = dict(CU, eps_th=et, eps_c=ec, n_hard=n)
        want = math.sqrt(et) / 2.0 ** (1.0 / n) * (ec ** n + et ** n) ** (1.0 / (2.0 * n))
        assert C.eps_threshold(2.0, m) == pytest.approx(want, rel=1e-13)


def test_threshold_strain_large_triaxiality_power_law():
    """For R_t -> inf, et^(1/R) -> 1 and ec^(2n/R) - et^(2n/R) ->
    (2n/R) ln(ec/et), so eps_thresh -> [(ec^2n - et^2n) / (2n ln(ec/et))]^(1/2n)
    R^(-1/2n), with a relative error that falls like 1/R."""
    et, ec, n = CU["eps_th"], CU["eps_c"], CU["n_hard"]
    lim = ((ec ** (2 * n) - et ** (2 * n)) / (2 * n * math.log(ec / et))) ** (1 / (2 * n))
    errs = []
    for R in (1e3, 1e4, 1e5):
        ratio = C.eps_threshold(R, CU) / (lim * R ** (-1.0 / (2 * n)))
        errs.append(abs(ratio - 1.0))
    assert errs[2] < 1e-4
    # the error falls by about a decade per decade of R (a wrong exponent of
    # R would leave a ratio growing or shrinking as a power of R)
    assert 5.0 < errs[0] / errs[1] < 20.0 and 5.0 < errs[1] / errs[2] < 20.0


# ---------------------------------------------------------------------------
# free surface: reflection doubles the particle velocity
# ---------------------------------------------------------------------------
def test_free_surface_reflection_doubles_particle_velocity():
    """Copper on copper at v = 2 m/s (elastic), free ends.  The compression
    wave entering the target carries u = v/2; reflected at the free end it
    returns as a release behind which the material moves at v (twice the
    particle velocity) with zero normal stress."""
    n, Lx, v = 200, 0.01, 2.0
    m = dict(CU, p_gate=-1.0e20)
    case = F.uniform_case(1, (n, 1, 1), [m], [1.0], [CU["rho0"]], [0.0], 0.0,
                          bc="free", lo=(0.0, 0, 0), hi=(Lx, 1, 1))
    L = Layout(1, case.mats)
    x = case.prim[L.X[0]].ravel()
    case.prim[L.mom[0]] = np.where(x < 0.25 * Lx, v, 0.0)[None, None, :]
    s = Solver(case)
    cL = math.sqrt((CU["K0"] + 4.0 * CU["G0"] / 3.0) / CU["rho0"])
    s.run(0.5 * Lx / cL)
    u_inc = s.prim().u[0].ravel()
    # incident wave: between the impact plane and its front (at 0.75 Lx)
    assert u_inc[80:130].mean() == pytest.approx(0.5 * v, rel=0.01)
    s.run(0.9 * Lx / cL)
    P = s.prim()
    u = P.u[0].ravel()
    sxx = P.sigma[0, 0].ravel()
    # the release reflected at t = 0.75 Lx / cL is at 0.85 Lx now; behind it:
    plateau = slice(int(0.90 * n), int(0.98 * n))
    assert u[plateau].mean() == pytest.approx(v, rel=0.02)
    assert u[plateau].mean() / u_inc[80:130].mean() == pytest.approx(2.0, rel=0.02)
    sig_inc = CU["rho0"] * cL * 0.5 * v
    assert np.max(np.abs(sxx[plateau])) < 0.03 * sig_inc
    # the incident stress is still there between the release from the
    # flyer's back (0.65 Lx now) and the reflected one (0.85 Lx)
    assert -sxx[int(0.69 * n):int(0.81 * n)].mean() == pytest.approx(sig_inc, rel=0.03)
    # no material left through the ends' closed faces before the release:
    # the free end moves outward at about v, the impact end at rest
    assert u[-1] == pytest.approx(v, rel=0.03)


# ---------------------------------------------------------------------------
# shear Riemann problem: the contact's tangential state
# ---------------------------------------------------------------------------
def test_shear_jump_splits_into_shear_waves():
    """A jump of tangential velocity u_y = +v_t | -v_t across x = 0 in
    copper at rest otherwise (plane strain, elastic): two shear waves move
    out at c_s = sqrt(G/rho); between them u_y is the impedance-weighted mean
    (0 for equal impedances) and sigma_xy = -rho c_s v_t."""
    nx, Lx, vt = 200, 0.01, 1.0
    case = F.uniform_case(2, (nx, 2, 1), [dict(CU, p_gate=-1.0e20)], [1.0],
                          [CU["rho0"]], [0.0, 0.0], 0.0, bc="periodic",
                          lo=(-0.5 * Lx, 0, 0), hi=(0.5 * Lx, 2 * Lx / nx, 1))
    case.bc = (("transmissive", "transmissive"), ("periodic", "periodic"),
               ("transmissive", "transmissive"))
    L = Layout(2, case.mats)
    x = case.prim[L.X[0]]
    case.prim[L.mom[1]] = np.where(x < 0.0, vt, -vt)
    s = Solver(case)
    cs = math.sqrt(CU["G0"] / CU["rho0"])
    cL = math.sqrt((CU["K0"] + 4.0 * CU["G0"] / 3.0) / CU["rho0"])
    dx = Lx / nx
    t = 50 * dx / cs
    s.run(t)
    P = s.prim()
    uy = P.u[1][0].mean(axis=0)
    sxy = P.sigma[0, 1][0].mean(axis=0)
    xc = -0.5 * Lx + (np.arange(nx) + 0.5) * dx
    # contact plateau (between the fronts at -/+ c_s t = 50 cells)
    mid = np.abs(xc) < 30 * dx
    assert np.max(np.abs(uy[mid])) < 0.02 * vt
    assert sxy[mid].mean() == pytest.approx(-CU["rho0"] * cs * vt, rel=0.02)
    # fronts: u_y crosses half the jump at x = -/+ c_s t
    right = xc[np.nonzero(uy < -0.5 * vt)[0].min()]
    left = xc[np.nonzero(uy > 0.5 * vt)[0].max()]
    assert right == pytest.approx(cs * s.t, abs=2 * dx)
    assert left == pytest.approx(-cs * s.t, abs=2 * dx)
    # a shear jump drives no normal wave: the normal stress stays at the
    # rounding of the second-order shear effects
    assert np.max(np.abs(P.sigma[0, 0][0])) < 0.01 * CU["rho0"] * cs * vt
    # nothing moved at the longitudinal speed: outside the shear fronts the
    # material is undisturbed
    far = np.abs(xc) > (cs * s.t + 6 * dx)
    assert np.all(np.abs(np.abs(uy[far]) - vt) < 1e-3 * vt)
    assert cL * s.t > cs * s.t + 6 * dx        # the test can tell the two apart

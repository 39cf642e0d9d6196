"""Pins of the trace-material reading of the mixture (CPU only).

A material whose volume fraction is below the trace threshold takes the
limit of its closures as its phasic density vanishes (the Romenskii cold
energy, cold pressure, stiffness and shear modulus of Section 2.3 all tend
to zero there).  What that fixes independently of the oracle's own code:

  * a gas cell holding a trace solid, with any distortion, damage or phasic
    density of the trace, obeys the ideal-gas law p = (gamma - 1) rho e and
    c^2 = gamma p / rho up to the trace's Grueneisen share of the thermal
    part (a relative amount of the order of the trace fraction), and carries
    no shear stress;
  * a strongly expanded solid crossing the threshold moves the thermal
    energy by no more than its mass times its cold binding energy, whatever
    its distortion;
  * the source step leaves such a cell with no elastic distortion and does
    no plastic work there, so neither the plastic strain nor the damage of
    the trace moves; a trace solid in a cell that another solid stiffens
    takes no share of that solid's plastic increment.
"""
import numpy as np
import pytest

import fvinputs as F
from oracle import mixture as M
from oracle.layout import Layout
from oracle.mixture import Options, prim_to_cons, cons_to_prim
from oracle.scheme import Geometry
from oracle.source import source_step

CU = F.COPPER
GAS = F.GAS


def _mix(phi_s, rho_s, phi_g, rho_g, rho_e, J2, D):
    mats = [CU, GAS]
    phi = np.array([[phi_s], [phi_g]])
    rho_l = np.array([[rho_s], [rho_g]])
    terms = M.material_terms(rho_l, {0: np.array([D])}, np.array([J2]), mats,
                             phi)
    p = M.pressure_from_energy(phi, terms, np.array([rho_e]), mats)
    rho = float(np.sum(phi * rho_l))
    c, G = M.sound_speed(phi, rho_l, terms, p, np.array([rho]), mats)
    H = np.zeros((3, 3, 1))
    h = np.sqrt(J2 / 1.5)                 # dev H = diag(h, -h/2, -h/2)
    H[0, 0, 0], H[1, 1, 0], H[2, 2, 0] = h, -0.5 * h, -0.5 * h
    sig = M.stress(phi, p, G, H)
    return p[0], c[0], G[0], sig[:, :, 0], rho


@pytest.mark.parametrize("phi_s", [1e-8, 3e-7, 0.999e-6])
@pytest.mark.parametrize("J2,D,rho_s", [(0.0, 0.0, 8930.0), (50.0, 0.9, 0.05),
                                         (8.0, 0.4, 1.0e5), (1e-3, 0.0, 1e-6)])
def test_gas_cell_with_a_trace_solid_is_an_ideal_gas(phi_s, J2, D, rho_s):
    gamma = GAS["gamma"] if "gamma" in GAS else 1.4
    phi_g = 1.0 - phi_s
    rho_g, e_g = 1.2e-3, 2.5e5              # rarefied gas
    rho_e = phi_g * rho_g * e_g
    p, c, G, sig, rho = _mix(phi_s, rho_s, phi_g, rho_g, rho_e, J2, D)
    p_ideal = (gamma - 1.0) * rho_e / phi_g   # the gas phase's own law
    tol = 10.0 * phi_s
    assert p == pytest.approx(p_ideal, rel=tol)
    assert G == 0.0
    assert np.all(sig - np.diag(np.diag(sig)) == 0.0)
    assert np.allclose(np.diag(sig), -p, rtol=0.0, atol=1e-15 * p)
    # c^2 = gamma p / rho_g for the gas phase (the trace's mass share of rho
    # is rho_s phi_s / rho, kept within the bound by rho_s <= 1e5)
    c_ideal = np.sqrt(gamma * p / (rho / phi_g))
    assert c == pytest.approx(c_ideal, rel=tol + 2.0 * phi_s * rho_s / rho)


@pytest.mark.parametrize("eta", [1e-7, 1e-4])
def test_threshold_jump_is_the_trace_binding_energy_whatever_the_distortion(eta):
    """A strongly expanded solid (eta = rho_s/rho0 of the fragments' wake)
    in near-vacuum gas, just above and just below the trace fraction.  Its
    reference terms vanish with its phasic density except the cold energy
    per unit mass, which tends to the binding energy K0/(2 rho0 alpha^2)
    (Section 2.3 cold curve as eta -> 0).  So switching the trace off moves
    the thermal energy by at most the trace mass times that energy,
    phi rho_s (1-D) K0/(2 rho0 alpha^2), whatever the distortion J^2: the
    jump in pressure is that amount times Gamma_gas / (phi_gas), and the
    same at J^2 = 0 and J^2 = 50.  (Evaluating a trace at its reference
    density would instead add phi (1-D) beta G0 J^2 / (Gamma xi) below the
    threshold: about 4e2 Pa at J^2 = 50 here, against a gas at 1 Pa.)"""
    rho_s = eta * CU["rho0"]
    phi_s, D = 1e-6, 0.5
    rho_e = 2.5                              # gas at ~1 Pa
    jumps = []
    for J2 in (0.0, 50.0):
        above = _mix(phi_s * (1 + 1e-12), rho_s, 0.4, 8e-6, rho_e, J2, D)
        below = _mix(phi_s * (1 - 1e-12), rho_s, 0.4, 8e-6, rho_e, J2, D)
        jumps.append(below[0] - above[0])
        # the shear stress of the expanded solid is negligible on both sides
        assert abs(above[3][1, 1] - above[3][2, 2]) < 1e-9 * abs(above[0])
    bind = phi_s * rho_s * (1 - D) * CU["K0"] / (2 * CU["rho0"] * CU["alpha"] ** 2)
    xi = 0.4 / GAS["Gamma0"] + phi_s / CU["Gamma0"]
    assert jumps[0] > 0.0
    assert jumps[0] <= bind / xi * (1 + 1e-6)
    assert jumps[1] == pytest.approx(jumps[0], rel=1e-6, abs=1e-15)


def _cell_with_trace(phi_s, rho_s, h):
    mats = [CU, dict(GAS)]
    case = F.uniform_case(1, (2, 1, 1), mats, [phi_s, 1.0 - phi_s],
                          [rho_s, 1.2], [0.0], 1.0e5, bc="periodic",
                          vbar=np.diag(np.exp(h)).tolist())
    L = Layout(1, case.mats)
    case.prim[L.eps[0]] = 0.3
    case.prim[L.dmg[0]] = 0.2
    opts = Options(cfl=case.cfl)
    U = prim_to_cons(case.prim.copy(), L, opts)
    geom = Geometry(case.dim, case.n, case.lo, case.hi, case.bc)
    U1 = source_step(U.copy(), case.phi0, geom, L, opts)
    return cons_to_prim(U, L), cons_to_prim(U1, L), L


def test_source_step_drops_distortion_of_a_cell_without_stiffness():
    h = np.array([1.5, -1.0, -0.5])              # J^2 = 3.5: far past yield
    P0, P1, L = _cell_with_trace(1e-8, CU["rho0"], h)
    assert np.allclose(P1.V[:, :, 0, 0, 0], np.eye(3), rtol=0, atol=1e-15)
    assert P1.eps[0][0, 0, 0] == pytest.approx(P0.eps[0][0, 0, 0], rel=1e-15)
    assert P1.D[0][0, 0, 0] == pytest.approx(P0.D[0][0, 0, 0], rel=1e-15)
    # the energy is untouched, and the pressure (gas only) with it
    assert P1.p[0, 0, 0] == pytest.approx(P0.p[0, 0, 0], rel=1e-14)


def test_source_step_returns_a_live_solid_to_its_yield_surface():
    """Control: the same distortion with the solid above the trace fraction
    is returned to the yield surface, with plastic strain sqrt(2/3) dJ."""
    h = np.array([2e-3, -1e-3, -1e-3])
    P0, P1, L = _cell_with_trace(0.5, CU["rho0"], h)
    J0 = np.sqrt(np.sum(h * h))
    Gt = CU["G0"]
    Jmax = CU["yield_stress"] / (np.sqrt(6.0) * Gt)
    assert J0 > Jmax
    assert np.sqrt(P1.J2[0, 0, 0]) == pytest.approx(Jmax, rel=1e-9)
    assert P1.eps[0][0, 0, 0] - P0.eps[0][0, 0, 0] == pytest.approx(
        np.sqrt(2.0 / 3.0) * (J0 - Jmax), rel=1e-9)


def test_trace_solid_takes_no_share_of_another_solids_plastic_work():
    """Two solids (the spallation test's aluminium and copper): the copper
    at a trace fraction in a yielding aluminium cell keeps its plastic
    strain and damage while the aluminium's grow by the return's increment."""
    al, cu = dict(F.AL_H32, jc_B=0.0, jc_C=0.0), dict(F.CUBE, jc_C=0.0, p_gate=1e30)
    h = np.array([2e-2, -1.2e-2, -0.8e-2])
    case = F.uniform_case(1, (2, 1, 1), [cu, al], [1e-8, 1.0 - 1e-8],
                          [cu["rho0"], al["rho0"]], [0.0], -2.0e9,
                          bc="periodic", vbar=np.diag(np.exp(h)).tolist())
    L = Layout(1, case.mats)
    case.prim[L.eps[0]] = 0.5
    case.prim[L.dmg[0]] = 0.3
    opts = Options(cfl=case.cfl)
    U = prim_to_cons(case.prim.copy(), L, opts)
    geom = Geometry(case.dim, case.n, case.lo, case.hi, case.bc)
    P0 = cons_to_prim(U, L)
    P1 = cons_to_prim(source_step(U.copy(), case.phi0, geom, L, opts), L)
    J0 = np.sqrt(np.sum(h * h))
    d_al = np.sqrt(2.0 / 3.0) * (J0 - al["yield_stress"] / (np.sqrt(6.0) * al["G0"]))
    assert P1.eps[1][0, 0, 0] - P0.eps[1][0, 0, 0] == pytest.approx(d_al, rel=1e-6)
    assert P1.eps[0][0, 0, 0] == pytest.approx(P0.eps[0][0, 0, 0], rel=1e-14)
    assert P1.D[0][0, 0, 0] == pytest.approx(P0.D[0][0, 0, 0], rel=1e-14)

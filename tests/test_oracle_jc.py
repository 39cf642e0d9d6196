"""Pins of the Johnson-Cook plasticity of the oracle (CPU only).

The paper names Johnson-Cook plasticity for its solids and tabulates its
constants (c1, c2, c3, n, m, T_melt, C_V) without printing the law; the
oracle takes the law of Johnson and Cook (1983), the radial return solved
for the plastic increment Delta with the yield evaluated at the end of the
step, and the temperature from the thermal energy of Section 2.2.  What the
mathematics fixes independently of the oracle's bisection:

  * linear hardening (n = 1): sqrt6 G (J - sqrt(3/2) Delta) = A + B (eps + Delta)
    has the closed form Delta = (sqrt6 G J - A - B eps) / (3 G + B);
  * the rate term alone: the root of sqrt6 G J - 3 G Delta =
    A (1 + C ln(Delta / dt)) found by an independent bracketing solver
    (scipy's brentq);
  * thermal softening: at the melting temperature the yield vanishes and the
    return removes the whole distortion; below it the constant-yield closed
    form holds with the yield scaled by 1 - T*^m;
  * the temperature of a state on its cold curve is T_REF eta^Gamma0, and an
    added thermal energy e_t raises it by e_t / C_V;
  * with c2 = c3 = 0 and no melting temperature the law is the constant
    yield of the other workloads.
"""
import numpy as np
import pytest
import scipy.optimize

import fvinputs as F
from oracle import closures as C
from oracle.layout import Layout
from oracle.mixture import Options, prim_to_cons, cons_to_prim
from oracle.scheme import Geometry
from oracle.source import source_step

STEEL = F.STEEL_304L


def _cell(m, h, eps_n=0.0, rho_ratio=1.0, p=0.0):
    """Two-cell periodic 1D state of material m with deviatoric Hencky
    eigenvalue logs h and plastic strain eps_n (damage gate closed)."""
    m = dict(m, p_gate=-1e30)
    case = F.uniform_case(1, (2, 1, 1), [m], [1.0], [rho_ratio * m["rho0"]],
                          [0.0], p, bc="periodic",
                          vbar=np.diag(np.exp(h)).tolist())
    L = Layout(1, case.mats)
    case.prim[L.eps[0]] = eps_n
    opts = Options(cfl=case.cfl)
    U = prim_to_cons(case.prim.copy(), L, opts)
    geom = Geometry(case.dim, case.n, case.lo, case.hi, case.bc)
    return case, L, U, geom, opts


def _return(m, h, eps_n=0.0, dt=None, rho_ratio=1.0, p=0.0):
    case, L, U, geom, opts = _cell(m, h, eps_n, rho_ratio, p)
    P0 = cons_to_prim(U, L)
    U1 = source_step(U.copy(), case.phi0, geom, L, opts, dt)
    P1 = cons_to_prim(U1, L)
    J0 = np.sqrt(np.sum(np.asarray(h) ** 2))
    J1 = float(np.sqrt(P1.J2[0, 0, 0]))
    d = float(P1.eps[0][0, 0, 0] - P0.eps[0][0, 0, 0])
    return J0, J1, d, P0


H = np.array([2e-2, -1.2e-2, -0.8e-2])          # far past the initial yield


def test_linear_hardening_has_the_closed_form_increment():
    m = dict(STEEL, jc_B=0.685e9, n_hard=1.0, jc_C=0.0, T_melt=0.0)
    eps_n = 0.05
    J0, J1, d, P0 = _return(m, H, eps_n)
    G = C.solid_shear_modulus(m["rho0"], m)
    A, B = m["yield_stress"], m["jc_B"]
    want = (np.sqrt(6.0) * G * J0 - A - B * eps_n) / (3.0 * G + B)
    assert want > 0
    assert d == pytest.approx(want, rel=1e-12)
    assert J1 == pytest.approx(J0 - np.sqrt(1.5) * want, rel=1e-12)
    # on the hardened yield surface
    assert np.sqrt(6.0) * G * J1 == pytest.approx(A + B * (eps_n + want), rel=1e-12)


def test_rate_term_matches_an_independent_root_finder():
    m = dict(STEEL, jc_B=0.0, jc_C=0.097, T_melt=0.0)
    dt = 2e-9
    J0, J1, d, P0 = _return(m, H, 0.0, dt)
    G = C.solid_shear_modulus(m["rho0"], m)
    A, Cc = m["yield_stress"], m["jc_C"]

    def f(x):
        return (np.sqrt(6.0) * G * J0 - 3.0 * G * x
                - A * (1.0 + Cc * np.log(max(x / dt, 1.0))))
    want = scipy.optimize.brentq(f, 1e-30, np.sqrt(2.0 / 3.0) * J0, xtol=1e-300,
                                 rtol=1e-15, maxiter=500)
    assert d == pytest.approx(want, rel=1e-12)
    # faster than the reference rate: the rate term raised the yield
    assert d / dt > 1.0
    assert np.sqrt(6.0) * G * J1 > A


def test_rate_term_is_off_without_a_time_step():
    m = dict(STEEL, jc_B=0.0, jc_C=0.097, T_melt=0.0)
    J0, J1, d, P0 = _return(m, H, 0.0, None)
    G = C.solid_shear_modulus(m["rho0"], m)
    assert np.sqrt(6.0) * G * J1 == pytest.approx(m["yield_stress"], rel=1e-12)


def _state_at_temperature(m, T, h):
    """Pressure of a reference-density state with deviatoric Hencky
    eigenvalue logs h whose temperature is T: its reference pressure is the
    shear term beta G0 J^2 (the cold pressure vanishes at rho0), and the
    thermal part adds rho Gamma0 C_V (T - T_REF)."""
    J2 = float(np.sum(np.asarray(h) ** 2))
    return (m["beta"] * m["G0"] * J2
            + m["rho0"] * m["Gamma0"] * m["C_V"] * (T - C.T_REF))


def test_temperature_of_the_cold_curve_and_of_added_heat():
    m = dict(STEEL, C_V=468.6)
    for eta in (0.9, 1.0, 1.1):
        rho = eta * m["rho0"]
        assert C.temperature(np.array([1e9]), np.array([1e9]), np.array([rho]),
                             m)[0] == pytest.approx(C.T_REF * eta ** m["Gamma0"], rel=1e-14)
    rho = m["rho0"]
    et = 2.0e5
    p = rho * m["Gamma0"] * et
    assert C.temperature(np.array([p]), np.array([0.0]), np.array([rho]),
                         m)[0] == pytest.approx(C.T_REF + et / m["C_V"], rel=1e-14)


@pytest.mark.parametrize("T", [900.0, 1689.0, 2000.0])
def test_thermal_softening(T):
    m = dict(STEEL, jc_B=0.0, jc_C=0.0, T_melt=1689.0, jc_m=2.044, C_V=468.6)
    h = [1e-3, -6e-4, -4e-4]
    p = _state_at_temperature(m, T, h)
    J0, J1, d, P0 = _return(m, h, 0.0, None, 1.0, p)
    G = C.solid_shear_modulus(m["rho0"], m)
    Ts = min(max((T - C.T_REF) / (m["T_melt"] - C.T_REF), 0.0), 1.0)
    Y = m["yield_stress"] * (1.0 - Ts ** m["jc_m"])
    if Y == 0.0:
        assert J1 == pytest.approx(0.0, abs=1e-15)
        assert d == pytest.approx(np.sqrt(2.0 / 3.0) * J0, rel=1e-12)
    else:
        assert np.sqrt(6.0) * G * J1 == pytest.approx(Y, rel=1e-9)


def test_constant_yield_is_the_special_case():
    m0 = dict(STEEL)
    m1 = dict(STEEL, jc_B=0.0, jc_C=0.0, T_melt=0.0)
    assert not C.jc_active(m0) and not C.jc_active(m1)
    a = _return(m0, H)
    b = _return(m1, H, 0.0, 1e-9)
    assert a[1] == b[1] and a[2] == b[2]
    G = C.solid_shear_modulus(m0["rho0"], m0)
    assert np.sqrt(6.0) * G * a[1] == pytest.approx(m0["yield_stress"], rel=1e-12)


def test_spallation_materials_from_paper_tables():
    """The two solids of the spallation test and the full 304L row carry
    the paper's Appendix A constants (tests/golden/paper_tables.json)."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                    "golden", "paper_tables.json")))
    for m, r, jc in ((F.CUBE, g["romenskii_cube"], g["johnson_cook_cube"]),
                     (F.AL_H32, g["romenskii_al_h32"], g["johnson_cook_al_h32"]),
                     (F.STEEL_304L_JC, g["romenskii_304l"], g["johnson_cook_304l"])):
        assert m["rho0"] == r["rho0"]
        assert m["K0"] == pytest.approx(r["K0_GPa"] * 1e9, rel=1e-15)
        assert m["G0"] == pytest.approx(r["G0_GPa"] * 1e9, rel=1e-15)
        assert (m["alpha"], m["beta"], m["Gamma0"]) == (r["alpha"], r["beta"], r["Gamma0"])
        assert m["yield_stress"] == pytest.approx(jc["c1_GPa"] * 1e9, rel=1e-15)
        assert m["jc_B"] == pytest.approx(jc["c2_GPa"] * 1e9, rel=1e-15)
        assert m["jc_C"] == jc["c3"] and m["n_hard"] == jc["n"]
    s = F.STEEL_304L_JC
    j = g["johnson_cook_304l"]
    assert (s["jc_m"], s["T_melt"], s["C_V"]) == (j["m"], j["T_melt"], j["C_V"])
    b = g["bonora_cube"]
    assert (F.CUBE["D_crit"], F.CUBE["eps_th"], F.CUBE["eps_c"], F.CUBE["bonora_alpha"]) == (
        b["D_crit"], b["eps_thresh"], b["eps_crit"], b["alpha"])
    c = F.al_cube_spall(2)
    assert c.n[:2] == (800, 800) and c.cfl == 0.4 and c.t_end == 5e-6
    assert c.hi[0] - c.lo[0] == pytest.approx(0.011, rel=1e-15)

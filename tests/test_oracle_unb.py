"""Pins of the U-Nb closures of the oracle (CPU only): the Steinberg shear
modulus, the Burakovsky-Preston Grueneisen function and Debye temperature,
and the simplified damage law of the paper's ring (Sections 2.3, 4.3).

What the definitions fix independently of the closed forms the oracle uses:
  * G~ = G0 at the reference density (p_c = 0), and the reference pressure
    and its derivative are the density derivatives of the reference energy
    with the shear energy G~ J^2 / rho (finite differences);
  * the Grueneisen function is the logarithmic derivative of the Debye
    temperature, and rho Gamma'/Gamma that of Gamma (finite differences);
  * the mixture sound speed is the isentropic derivative of the pressure;
  * the temperature of a state on its cold curve is T_REF theta_D(rho);
  * the simplified law integrated by the source step's RK4 matches its
    closed form D = 1 - (1 - D_n) exp(-Ddot0 d_eps);
  * the constants are the paper's rows (tests/golden/paper_tables.json).
"""
import json
import os

import numpy as np
import pytest

import fvinputs as F
from oracle import closures as C
from oracle import mixture as M
from oracle.source import damage_rk4

U = F.UNB
HERE = os.path.dirname(os.path.abspath(__file__))


def fd(f, x, h):
    return (f(x + h) - f(x - h)) / (2 * h)


def test_steinberg_modulus_at_reference_density():
    G, rG1, r2G2 = C.shear_terms(np.array([U["rho0"]]), U)
    assert G[0] == pytest.approx(U["G0"], rel=1e-15)


@pytest.mark.parametrize("eta", [0.85, 1.0, 1.12])
@pytest.mark.parametrize("J2", [0.0, 3e-4])
def test_reference_pressure_and_stiffness_are_energy_derivatives(eta, J2):
    rho = eta * U["rho0"]
    D = 0.05

    def e_ref(r):
        re, _, _, _ = C.ref_terms(np.array([r]), np.array([J2]), np.array([D]), U)
        return re[0] / r

    def p_ref(r):
        return C.ref_terms(np.array([r]), np.array([J2]), np.array([D]), U)[1][0]
    h = 1e-5 * rho
    re, pref, rdp, G = C.ref_terms(np.array([rho]), np.array([J2]), np.array([D]), U)
    # finite differences of energies of order K0 round at ~1e-11 K0
    tol = 1e-9 * U["K0"]
    assert pref[0] == pytest.approx(rho * rho * fd(e_ref, rho, h), rel=1e-6, abs=tol)
    assert rdp[0] == pytest.approx(rho * fd(p_ref, rho, h), rel=1e-6, abs=tol)
    # the Steinberg modulus is G0 + G_p p_c eta^(-1/3)
    _, pc, _ = C.solid_cold(np.array([rho]), U)
    assert G[0] == pytest.approx((1 - D) * (U["G0"] + U["G_p"] * pc[0] * eta ** (-1 / 3)),
                                 rel=1e-14)


@pytest.mark.parametrize("eta", [0.8, 1.0, 1.25])
def test_gruneisen_is_log_derivative_of_debye_temperature(eta):
    rho = eta * U["rho0"]
    h = 1e-6
    lnth = lambda lr: np.log(C.debye_theta(U, np.exp(lr)))
    g = fd(lnth, np.log(rho), h)
    assert C.gruneisen(U, np.array([rho]))[0] == pytest.approx(g, rel=1e-8)
    lng = lambda lr: np.log(C.gruneisen(U, np.array([np.exp(lr)]))[0])
    assert C.gruneisen_dlog(U, np.array([rho]))[0] == pytest.approx(
        fd(lng, np.log(rho), h), rel=1e-7)
    # at the reference density Gamma = Gamma0 + Gamma1 + Gamma2
    assert C.gruneisen(U, np.array([U["rho0"]]))[0] == pytest.approx(
        U["Gamma0"] + U["Gamma1"] + U["Gamma2"], rel=1e-15)


@pytest.mark.parametrize("eta,J2,D", [(1.0, 0.0, 0.0), (1.06, 2e-4, 0.02),
                                      (0.93, 1e-4, 0.05)])
def test_sound_speed_is_isentropic_derivative(eta, J2, D):
    rho = eta * U["rho0"]
    mats = [U]
    phi = np.array([[1.0]])

    def p_of(r, e):
        terms = M.material_terms(np.array([[r]]), {0: np.array([D])}, np.array([J2]), mats)
        return M.pressure_from_energy(phi, terms, np.array([r * e]), mats)[0]
    e = 1.0e5
    p = p_of(rho, e)
    terms = M.material_terms(np.array([[rho]]), {0: np.array([D])}, np.array([J2]), mats)
    c, G = M.sound_speed(phi, np.array([[rho]]), terms, np.array([p]), np.array([rho]), mats)
    h = 1e-5 * rho
    pp = p_of(rho + h, e + p / rho ** 2 * h)
    pm = p_of(rho - h, e - p / rho ** 2 * h)
    cb2 = (pp - pm) / (2 * h)
    assert c[0] ** 2 == pytest.approx(cb2 + 4.0 / 3.0 * G[0] / rho, rel=1e-6)


def test_cold_curve_temperature_uses_the_debye_temperature():
    for eta in (0.9, 1.0, 1.1):
        rho = eta * U["rho0"]
        T = C.temperature(np.array([2e9]), np.array([2e9]), np.array([rho]), U)[0]
        assert T == pytest.approx(C.T_REF * C.debye_theta(U, rho), rel=1e-14)


@pytest.mark.parametrize("Dn,deps", [(0.0, 0.05), (0.03, 0.2), (0.09, 0.3)])
def test_simplified_damage_matches_closed_form(Dn, deps):
    D = damage_rk4(np.array([Dn]), np.array([0.3]), np.array([deps]), np.array([1.0]), U)[0]
    exact = 1.0 - (1.0 - Dn) * np.exp(-U["Ddot0"] * deps)
    # RK4's local error on y' = -k y is y (k h)^5 / 120 at leading order
    bound = 2.0 * (1.0 - Dn) * (U["Ddot0"] * deps) ** 5 / 120.0
    assert abs(D - min(exact, U["D_crit"])) <= bound


def test_unb_constants_from_paper_tables():
    g = json.load(open(os.path.join(HERE, "golden", "paper_tables.json")))
    r, j, d = g["romenskii_steinberg_unb"], g["johnson_cook_unb"], g["simplified_damage_unb"]
    assert U["rho0"] == r["rho0"] and U["alpha"] == r["alpha"]
    assert U["K0"] == pytest.approx(r["K0_GPa"] * 1e9, rel=1e-15)
    assert U["G0"] == pytest.approx(r["G0_GPa"] * 1e9, rel=1e-15)
    assert (U["G_p"], U["Gamma0"], U["Gamma1"], U["Gamma2"], U["gamma_bp"]) == (
        r["G_p"], r["Gamma0"], r["Gamma1"], r["Gamma2"], r["gamma"])
    assert U["yield_stress"] == pytest.approx(j["c1_GPa"] * 1e9, rel=1e-15)
    assert U["jc_B"] == pytest.approx(j["c2_GPa"] * 1e9, rel=1e-15)
    assert (U["jc_C"], U["n_hard"], U["jc_m"], U["T_melt"], U["C_V"]) == (
        j["c3"], j["n"], j["m"], j["T_melt"], j["C_V"])
    assert (U["Ddot0"], U["D_crit"]) == (d["Ddot0"], d["D_crit"])


def test_driver_radius_is_the_integral_of_its_speed():
    import scipy.integrate
    from oracle.driver import driver_radius, driver_speed
    d = F.UNB_DRIVER
    for t in (5e-6, 17.5e-6, 25e-6, 35e-6, 48e-6):
        integral, _ = scipy.integrate.quad(lambda s: driver_speed(d, s), 0.0, t,
                                           points=[d[3], d[4]], epsabs=1e-15)
        assert driver_radius(d, t) == pytest.approx(d[0] + integral, rel=1e-13)
    # continuous speed at t0 and t1
    assert driver_speed(d, d[3] * (1 - 1e-12)) == pytest.approx(d[1], rel=1e-9)
    assert driver_speed(d, d[4] * (1 - 1e-12)) == pytest.approx(d[2], rel=1e-9)


def test_driver_sets_the_radial_speed_behind_its_surface_and_adds_its_work():
    from oracle.driver import apply_driver, driver_radius, driver_speed
    from oracle.layout import Layout
    from oracle.mixture import Options, prim_to_cons, cons_to_prim
    from oracle.scheme import Geometry
    n = 24
    mats = [U]
    case = F.uniform_case(2, (n, n, 1), mats, [1.0], [U["rho0"]], [3.0, -4.0],
                          1.0e8, bc="transmissive", lo=(-0.024, -0.024, 0.0),
                          hi=(0.024, 0.024, 1.0))
    L = Layout(2, mats)
    U0 = prim_to_cons(case.prim.copy(), L, Options())
    geom = Geometry(2, case.n, case.lo, case.hi, case.bc)
    d = (0.010, 210.0, 160.0, 17.5e-6, 35.0e-6, 0.030)
    t = 20e-6
    U1 = apply_driver(U0.copy(), geom, L, d, t)
    Rd, vr = driver_radius(d, t), driver_speed(d, t)
    cx = case.lo[0] + (np.arange(n) + 0.5) * 0.048 / n
    X, Y = np.meshgrid(cx, cx, indexing="xy")
    r = np.sqrt(X * X + Y * Y)
    rho = U0[L.mass[0]][0]
    u0 = np.stack([U0[L.mom[k]][0] / rho for k in range(2)])
    u1 = np.stack([U1[L.mom[k]][0] / rho for k in range(2)])
    inside = r <= Rd
    assert inside.sum() > 10 and (~inside).sum() > 10
    ur1 = (u1[0] * X + u1[1] * Y) / r
    assert np.allclose(ur1[inside], vr, rtol=1e-12)
    # tangential velocity kept
    ut0 = (-u0[0] * Y + u0[1] * X) / r
    ut1 = (-u1[0] * Y + u1[1] * X) / r
    assert np.allclose(ut1, ut0, rtol=1e-12, atol=1e-12)
    assert np.array_equal(U1[:, 0][:, ~inside], U0[:, 0][:, ~inside])
    dE = U1[L.energy][0] - U0[L.energy][0]
    assert np.allclose(dE[inside], 0.5 * rho[inside] * (np.sum(u1 * u1, 0) - np.sum(u0 * u0, 0))[inside],
                       rtol=1e-10)
    assert np.array_equal(U1[L.mass], U0[L.mass])
    # arrested beyond r_max
    U2 = apply_driver(U0.copy(), geom, L, (0.010, 210.0, 160.0, 17.5e-6, 35.0e-6, 0.012), t)
    assert np.array_equal(U2, U0)

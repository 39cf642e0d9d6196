"""Pins of the oracle's closures against what the paper and the mathematics
fix (CPU only): derivative identities of the EOS, limits, the uniaxial-strain
closed form, the Bonora closed-form integral, the triaxiality identity of the
log EOS (Section 2.2), and library matrix logarithms."""
import numpy as np
import pytest
import scipy.linalg

import fvinputs as F
from oracle import closures as C
from oracle import kinematics as K
from oracle import mixture as M
from oracle.source import damage_rk4

CU = F.COPPER
GAS = F.GAS


def fd(f, x, h):
    return (f(x + h) - f(x - h)) / (2 * h)


def test_romenskii_reference_point():
    """p_c(rho0) = 0 and dp_c/drho(rho0) = K0/rho0 (both forms of the
    Romenskii energy give K0 at rho0)."""
    rho0 = CU["rho0"]
    rho_ec, pc, rho_dpc = C.solid_cold(np.array([rho0]), CU)
    assert pc[0] == 0.0
    assert rho_ec[0] == 0.0
    assert rho_dpc[0] == pytest.approx(CU["K0"], rel=1e-14)


@pytest.mark.parametrize("alpha", [1.0, 0.569, 0.627354])
def test_romenskii_pressure_is_energy_derivative(alpha):
    """p_c = rho^2 de_c/drho and rho dp_c/drho checked by finite
    differences of the energy (Section 2.2, pressure as energy derivative)."""
    m = dict(CU, alpha=alpha)
    for eta in (0.8, 0.97, 1.0, 1.05, 1.3):
        rho = eta * m["rho0"]

        def ec(r):
            return C.solid_cold(np.array([r]), m)[0][0] / r

        def pc(r):
            return C.solid_cold(np.array([r]), m)[1][0]

        h = 1e-4 * rho
        p_fd = rho * rho * fd(ec, rho, h)
        _, p, rdp = C.solid_cold(np.array([rho]), m)
        assert p[0] == pytest.approx(p_fd, rel=1e-7, abs=1e-8 * m["K0"])
        assert rdp[0] == pytest.approx(rho * fd(pc, rho, h), rel=1e-7)


def test_romenskii_alpha_to_zero_is_log_eos():
    """alpha -> 0 gives the logarithmic EOS the paper uses in its proof
    (Section 2.2): e_c = K0/(2 rho0) ln^2(rho/rho0)."""
    m = dict(CU, alpha=1e-7)
    for eta in (0.7, 0.9, 1.1, 1.4):
        rho = eta * m["rho0"]
        rho_ec, pc, _ = C.solid_cold(np.array([rho]), m)
        log_ec = m["K0"] / (2 * m["rho0"]) * np.log(eta) ** 2
        log_pc = m["K0"] * eta * np.log(eta)
        assert rho_ec[0] / rho == pytest.approx(log_ec, rel=1e-5)
        assert pc[0] == pytest.approx(log_pc, rel=1e-5)


def test_shear_pressure_is_energy_derivative():
    """rho^2 d(G J^2/rho)/drho = beta G J^2 for G = G0 eta^(beta+1)."""
    J2 = 3e-6
    for eta in (0.9, 1.0, 1.2):
        rho = eta * CU["rho0"]

        def es(r):
            return C.solid_shear_modulus(r, CU) * J2 / r

        p_fd = rho * rho * fd(es, rho, 1e-4 * rho)
        _, pref, _, _ = C.ref_terms(np.array([rho]), np.array([J2]),
                                    np.array([0.0]), CU)
        _, pc, _ = C.solid_cold(np.array([rho]), CU)
        assert pref[0] - pc[0] == pytest.approx(p_fd, rel=1e-6)


def _single(m, rho, e, J2=0.0, D=0.0):
    phi = np.array([[1.0]])
    rho_l = np.array([[rho]])
    terms = M.material_terms(rho_l, {0: np.array([D])} if m["kind"] == "solid"
                             else {}, np.array([J2]), [m])
    p = M.pressure_from_energy(phi, terms, np.array([rho * e]), [m])
    c, G = M.sound_speed(phi, rho_l, terms, p, np.array([rho]), [m])
    return p[0], c[0], G[0]


def test_ideal_gas_limit():
    """Gas: e_ref = p_ref = 0 and Gamma = gamma - 1 give p = 0.4 rho e and
    c^2 = 1.4 p / rho."""
    p, c, G = _single(GAS, 1.3, 2.0e5)
    assert p == pytest.approx(0.4 * 1.3 * 2.0e5, rel=1e-15)
    assert c == pytest.approx(np.sqrt(1.4 * p / 1.3), rel=1e-15)
    assert G == 0.0


@pytest.mark.parametrize("eta,J2,D", [(1.0, 0.0, 0.0), (1.04, 2e-6, 0.0),
                                      (0.95, 1e-6, 0.3)])
def test_sound_speed_is_isentropic_derivative(eta, J2, D):
    """The bulk part of c^2 equals dp/drho along de = p/rho^2 drho (finite
    differences of the pressure function), plus (4/3) G / rho."""
    rho = eta * CU["rho0"]
    e = 5.0e4          # above the cold curve (positive thermal energy)
    p, c, G = _single(CU, rho, e, J2, D)
    h = 1e-5 * rho
    pp, _, _ = _single(CU, rho + h, e + p / rho ** 2 * h, J2, D)
    pm, _, _ = _single(CU, rho - h, e - p / rho ** 2 * h, J2, D)
    cb2 = (pp - pm) / (2 * h)
    assert c * c == pytest.approx(cb2 + 4.0 / 3.0 * G / rho, rel=1e-6)


def test_mixture_sound_speed_is_isentropic_derivative():
    """Two materials and void, volume fractions fixed: the bulk part of the
    mixture c^2 equals d((1 - nu) p)/drho along the mixture isentrope with
    every phasic density scaled alike."""
    mats = [CU, GAS]
    phi = np.array([[0.6], [0.3]])
    rho_l = np.array([[8.7e3], [1.7]])
    D = {0: np.array([0.1])}
    J2 = np.array([1e-6])
    rho = float(np.sum(phi * rho_l))
    rho_e = 2.0e9      # p > 0: both phases above their cold curves

    def pmix(scale, re):
        rl = rho_l * scale
        terms = M.material_terms(rl, D, J2, mats)
        p = M.pressure_from_energy(phi, terms, np.array([re]), mats)
        return M.solid_fraction(phi)[0] * p[0]

    terms = M.material_terms(rho_l, D, J2, mats)
    p = M.pressure_from_energy(phi, terms, np.array([rho_e]), mats)
    c, G = M.sound_speed(phi, rho_l, terms, p, np.array([rho]), mats)
    pm_ = M.solid_fraction(phi)[0] * p[0]
    h = 1e-6
    # d(rho e) = (rho e + p_mix) drho / rho along the isentrope
    dre = (rho_e + pm_) * h
    cb2 = (pmix(1 + h, rho_e + dre) - pmix(1 - h, rho_e - dre)) / (2 * h * rho)
    assert c[0] ** 2 == pytest.approx(cb2 + 4.0 / 3.0 * G[0] / rho, rel=1e-6)


def test_mixture_reduces_to_single_material():
    """phi_gas at the floor: mixture pressure equals the copper EOS."""
    mats = [CU, GAS]
    rho = 9.1e3
    e = 5.0e3
    phi = np.array([[1.0], [0.0]])
    rho_l = np.array([[rho], [1.0]])
    terms = M.material_terms(rho_l, {0: np.array([0.0])}, np.array([0.0]),
                             mats)
    p2 = M.pressure_from_energy(phi, terms, np.array([rho * e]), mats)
    p1, _, _ = _single(CU, rho, e)
    assert p2[0] == pytest.approx(p1, rel=1e-14)


def test_uniaxial_strain_closed_form():
    """Vbar = diag(eta^-2/3, eta^1/3, eta^1/3): J^2 = (2/3) ln^2 eta and
    sigma_eq = sqrt(6) G J = 2 G |ln eta| (Section 2.2)."""
    for eta in (0.9, 0.99, 1.02, 1.2):
        V = np.zeros((3, 3, 1))
        V[0, 0, 0] = eta ** (-2.0 / 3.0)
        V[1, 1, 0] = V[2, 2, 0] = eta ** (1.0 / 3.0)
        H, h, Q = K.hencky(V)
        J2 = K.J2_of(H)[0]
        assert J2 == pytest.approx(2.0 / 3.0 * np.log(eta) ** 2, rel=1e-12)
        G = 45e9
        assert np.sqrt(6 * J2) * G == pytest.approx(2 * G * abs(np.log(eta)),
                                                    rel=1e-12)


def test_hencky_matches_scipy_logm():
    rng = np.random.default_rng(7)
    for _ in range(20):
        A = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
        A /= np.cbrt(np.linalg.det(A))
        H, h, Q = K.hencky(A[:, :, None])
        B = A @ A.T
        ref = 0.5 * scipy.linalg.logm(B).real
        ref -= np.trace(ref) / 3 * np.eye(3)
        assert np.allclose(H[:, :, 0], ref, atol=1e-13)
        V = K.stretch_from_log(h, Q)[:, :, 0]
        assert np.allclose(V @ V.T, B / np.cbrt(np.linalg.det(B)), atol=1e-13)
        assert np.allclose(V, V.T, atol=1e-14)


def test_moduli_relations():
    """E/K = 3(1 - 2 nu) and E/(2G) = 1 + nu (Section 2.2)."""
    nu = C.poisson_ratio(CU)
    E = C.young_modulus(CU)
    assert E / CU["K0"] == pytest.approx(3 * (1 - 2 * nu), rel=1e-14)
    assert E / (2 * CU["G0"]) == pytest.approx(1 + nu, rel=1e-14)


def test_triaxiality_uniaxial_tension_is_one():
    """Uniaxial tension p / sigma_eq = -1/3 at rho = rho0 gives R_t = 1 for
    any Poisson ratio (Section 2.2), and the threshold strain is eps_th."""
    for G0 in (20e9, 45e9, 80e9):
        m = dict(CU, G0=G0)
        R = C.triaxiality(np.array([-30e6]), np.array([90e6]),
                          np.array([m["rho0"]]), m)
        assert R[0] == pytest.approx(1.0, rel=1e-14)
    assert C.eps_threshold(1.0, CU) == pytest.approx(CU["eps_th"], rel=1e-14)


def test_triaxiality_log_eos_identity():
    """For the logarithmic cold energy the energy release rate
    rho e~_c + G~ J^2 equals sigma_eq^2/((1-D)^2 2E) R_t(p_c/sigma_eq) with
    the nominal stresses sigma_eq = (1-D) sqrt(6) G~ J and
    p_c = (1-D) p~_c (Section 2.2, proof of the triaxiality form)."""
    m = CU
    Kb, G = m["K0"], m["G0"]
    E = C.young_modulus(m)
    D = 0.2
    for eta, J in ((0.97, 1e-3), (1.03, 2e-3), (0.9, 5e-4)):
        rho = eta * m["rho0"]
        rho_ec = rho * Kb / (2 * m["rho0"]) * np.log(eta) ** 2
        # nominal (damaged) cold pressure, as the identity requires
        pc = (1 - D) * Kb * eta * np.log(eta)
        lhs = rho_ec + G * J * J
        seq = (1 - D) * np.sqrt(6.0) * G * J
        R = C.triaxiality(np.array([pc]), np.array([seq]), np.array([rho]), m)
        rhs = seq ** 2 / ((1 - D) ** 2 * 2 * E) * R[0]
        assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("R", [1.0, 1.7, 3.0])
def test_bonora_rk4_matches_closed_form(R):
    """At constant triaxiality the Bonora rate integrates in closed form;
    D = D_c exactly at eps_c when R = 1 (Section 2.2)."""
    m = CU
    eps = m["eps_th"]
    D = np.array([m["D0"]])
    n = 4000
    e_end = m["eps_th"] * np.exp(0.9 * np.log(m["eps_c"] / m["eps_th"]) / R)
    h = (e_end - eps) / n
    for _ in range(n):
        D = damage_rk4(D, np.array([eps]), np.array([h]), np.array([R]), m)
        eps += h
    ref = C.bonora_closed_form(np.array([e_end]), R, m)[0]
    assert D[0] == pytest.approx(ref, rel=1e-9)
    assert C.bonora_closed_form(np.array([m["eps_c"]]), 1.0, m)[0] == \
        pytest.approx(m["D_crit"], rel=1e-15)


def test_bonora_clamps_at_critical():
    m = CU
    D = damage_rk4(np.array([0.899]), np.array([0.1]), np.array([0.05]),
                   np.array([5.0]), m)
    assert D[0] == m["D_crit"]


def test_threshold_strain_spall_value():
    """Large triaxiality (spall, R_t ~ 245) drives the threshold strain to
    ~1e-5."""
    v = C.eps_threshold(245.0, CU)
    assert 1e-6 < v < 1e-4


def test_sound_speed_below_cold_curve_keeps_cold_stiffness():
    """A state below the cold curve (negative thermal energy) takes the cold
    pressure and keeps the cold and shear stiffness in c^2 (mixture reading:
    the thermal part is bounded below by zero)."""
    rho = 1.04 * CU["rho0"]
    J2 = 2e-6
    p, c, G = _single(CU, rho, 3.0e3, J2)
    terms = M.material_terms(np.array([[rho]]), {0: np.array([0.0])},
                             np.array([J2]), [CU])
    _, pref, rho_dpref, _ = terms[0]
    # the pressure inversion clamps the thermal part: p is the cold pressure
    assert p == pytest.approx(pref[0], rel=1e-14)
    assert c * c == pytest.approx(rho_dpref[0] / rho + 4.0 / 3.0 * G / rho,
                                  rel=1e-13)

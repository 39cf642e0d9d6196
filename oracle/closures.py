"""Single-material closures (Sections 2.2 and 2.3) -- oracle, FP64.

Energies are per unit mass, pressures in Pa.  To stay finite for a vanishing
phasic density the helpers return products with the density (rho*e, rho*dp/drho)
rather than specific quantities divided by it.

Readings of garbled or silent passages:
  * Romenskii cold energy (Section 2.3): the denominator is read as
    2 rho0 alpha^2, so that alpha -> 0 gives the logarithmic EOS the paper
    uses in its triaxiality proof (Section 2.2).
  * Thermal part (Section 2.2) with the Romenskii Debye temperature
    theta = eta^Gamma0 gives Gamma = Gamma0 and the Mie-Grueneisen form
    p = p_ref(rho) + rho Gamma0 (e - e_ref(rho)) with e_ref = e_c + e_s.
  * Damage degrades both cold and shear energies by (1 - D) (Section 2.2).
"""
import numpy as np


def solid_cold(rho, m, second=False):
    """Romenskii cold compression (Section 2.3, Romenskii EOS):
    e_c = K0/(2 rho0 alpha^2) (eta^alpha - 1)^2, eta = rho/rho0.
    Returns (rho*e_c, p_c = rho^2 de_c/drho, rho * dp_c/drho), and with
    `second` also rho^2 d2p_c/drho2; with p_c = (K0/alpha)(eta^(2a+1) -
    eta^(a+1)) the derivatives are eta-derivatives:
    rho p_c' = (K0/a)((2a+1) eta^(2a+1) - (a+1) eta^(a+1)),
    rho^2 p_c'' = (K0/a)((2a+1) 2a eta^(2a+1) - (a+1) a eta^(a+1))."""
    K0, rho0, a = m["K0"], m["rho0"], m["alpha"]
    eta = rho / rho0
    ea = eta ** a
    rho_ec = rho * K0 / (2.0 * rho0 * a * a) * (ea - 1.0) ** 2
    pc = (K0 / a) * eta ** (a + 1.0) * (ea - 1.0)
    rho_dpc = (K0 / a) * eta ** (a + 1.0) * ((2.0 * a + 1.0) * ea - (a + 1.0))
    if not second:
        return rho_ec, pc, rho_dpc
    r2 = (K0 / a) * eta ** (a + 1.0) * ((2.0 * a + 1.0) * 2.0 * a * ea - (a + 1.0) * a)
    return rho_ec, pc, rho_dpc, r2


def steinberg(m):
    """Whether a solid takes the Steinberg shear modulus (G_p given)."""
    return m.get("G_p", 0.0) > 0.0


def shear_terms(rho, m):
    """Shear modulus G~ and its density derivatives rho G~' and rho^2 G~''.
    Romenskii (Section 2.3): G~ = G0 eta^(beta+1), so rho G~' = (beta+1) G~
    and rho^2 G~'' = (beta+1) beta G~.  Steinberg (Section 2.3, the U-Nb
    ring): G~ = G0 + G_p p_c(rho) eta^(-1/3), whose derivatives follow from
    those of the cold pressure:
    rho G~' = G_p eta^(-1/3) (rho p_c' - p_c/3),
    rho^2 G~'' = G_p eta^(-1/3) (rho^2 p_c'' - (2/3) rho p_c' + (4/9) p_c)."""
    if not steinberg(m):
        b1 = m["beta"] + 1.0
        G = m["G0"] * (rho / m["rho0"]) ** b1
        return G, b1 * G, b1 * (b1 - 1.0) * G
    _, pc, rdpc, r2 = solid_cold(rho, m, second=True)
    e3 = (rho / m["rho0"]) ** (-1.0 / 3.0)
    Gp = m["G_p"]
    G = m["G0"] + Gp * pc * e3
    return (G, Gp * e3 * (rdpc - pc / 3.0),
            Gp * e3 * (r2 - (2.0 / 3.0) * rdpc + (4.0 / 9.0) * pc))


def solid_shear_modulus(rho, m):
    """Shear modulus G~ (Romenskii or Steinberg form, Section 2.3)."""
    return shear_terms(rho, m)[0]


def ref_terms(rho, J2, D, m):
    """Reference (zero-temperature) terms of one material for the
    Mie-Grueneisen form: rho*e_ref, p_ref, rho*dp_ref/drho and the degraded
    shear modulus G = (1-D) G~ (Sections 2.2, 2.3).  With the shear energy
    e_s = G~ J^2 / rho of Section 2.2:

    e_ref = (1-D)(e~_c + G~ J^2 / rho),
    p_ref = rho^2 de_ref/drho = (1-D)(p~_c + (rho G~' - G~) J^2),
    rho dp_ref/drho = (1-D)(rho p~_c' + rho^2 G~'' J^2)
    (for the Romenskii modulus rho G~' - G~ = beta G~).  Gas: all zero."""
    if m["kind"] != "solid":
        z = np.zeros_like(rho)
        return z, z, z, z
    rho_ec, pc, rho_dpc = solid_cold(rho, m)
    Gt, rG1, r2G2 = shear_terms(rho, m)
    w = 1.0 - D
    rho_eref = w * (rho_ec + Gt * J2)
    pref = w * (pc + (rG1 - Gt) * J2)
    rho_dpref = w * (rho_dpc + r2G2 * J2)
    return rho_eref, pref, rho_dpref, w * Gt


# A damage value within this relative distance of D_crit counts as critical.
# The source step clamps damage at D_crit; the stages then carry it as the
# ratio (phi rho D)/(phi rho) of two independently updated fields.  In double
# precision each stage rounds both at the unit 2^-53 (about 1.1e-16), scaled by
# the cancellation between a cell's mass and its flux differences, so a cell
# that stays critical (its neighbours critical too) returns D_crit only to a
# relative 1e-13..1e-11 after the 10^4..10^5 steps of the workloads (more in
# near-empty cells).  The critical test of Section 3.1 (D >= D_crit) is read as
# holding within 1e-9 of D_crit: far above that rounding, far below the
# healing the same section describes (diffusion mixing undamaged material
# into a critical cell), which moves the ratio by the mixed-in mass fraction.
CRIT_REL_TOL = 1.0e-9


# The sign tests on stress, the tension of the void-opening modifier (Section
# 3.1) and the pressure gate of the damage law, hold beyond the same relative
# band of the solid's bulk modulus.  A void cell relaxed to its film's zero
# pressure sits at zero stress up to the rounding of its state (K times the
# unit of the storage precision); the band puts such a cell on the side of no
# tension and a closed gate instead of letting rounding decide.
def stress_band(m, rel_tol=CRIT_REL_TOL):
    """Width of the band of the stress sign tests: rel_tol K0 (Pa)."""
    return rel_tol * m["K0"]


def is_critical(D, m, rel_tol=CRIT_REL_TOL):
    """Critical damage test of Section 3.1, D >= D_crit, up to the double
    precision rounding of the advected ratio (see CRIT_REL_TOL).  rel_tol
    lets a test run the oracle with another band (the single-precision
    storage policy of the FP32-bulk kernels) to separate the effect of the
    band from that of the arithmetic."""
    return D >= m["D_crit"] * (1.0 - rel_tol)


def burakovsky_preston(m):
    """Whether a material takes the Burakovsky-Preston Grueneisen function
    (Gamma1 or Gamma2 given)."""
    return m.get("Gamma1", 0.0) != 0.0 or m.get("Gamma2", 0.0) != 0.0


def gruneisen(m, rho=None):
    """Grueneisen function.  Romenskii (and gases): the constant Gamma0.
    Burakovsky-Preston (Section 2.3, with the Steinberg modulus):
    Gamma = Gamma0 + Gamma1 eta^(-1/3) + Gamma2 eta^(-gamma), Gamma0 in the
    role of Gamma_infinity."""
    if rho is None or not burakovsky_preston(m):
        return m["Gamma0"] if rho is None else np.full_like(np.asarray(rho, dtype=float), m["Gamma0"])
    eta = rho / m["rho0"]
    return (m["Gamma0"] + m["Gamma1"] * eta ** (-1.0 / 3.0)
            + m["Gamma2"] * eta ** (-m["gamma_bp"]))


def gruneisen_dlog(m, rho):
    """rho Gamma'(rho) / Gamma: zero for a constant Gamma; for
    Burakovsky-Preston (-Gamma1 eta^(-1/3)/3 - gamma Gamma2 eta^(-gamma))
    / Gamma."""
    if not burakovsky_preston(m):
        return np.zeros_like(np.asarray(rho, dtype=float))
    eta = rho / m["rho0"]
    d = (-m["Gamma1"] * eta ** (-1.0 / 3.0) / 3.0
         - m["gamma_bp"] * m["Gamma2"] * eta ** (-m["gamma_bp"]))
    return d / gruneisen(m, rho)


def debye_theta(m, rho):
    """Non-dimensional Debye temperature theta_D (Section 2.3): eta^Gamma0
    (Romenskii), or eta^Gamma0 exp[3 Gamma1 (1 - eta^(-1/3)) + (Gamma2 /
    gamma)(1 - eta^(-gamma))] (Burakovsky-Preston), whose logarithmic
    derivative is the Grueneisen function."""
    eta = rho / m["rho0"]
    th = eta ** m["Gamma0"]
    if burakovsky_preston(m):
        g = m["gamma_bp"]
        th = th * np.exp(3.0 * m["Gamma1"] * (1.0 - eta ** (-1.0 / 3.0))
                         + (m["Gamma2"] / g) * (1.0 - eta ** (-g)))
    return th


def poisson_ratio(m):
    """nu~ = (3K - 2G) / (2 (3K + G)) from the undamaged moduli at rho0
    (the moduli relations used in the triaxiality proof, Section 2.2)."""
    K, G = m["K0"], m["G0"]
    return (3.0 * K - 2.0 * G) / (2.0 * (3.0 * K + G))


def young_modulus(m):
    K, G = m["K0"], m["G0"]
    return 9.0 * K * G / (3.0 * K + G)


def triaxiality(p, sigma_eq, rho, m):
    """Stress triaxiality function in the paper's first form with the
    hydrostatic pressure (Section 2.2):
    R_t = 3 (1 - 2 nu) (rho0/rho) (p/sigma_eq)^2 + (2/3)(1 + nu)."""
    nu = poisson_ratio(m)
    return (3.0 * (1.0 - 2.0 * nu) * (m["rho0"] / rho) * (p / sigma_eq) ** 2
            + (2.0 / 3.0) * (1.0 + nu))


def eps_threshold(R, m):
    """Triaxiality-dependent threshold plastic strain (Section 2.2, last
    equation of the Pirondi-Bonora extension):
    eps_th^(1/R) / R^(1/n) * ((eps_c^(2n) - eps_th^(2n)) /
                              (eps_c^(2n/R) - eps_th^(2n/R)))^(1/(2n))."""
    et, ec, n = m["eps_th"], m["eps_c"], m["n_hard"]
    num = ec ** (2.0 * n) - et ** (2.0 * n)
    den = ec ** (2.0 * n / R) - et ** (2.0 * n / R)
    return et ** (1.0 / R) / R ** (1.0 / n) * (num / den) ** (1.0 / (2.0 * n))


def bonora_prefactor(m):
    """alpha (D_c - D_0)^(1/alpha) / ln(eps_c / eps_th) of the Bonora damage
    rate (Section 2.2, damage source term)."""
    a = m["bonora_alpha"]
    return (a * (m["D_crit"] - m["D0"]) ** (1.0 / a)
            / np.log(m["eps_c"] / m["eps_th"]))


def bonora_dD_deps(D, eps, R, m):
    """dD/d(eps_p) of the Bonora law (Section 2.2):
    A R (D_c - D)^((alpha-1)/alpha) / eps_p, zero at or above D_c."""
    a = m["bonora_alpha"]
    Dc = m["D_crit"]
    y = np.maximum(Dc - D, 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = bonora_prefactor(m) * R * y ** ((a - 1.0) / a) / eps
    return np.where(D >= Dc, 0.0, r)


def bonora_closed_form(eps, R, m):
    """D(eps_p) from D_0 at eps_th under constant triaxiality: the exact
    integral of the Bonora law (used as a pin, not by the solver)."""
    a = m["bonora_alpha"]
    Dc, D0 = m["D_crit"], m["D0"]
    s = 1.0 - R * np.log(eps / m["eps_th"]) / np.log(m["eps_c"] / m["eps_th"])
    s = np.maximum(s, 0.0)
    return Dc - ((Dc - D0) ** (1.0 / a) * s) ** a


# ---------------------------------------------------------------------------
# Johnson-Cook plasticity (named by the paper for its solids, with the
# constants of its Appendix A plasticity table: c1, c2, c3, n, m, T_melt,
# C_V; the law itself is not printed).  The form is the one of Johnson and
# Cook (1983):
#   sigma_Y = (c1 + c2 eps_p^n) (1 + c3 ln max(rate / RATE_REF, 1))
#             (1 - T*^m),   T* = clamp((T - T_REF) / (T_melt - T_REF), 0, 1).
# Readings: the reference strain rate is 1/s and rates below it leave the
# yield at its quasi-static value; the reference temperature of the law and
# of the thermal energy below is room temperature, 300 K; a material without
# a melting temperature (the paper's "-" entries) has no thermal softening.
# With c2 = c3 = 0 and no melting temperature the law is the constant yield
# c1 of the workloads that do not use it.
# ---------------------------------------------------------------------------
T_REF = 300.0
RATE_REF = 1.0


def jc_active(m):
    """Whether a material's yield depends on strain, rate or temperature."""
    return (m["kind"] == "solid"
            and (m.get("jc_B", 0.0) != 0.0 or m.get("jc_C", 0.0) != 0.0
                 or m.get("T_melt", 0.0) > 0.0))


def jc_flow_stress(eps, rate, T, m):
    """Johnson-Cook flow stress at plastic strain eps, plastic strain rate
    `rate` [1/s] and temperature T [K] (see above)."""
    A, B, C = m["yield_stress"], m.get("jc_B", 0.0), m.get("jc_C", 0.0)
    hard = A + B * np.power(np.maximum(eps, 0.0), m["n_hard"])
    rfac = 1.0 + C * np.log(np.maximum(rate / RATE_REF, 1.0))
    Tm = m.get("T_melt", 0.0)
    if Tm > 0.0:
        Ts = np.clip((T - T_REF) / (Tm - T_REF), 0.0, 1.0)
        tfac = 1.0 - Ts ** m["jc_m"]
    else:
        tfac = 1.0
    return hard * rfac * tfac


def temperature(p, pref, rho, m):
    """Phase temperature from the thermal energy of Section 2.2,
    E_t = C_V (T - T0 theta_D(rho)) with T0 = T_REF: under the Mie-Grueneisen
    form the thermal energy per unit mass is e_t = (p - p_ref)/(rho Gamma),
    taken non-negative (the cold curve is the zero-temperature bound), so
    T = e_t / C_V + T_REF theta_D(rho).  A material without C_V has no
    temperature (returned as T_REF)."""
    cv = m.get("C_V", 0.0)
    if cv <= 0.0:
        return np.full_like(np.asarray(p, dtype=float), T_REF)
    g = gruneisen(m, rho)
    et = np.maximum(p - pref, 0.0) / (rho * g)
    return et / cv + T_REF * debye_theta(m, rho)

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


def solid_cold(rho, m):
    """Romenskii cold compression (Section 2.3, Romenskii EOS):
    e_c = K0/(2 rho0 alpha^2) (eta^alpha - 1)^2, eta = rho/rho0.
    Returns (rho*e_c, p_c = rho^2 de_c/drho, rho * dp_c/drho)."""
    K0, rho0, a = m["K0"], m["rho0"], m["alpha"]
    eta = rho / rho0
    ea = eta ** a
    rho_ec = rho * K0 / (2.0 * rho0 * a * a) * (ea - 1.0) ** 2
    pc = (K0 / a) * eta ** (a + 1.0) * (ea - 1.0)
    rho_dpc = (K0 / a) * eta ** (a + 1.0) * ((2.0 * a + 1.0) * ea - (a + 1.0))
    return rho_ec, pc, rho_dpc


def solid_shear_modulus(rho, m):
    """Romenskii shear modulus G = G0 eta^(beta+1) (Section 2.3)."""
    return m["G0"] * (rho / m["rho0"]) ** (m["beta"] + 1.0)


def ref_terms(rho, J2, D, m):
    """Reference (zero-temperature) terms of one material for the
    Mie-Grueneisen form: rho*e_ref, p_ref, rho*dp_ref/drho and the degraded
    shear modulus G = (1-D) G~ (Sections 2.2, 2.3).

    e_ref = (1-D)(e~_c + G~ J^2 / rho);  p_ref = (1-D)(p~_c + beta G~ J^2)
    since rho^2 d(G~ J^2/rho)/drho = beta G~ J^2 for the Romenskii modulus.
    Gas: all zero."""
    if m["kind"] != "solid":
        z = np.zeros_like(rho)
        return z, z, z, z
    rho_ec, pc, rho_dpc = solid_cold(rho, m)
    Gt = solid_shear_modulus(rho, m)
    b = m["beta"]
    w = 1.0 - D
    rho_eref = w * (rho_ec + Gt * J2)
    pref = w * (pc + b * Gt * J2)
    rho_dpref = w * (rho_dpc + b * (b + 1.0) * Gt * J2)
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


def is_critical(D, m, rel_tol=CRIT_REL_TOL):
    """Critical damage test of Section 3.1, D >= D_crit, up to the double
    precision rounding of the advected ratio (see CRIT_REL_TOL).  rel_tol
    lets a test run the oracle with another band (the single-precision
    storage policy of the FP32-bulk kernels) to separate the effect of the
    band from that of the arithmetic."""
    return D >= m["D_crit"] * (1.0 - rel_tol)


def gruneisen(m):
    return m["Gamma0"]


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
    E_t = C_V (T - T0 theta_D(rho)), with the Romenskii Debye temperature
    theta_D = eta^Gamma0 and T0 = T_REF: under the Mie-Grueneisen form the
    thermal energy per unit mass is e_t = (p - p_ref) / (rho Gamma0), taken
    non-negative (the cold curve is the zero-temperature bound), so
    T = e_t / C_V + T_REF eta^Gamma0.  A material without C_V has no
    temperature (returned as T_REF)."""
    cv = m.get("C_V", 0.0)
    if cv <= 0.0:
        return np.full_like(np.asarray(p, dtype=float), T_REF)
    g = m["Gamma0"]
    et = np.maximum(p - pref, 0.0) / (rho * g)
    return et / cv + T_REF * (rho / m["rho0"]) ** g

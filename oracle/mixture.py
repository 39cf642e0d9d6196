"""Mixture closures and conserved <-> primitive conversion -- oracle, FP64.

The mixture rules are deferred by the paper to earlier work (Section 2.3,
last paragraph); the reading used here is the Allaire-type closure under the
paper's mechanical and thermal equilibrium assumption (Section 2.1):

  * pressure: rho e = sum_l phi_l rho_l e_l(rho_l, p) solved for the common
    p with each e_l in Mie-Grueneisen form, i.e.
      p = [rho e - sum phi_l rho_l e_ref,l + sum phi_l p_ref,l / Gamma_l]
          / sum (phi_l / Gamma_l)
  * stress: the void carries none, so the mixture stress is the
    volume-weighted material stress
      sigma = -(1 - nu) p I + 2 G_mix dev(H),  G_mix = sum phi_l G_l
    (this makes the mixture work rate equal sum phi_l p_l div u, the
    energy-consistent choice; with no void it is -p I + 2 G dev H)
  * trace materials (phi < PHI_TRACE) take the vanishing-density limit of
    their closures: no reference energy, pressure, stiffness or shear
    modulus, only their Grueneisen share in the thermal part; the thermal
    energy density is taken non-negative in the pressure inversion (both
    guard cells emptied to near vacuum).
  * sound speed: the frozen (Allaire) mixture bulk speed scaled by (1 - nu),
    plus the shear contribution, c^2 = c_b^2 + (4/3) G_mix / rho; each
    phase's thermal term (Gamma + 1 + rho Gamma'/Gamma)(p - p_ref) enters
    non-negative (a state
    below the cold curve, as a gas fraction pulled into tension in a mixed
    cell, must not drive the wave-speed estimate to zero).
Parity of the mixture rule itself is unpinned against the paper (it is not
printed there); the single-material limit is pinned.
"""
import numpy as np

from .closures import ref_terms, gruneisen, gruneisen_dlog
from .kinematics import full_vbar, hencky, J2_of

C_MIN2 = 1.0e-6       # floor on c^2 [m^2/s^2]


class Options:
    def __init__(self, phi_floor=1.0e-8, cfl=0.6, weno_eps=1.0e-6,
                 crit_rel_tol=None, seed_nu=0.0, thinc_beta=0.0):
        self.phi_floor = phi_floor
        # THINC steepness for the volume fractions (0: MUSCL)
        self.thinc_beta = thinc_beta
        self.cfl = cfl
        self.weno_eps = weno_eps
        # void-fraction threshold of the Lagrangian seeding (0: off)
        self.seed_nu = seed_nu
        # band of the critical-damage test (None: the double-precision
        # reading, closures.CRIT_REL_TOL)
        self.crit_rel_tol = crit_rel_tol


# Volume fraction below which a material is a trace: its phasic density, the
# ratio of two trace quantities, is noise.  A trace material takes the limit
# of its closures as its phasic density vanishes, where the Romenskii cold
# energy, cold pressure, stiffness and shear modulus all go to zero: it
# carries no reference terms and no shear stiffness, and enters the mixture
# only through its Grueneisen share of the thermal part.  The trace solids
# that matter are the ones left in cells emptied to near vacuum, whose phasic
# density is far below rho0; there the limit is continuous with the closures
# just above the threshold.  (Evaluating a trace at its reference density
# instead gives it the full modulus G0: in a near-vacuum cell whose stretch
# the return no longer bounds -- an expanded solid has almost no modulus, so
# any distortion is elastic -- crossing the threshold then switched on a
# reference energy phi G0 J^2 larger than the cell's whole energy.)
PHI_TRACE = 1.0e-6


def closure_density(phi_l, rho_l, m):
    """Density at which closures that need one (the triaxiality's rho0/rho)
    are evaluated: the reference density for a trace material."""
    return np.where(phi_l < PHI_TRACE, m["rho0"], rho_l)


class Terms(tuple):
    """(rho e_ref, p_ref, rho dp_ref/drho, G) of one material, carrying its
    Grueneisen share as attributes: inv_gamma = 1/Gamma(rho_l) and
    g1 = Gamma + 1 + rho Gamma'/Gamma, the factor of the thermal pressure in
    rho c^2 (d/drho of p = p_ref + rho Gamma (e - e_ref) along an isentrope,
    with p_ref = rho^2 de_ref/drho, gives rho c^2 = rho p_ref' +
    (Gamma + 1 + rho Gamma'/Gamma)(p - p_ref))."""
    pass


def material_terms(rho_l, D_l, J2, mats, phi=None):
    """Per-material (rho e_ref, p_ref, rho dp_ref/drho, G) lists with their
    Grueneisen shares (see Terms); zero reference terms for a trace material
    (phi < PHI_TRACE), whose Grueneisen function is taken at the reference
    density."""
    out = []
    for l, m in enumerate(mats):
        D = D_l[l] if l in D_l else np.zeros_like(J2)
        t = ref_terms(rho_l[l], J2, D, m)
        rg = rho_l[l]
        if phi is not None:
            live = phi[l] >= PHI_TRACE
            t = tuple(np.where(live, v, 0.0) for v in t)
            rg = np.where(live, rho_l[l], m["rho0"])
        t = Terms(t)
        g = gruneisen(m, rg)
        t.inv_gamma = 1.0 / g
        t.g1 = g + 1.0 + gruneisen_dlog(m, rg)
        out.append(t)
    return out


def _inv_gamma(t, m):
    return getattr(t, "inv_gamma", 1.0 / gruneisen(m))


def _g1(t, m):
    return getattr(t, "g1", gruneisen(m) + 1.0)


def pressure_from_energy(phi, terms, rho_e, mats):
    """Mixture pressure inversion; the thermal energy density
    rho e - sum phi rho e_ref is taken non-negative (the cold curve is the
    zero-temperature bound; below it the state is numerical, as in cells
    emptied to near vacuum or a gas fraction pulled into tension)."""
    xi = sum(phi[l] * _inv_gamma(terms[l], m) for l, m in enumerate(mats))
    th = rho_e.copy()
    cold = np.zeros_like(rho_e)
    for l, m in enumerate(mats):
        rho_eref, pref, _, _ = terms[l]
        th = th - phi[l] * rho_eref
        cold = cold + phi[l] * pref * _inv_gamma(terms[l], m)
    return (np.maximum(th, 0.0) + cold) / xi


def energy_from_pressure(phi, terms, p, mats):
    xi = sum(phi[l] * _inv_gamma(terms[l], m) for l, m in enumerate(mats))
    rho_e = xi * p
    for l, m in enumerate(mats):
        rho_eref, pref, _, _ = terms[l]
        rho_e = rho_e + phi[l] * rho_eref - phi[l] * pref * _inv_gamma(terms[l], m)
    return rho_e


def solid_fraction(phi):
    """1 - nu with the void fraction nu = 1 - sum phi clamped to [0, 1]."""
    s = np.sum(phi, axis=0)
    return np.clip(s, 0.0, 1.0)


def sound_speed(phi, rho_l, terms, p, rho, mats):
    """Longitudinal mixture sound speed (see module docstring)."""
    xi = sum(phi[l] * _inv_gamma(terms[l], m) for l, m in enumerate(mats))
    acc = np.zeros_like(p)
    Gmix = np.zeros_like(p)
    for l, m in enumerate(mats):
        _, pref, rho_dpref, G = terms[l]
        # thermal part taken non-negative: a state below the cold curve is
        # not physical and must not pull the wave-speed estimate to zero
        acc = acc + phi[l] * _inv_gamma(terms[l], m) * (
            rho_dpref + _g1(terms[l], m) * np.maximum(p - pref, 0.0))
        Gmix = Gmix + phi[l] * G
    # acc = sum phi_l xi_l rho_l c_l^2 (with rho_l c_l^2 = rho_l p_ref' +
    # (Gamma_l + 1)(p - p_ref,l)); bulk c^2 = (1-nu) acc / (xi rho)
    cb2 = solid_fraction(phi) * acc / (xi * rho)
    c2 = np.maximum(cb2, 0.0) + (4.0 / 3.0) * Gmix / rho
    return np.sqrt(np.maximum(c2, C_MIN2)), Gmix


def stress(phi, p, Gmix, H):
    s = 2.0 * Gmix[None, None] * H
    f = solid_fraction(phi)
    for i in range(3):
        s[i, i] = s[i, i] - f * p
    return s


def prim_to_cons(W, layout, opts):
    """Conserved state from the generator's primitive array (same field
    order, rho_l in place of phi_l rho_l, eps/D in place of the history
    densities, velocity, pressure in place of energy).  Volume fractions are
    clamped to [phi_floor, 1]."""
    L = layout
    dim, mats = L.dim, L.mats
    shape = W.shape[1:]
    phi = np.clip(W[L.phi], opts.phi_floor, 1.0)
    rho_l = W[L.mass]
    D_l = {l: W[L.dmg[l]] for l in L.solids}
    V = full_vbar(W[L.vbar], L.vcomps, shape)
    H, _, _ = hencky(V)
    J2 = J2_of(H)
    terms = material_terms(rho_l, D_l, J2, mats, phi)
    p = W[L.energy]                       # pressure sits in the energy slot
    rho_e = energy_from_pressure(phi, terms, p, mats)
    rho = np.sum(phi * rho_l, axis=0)
    u = W[L.mom]
    U = np.zeros_like(W)
    U[L.phi] = phi
    U[L.mass] = phi * rho_l
    for l in L.solids:
        U[L.eps[l]] = phi[l] * rho_l[l] * W[L.eps[l]]
        U[L.dmg[l]] = phi[l] * rho_l[l] * W[L.dmg[l]]
    U[L.mom] = rho[None] * u
    U[L.energy] = rho_e + 0.5 * rho * np.sum(u * u, axis=0)
    U[L.vbar] = W[L.vbar]
    U[L.X] = W[L.X]
    return U


class Prim:
    """Cell primitives and derived quantities."""
    pass


def cons_to_prim(U, layout):
    """Primitive and derived cell quantities from the conserved state."""
    L = layout
    dim, mats = L.dim, L.mats
    shape = U.shape[1:]
    P = Prim()
    phi = U[L.phi]
    mass = np.maximum(U[L.mass], 0.0)
    rho_l = mass / phi
    rho = np.sum(mass, axis=0)
    P.phi, P.rho_l, P.rho = phi, rho_l, rho
    P.eps, P.D = {}, {}
    for l in L.solids:
        ml = U[L.mass[l]]
        pos = ml > 0
        safe = np.where(pos, ml, 1.0)
        P.eps[l] = np.where(pos, U[L.eps[l]] / safe, 0.0)
        P.D[l] = np.where(pos, U[L.dmg[l]] / safe, 0.0)
    u = np.zeros((3,) + shape)
    for k in range(dim):
        u[k] = U[L.mom[k]] / rho
    P.u = u
    rho_e = U[L.energy] - 0.5 * rho * np.sum(u * u, axis=0)
    V = full_vbar(U[L.vbar], L.vcomps, shape)
    H, _, _ = hencky(V)
    J2 = J2_of(H)
    terms = material_terms(rho_l, P.D, J2, mats, phi)
    p = pressure_from_energy(phi, terms, rho_e, mats)
    c, Gmix = sound_speed(phi, rho_l, terms, p, rho, mats)
    P.V, P.H, P.J2, P.p, P.c, P.Gmix = V, H, J2, p, c, Gmix
    P.sigma = stress(phi, p, Gmix, H)
    P.X = U[L.X]
    P.rho_e = rho_e
    return P


def face_state(phi, rho_l, eps, D, u, p, H, mats):
    """Conserved-side quantities of a reconstructed face state: mixture
    density, total energy density, stress and sound speed."""
    J2 = J2_of(H)
    terms = material_terms(rho_l, D, J2, mats, phi)
    rho = np.sum(phi * rho_l, axis=0)
    rho_e = energy_from_pressure(phi, terms, p, mats)
    rhoE = rho_e + 0.5 * rho * np.sum(u * u, axis=0)
    c, Gmix = sound_speed(phi, rho_l, terms, p, rho, mats)
    sig = stress(phi, p, Gmix, H)
    return rho, rhoE, sig, c, Gmix

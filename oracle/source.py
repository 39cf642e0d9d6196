"""Per-cell source step -- oracle, FP64.

Applied once per time step after the three SSP-RK3 stages (Lie splitting;
the paper is silent on the splitting).  Readings:

  * perturbation (Section 2.4, 3.2.2): phi = phi0(X) by multilinear
    interpolation of the cell-centred initial field at the cell's Lagrangian
    coordinates, X clamped to the span of the initial cell centres.
  * plasticity (Section 2.1 plastic source, deferred to earlier work; the
    perturbed yield of Section 2.4): instantaneous radial return of the
    deviatoric Hencky strain to the perturbed yield surface.  The mixture
    yield is sum phi_l (1-D_l) phi sigma_Y,l and the mixture modulus
    sum phi_l (1-D_l) G~_l, so J_max = Y_mix / (sqrt(6) G_mix); for one solid
    this is phi sigma_Y / (sqrt(6) G~), the effective-stress form.  The yield
    is constant (sigma_Y) and drops to zero once D >= D_crit (Section 3.1,
    second healing remark).  Delta eps_p = sqrt(2/3) (J - J_max).  Trace
    solids (volume fraction below the mixture's trace threshold) have no
    shear stiffness and take no part in the sums; a cell whose mixture
    modulus is zero carries no elastic distortion (Vbar is reset to the
    identity, the stress does not depend on it) and does no plastic work
    (Delta eps_p = 0, so no damage either).  A trace solid in a cell that
    another solid stiffens takes no share of the increment either: its
    plastic strain and damage stand.
  * damage (Section 2.2 Bonora rate with the Pirondi-Bonora gate, Section 3.1
    RK4): gate frozen at the start of the step (p < p_gate, eps_p^n above the
    triaxiality-dependent threshold, Delta eps_p > 0, D < D_crit); triaxiality
    from the hydrostatic pressure and the nominal equivalent stress at yield
    (1-D) phi sigma_Y, frozen over the step; classical RK4 in eps_p from
    eps_p^n to eps_p^n + Delta eps_p (eps_p linear in time over the step),
    every stage argument and the result clamped to [0, D_crit].
  * the simplified damage law of the U-Nb ring (Section 4.3),
    dD/deps_p = Ddot0 (1 - D), has no gate: it runs with the same RK4 on
    any plastic increment of a live solid below D_crit.
  * Vbar is rebuilt as the symmetric unimodular stretch Q exp(h) Q^T.
  * Total energy is unchanged, so the dissipated elastic energy becomes heat.
"""
import numpy as np

from .closures import (solid_shear_modulus, triaxiality, eps_threshold,
                       bonora_dD_deps, is_critical, jc_active, jc_flow_stress,
                       temperature)
from .scheme import _critical, _stress_band
from .kinematics import hencky, stretch_from_log
from .mixture import cons_to_prim, closure_density, PHI_TRACE, material_terms


def phi0_at(X, phi0, geom):
    """Multilinear interpolation of phi0 (nz, ny, nx) at coordinates
    X (d, ...) (Section 3.2.2: the initial field is interpolated at the
    evolved Lagrangian coordinates).  Written as nested linear
    interpolations a + t (b - a), x first, so a constant field is returned
    exactly."""
    dim = geom.dim
    base, wts = [], []
    for k in range(dim):
        nk = geom.n[k]
        s = (X[k] - (geom.lo[k] + 0.5 * geom.dx[k])) / geom.dx[k]
        s = np.clip(s, 0.0, nk - 1.0)
        i0 = np.minimum(np.floor(s), max(nk - 2, 0)).astype(np.int64)
        base.append(i0)
        wts.append(s - i0)

    def corner(bits):
        idx = [np.zeros(X.shape[1:], dtype=np.int64) for _ in range(3)]
        for k in range(dim):
            idx[k] = np.minimum(base[k] + bits[k], geom.n[k] - 1)
        return phi0[idx[2], idx[1], idx[0]]

    def lerp(a, b, t):
        return a + t * (b - a)

    if dim == 1:
        return lerp(corner((0,)), corner((1,)), wts[0])
    if dim == 2:
        f0 = lerp(corner((0, 0)), corner((1, 0)), wts[0])
        f1 = lerp(corner((0, 1)), corner((1, 1)), wts[0])
        return lerp(f0, f1, wts[1])
    g = []
    for bz in (0, 1):
        f0 = lerp(corner((0, 0, bz)), corner((1, 0, bz)), wts[0])
        f1 = lerp(corner((0, 1, bz)), corner((1, 1, bz)), wts[0])
        g.append(lerp(f0, f1, wts[1]))
    return lerp(g[0], g[1], wts[2])


def simplified_law(m):
    """Whether a solid takes the simplified damage law of the U-Nb ring
    (Section 4.3): dD/dt = Ddot0 (1 - D) deps_p/dt, Ddot0 given."""
    return m.get("Ddot0", 0.0) > 0.0


def damage_rk4(D, eps0, deps, R, m):
    """Classical RK4 for dD/d(eps_p) from eps0 over deps, clamped: the
    Bonora rate, or Ddot0 (1 - D) for the simplified law (zero once
    critical, like the Bonora rate)."""
    Dc = m["D_crit"]

    def f(Dv, e):
        if simplified_law(m):
            return np.where(Dv >= Dc, 0.0, m["Ddot0"] * (1.0 - Dv))
        return bonora_dD_deps(Dv, e, R, m)

    def cl(v):
        return np.clip(v, 0.0, Dc)

    h = deps
    k1 = f(D, eps0)
    k2 = f(cl(D + 0.5 * h * k1), eps0 + 0.5 * h)
    k3 = f(cl(D + 0.5 * h * k2), eps0 + 0.5 * h)
    k4 = f(cl(D + h * k3), eps0 + h)
    return cl(D + h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4))


# bisection steps of the Johnson-Cook return: each halves the bracket
# [0, sqrt(2/3) J], so 200 of them reach the double-precision root
JC_BISECTIONS = 200


def _mixture_yield(P, mats, solids, pert, opts, dgam, dt, temps):
    """Y_mix(Delta eps_p) = sum over live solids of
    phi_l (1 - D_l) phi0 sigma_Y,l(eps_l + Delta, Delta/dt, T_l), zero for a
    critical solid (the yield vanishes once D >= D_crit)."""
    Y = np.zeros_like(dgam)
    for l in solids:
        m = mats[l]
        live = P.phi[l] >= PHI_TRACE
        ok = live & ~_critical(P.D[l], m, opts)
        rate = dgam / dt if dt is not None and dt > 0 else np.zeros_like(dgam)
        sy = jc_flow_stress(P.eps[l] + dgam, rate, temps[l], m)
        Y = Y + np.where(ok, P.phi[l] * (1.0 - P.D[l]) * pert * sy, 0.0)
    return Y


def source_step(U, phi0, geom, layout, opts, dt=None):
    """Plastic return, damage and Vbar re-symmetrisation on U (in place).
    dt, the step's time step, sets the plastic strain rate of a
    rate-dependent yield (Johnson-Cook c3); without it the rate term is
    off."""
    L = layout
    mats = L.mats
    P = cons_to_prim(U, L)
    pert = phi0_at(P.X, phi0, geom)
    _, h, Q = hencky(P.V)
    J = np.sqrt(np.sum(h * h, axis=0))
    Gmix = np.zeros_like(J)
    for l in L.solids:
        m = mats[l]
        live = P.phi[l] >= PHI_TRACE
        w = 1.0 - P.D[l]
        Gt = solid_shear_modulus(P.rho_l[l], m)
        Gmix = Gmix + np.where(live, P.phi[l] * w * Gt, 0.0)
    pos = Gmix > 0
    # temperatures of the state entering the return, frozen over it
    terms = material_terms(P.rho_l, P.D, P.J2, mats, P.phi)
    temps = {l: temperature(P.p, terms[l][1], P.rho_l[l], mats[l])
             for l in L.solids}
    zero = np.zeros_like(J)
    Y0 = _mixture_yield(P, mats, L.solids, pert, opts, zero, dt, temps)
    yielding = pos & (np.sqrt(6.0) * Gmix * J > Y0)
    dmax = np.sqrt(2.0 / 3.0) * J
    if any(jc_active(mats[l]) for l in L.solids):
        # yield rising with Delta (hardening, rate): the residual
        # f(Delta) = sqrt6 G (J - sqrt(3/2) Delta) - Y_mix(Delta) falls from
        # f(0) > 0 to f(sqrt(2/3) J) = -Y_mix <= 0; bisect for its root
        lo = np.zeros_like(J)
        hi = np.where(yielding, dmax, 0.0)
        for _ in range(JC_BISECTIONS):
            mid = 0.5 * (lo + hi)
            f = (np.sqrt(6.0) * Gmix * (J - np.sqrt(1.5) * mid)
                 - _mixture_yield(P, mats, L.solids, pert, opts, mid, dt, temps))
            lo = np.where(f > 0.0, mid, lo)
            hi = np.where(f > 0.0, hi, mid)
        deps = np.where(yielding, 0.5 * (lo + hi), 0.0)
        Jnew = J - np.sqrt(1.5) * deps
    else:
        Jmax = np.where(pos, Y0 / (np.sqrt(6.0) * np.where(pos, Gmix, 1.0)), 0.0)
        deps = np.where(yielding, np.sqrt(2.0 / 3.0) * (J - Jmax), 0.0)
        Jnew = Jmax
    # no stiffness: the distortion is dropped (no plastic work)
    yielding = yielding | (~pos & (J > 0.0))
    Jnew = np.where(pos, Jnew, 0.0)
    scale = np.where(yielding, Jnew / np.where(yielding, J, 1.0), 1.0)
    Vn = stretch_from_log(h * scale[None], Q)
    for q, (i, j) in enumerate(L.vcomps):
        U[L.vbar[q]] = Vn[i, j]
    for l in L.solids:
        m = mats[l]
        mass = U[L.mass[l]]
        eps_n = P.eps[l]
        D_n = P.D[l]
        # a trace solid does no plastic work: its histories stand
        dl = np.where(P.phi[l] >= PHI_TRACE, deps, 0.0)
        rate = dl / dt if dt is not None and dt > 0 else np.zeros_like(dl)
        sig_eq = (1.0 - D_n) * pert * jc_flow_stress(eps_n + dl, rate, temps[l], m)
        # the simplified law has no gate: damage grows with any plastic
        # increment of a live, not yet critical solid
        open_p = True if simplified_law(m) else (P.p < m["p_gate"] - _stress_band(m, opts))
        gate = open_p & (dl > 0) & ~_critical(D_n, m, opts)
        ok = sig_eq > 0
        R = triaxiality(P.p, np.where(ok, sig_eq, 1.0),
                        closure_density(P.phi[l], P.rho_l[l], m), m)
        R = np.where(ok, R, 1.0)
        if not simplified_law(m):
            thr = eps_threshold(R, m)
            gate = gate & ((eps_n > thr) | ~ok)
        Dnew = D_n.copy()
        # the simplified law needs no triaxiality: it integrates wherever
        # the gate is open
        g1 = gate & (ok | simplified_law(m))
        if np.any(g1):
            Dnew[g1] = damage_rk4(D_n[g1], eps_n[g1], dl[g1], R[g1], m)
        Dnew[gate & ~ok & (not simplified_law(m))] = m["D_crit"]
        U[L.eps[l]] = mass * (eps_n + dl)
        U[L.dmg[l]] = mass * Dnew
    return U

"""Hyperbolic update -- oracle, FP64, vectorised over cells and faces.

The base finite-volume scheme is deferred by the paper to earlier work
(Section 3, first paragraph).  Readings:

  * reconstruction: piecewise-linear MUSCL of the primitives
    (phi_l, rho_l, eps_p, D, u, p, dev H, Vbar) with the van Leer limiter,
    slope 2ab/(a+b) if ab > 0 else 0; two ghost layers.  dev H is taken at
    cell centres and reconstructed, its trace removed again at the face.
  * interface sharpening (named by the paper for its ring): with a THINC
    steepness beta > 0 the volume fractions take the THINC face values of
    Xiao, Honma and Kono (2005) instead of MUSCL in cells where they are
    monotone (see thinc_faces); beta = 0 (the default) leaves MUSCL.
  * Lagrangian coordinates: third-order upwind WENO (Section 3.2.1) with
    Jiang-Shu weights, smoothness floor eps_w = weno_eps * L^2 with L
    the domain extent along the sweep (the paper gives no value).
  * flux: HLLC with Davis wave speeds for the conserved equations
    (phasic mass and history, momentum, energy, Section 2.1) with the
    contact's tangential velocity and traction resolved by linearised shear
    waves (see hllc), the Godunov face velocity for the non-conservative
    terms and upwinded face values of phi_l, X and Vbar.
  * void-opening modifier (Section 3.1): a face opens when either
    neighbouring cell is critically damaged and the sum of the two cell-centre
    normal stresses along the sweep is tensile, while the two one-sided
    velocities separate (u*_L <= u*_R).  An opened face transmits no
    traction: each side sees its own one-sided free-surface velocity
    u* = u_n -/+ sigma_nn/(rho c); a side whose u* points through the face
    carries its material (conserved variables and volume fractions) into the
    neighbour, otherwise void enters it; X and Vbar use each side's own
    centre values, so opening does not change them.  (The paper's modifier
    also separates material interfaces in tension; judged along the sweep
    direction that would cut tensile solids along their surface, so this
    rule does not open interfaces: that needs an interface-normal
    criterion.)
  * free-surface boundaries behave like an opened face towards void; the
    material leaves through it when u* points outward.
  * time integration: SSP-RK3 (Shu-Osher) for all transported fields,
    unsplit (the X update of Section 3.2.1 runs concurrently, with the same
    stages).  Volume fractions are clamped to [phi_floor, 1] after each stage.
Parity of the flux scheme is unpinned against the paper beyond the invariants
and exact solutions checked by the tests (uniform states, conservation,
linear X transport, mirror symmetry, elastic wave speeds, convergence order,
free-surface reflection, the shear Riemann problem, and the opened face's
zero traction between separating critical halves).
"""
import numpy as np

from .layout import hencky_comps
from .closures import is_critical, stress_band
from .mixture import cons_to_prim, face_state

AX = {0: -1, 1: -2, 2: -3}          # x, y, z -> axis from the end

# Contact and face speeds below this fraction of the largest signal speed
# count as stationary: every upwind choice made on their sign takes the mean
# of the two sides.  Without shear waves in the approximate solver the star
# fluxes of the two sides differ by the jump in tangential traction when the
# contact speed passes zero, and the face stretch differs when the face speed
# does, so the choice must not hinge on the sign of a rounding residue (as on
# a symmetry plane).
TIE_REL = 1.0e-12


class Geometry:
    def __init__(self, dim, n, lo, hi, bc):
        self.dim = dim
        self.n = tuple(n)
        self.lo = tuple(lo)
        self.hi = tuple(hi)
        self.bc = tuple(tuple(b) for b in bc)
        self.dx = tuple((hi[k] - lo[k]) / n[k] for k in range(3))
        self.gw = [2 if k < dim else 0 for k in range(3)]
        for k in range(dim):
            lo_b, hi_b = self.bc[k]
            if (lo_b == "periodic") != (hi_b == "periodic"):
                raise ValueError("periodic boundaries must be paired")
            for b in (lo_b, hi_b):
                if b not in ("transmissive", "free", "periodic"):
                    raise ValueError(f"unsupported boundary {b}")


def pad(U, geom):
    """Two ghost layers per active direction: zero-gradient copies for
    transmissive and free-surface sides, wrap-around for periodic ones."""
    out = U
    for k in range(geom.dim):
        ax = out.ndim + AX[k]
        pw = [(0, 0)] * out.ndim
        pw[ax] = (2, 2)
        mode = "wrap" if geom.bc[k][0] == "periodic" else "edge"
        out = np.pad(out, pw, mode=mode)
    return out


def _sweep_view(arr, a, geom):
    """Crop the transverse active axes to the interior and move the sweep
    axis `a` last."""
    sl = [slice(None)] * arr.ndim
    for k in range(3):
        if k != a and geom.gw[k] > 0:
            sl[arr.ndim + AX[k]] = slice(geom.gw[k], -geom.gw[k])
    v = arr[tuple(sl)]
    return np.moveaxis(v, arr.ndim + AX[a], -1)


def _unsweep(arr, a):
    return np.moveaxis(arr, -1, arr.ndim + AX[a])


def van_leer(dm, dp):
    """van Leer limited slope: 2ab/(a+b) where ab > 0, else 0."""
    prod = dm * dp
    den = np.where(prod > 0, dm + dp, 1.0)
    return np.where(prod > 0, 2.0 * prod / den, 0.0)


def weno3_faces(q, eps):
    """Third-order WENO face values from the left and from the right at faces
    f = 0..n of a padded line q[..., 0..n+3] (cells f+1 | f+2 meet at f)."""
    qm, q0, q1, q2 = q[..., :-3], q[..., 1:-2], q[..., 2:-1], q[..., 3:]
    # from the left (upwind cell f+1 = q0)
    p0 = -0.5 * qm + 1.5 * q0
    p1 = 0.5 * q0 + 0.5 * q1
    b0 = (q0 - qm) ** 2
    b1 = (q1 - q0) ** 2
    a0 = (1.0 / 3.0) / (eps + b0) ** 2
    a1 = (2.0 / 3.0) / (eps + b1) ** 2
    left = (a0 * p0 + a1 * p1) / (a0 + a1)
    # from the right (upwind cell f+2 = q1), mirror image
    r0 = -0.5 * q2 + 1.5 * q1
    r1 = 0.5 * q1 + 0.5 * q0
    c0 = (q1 - q2) ** 2
    c1 = (q0 - q1) ** 2
    e0 = (1.0 / 3.0) / (eps + c0) ** 2
    e1 = (2.0 / 3.0) / (eps + c1) ** 2
    right = (e0 * r0 + e1 * r1) / (e0 + e1)
    return left, right


# cells where the THINC profile is used: the normalised cell value C lies
# in (THINC_EPS, 1 - THINC_EPS) of the span of its two neighbours
THINC_EPS = 1.0e-6


def _thinc_cell(qm, q0, q1, beta):
    """THINC reconstruction in one cell (Xiao, Honma and Kono 2005): the
    profile q_min + (dq/2)(1 + theta tanh(beta (x - x_c))) on the unit cell,
    with q_min, dq the minimum and span of the neighbours qm, q1, theta the
    sign of q1 - qm, and x_c set so that the cell average is q0.  In closed
    form, with C = (q0 - q_min)/dq, B = exp(theta beta (2C - 1)) and
    A = (B / cosh(beta) - 1) / tanh(beta), the value at the cell's lower
    face is q_min + (dq/2)(1 + theta A) and at its upper face
    q_min + (dq/2)(1 + theta (tanh(beta) + A) / (1 + A tanh(beta))).
    Returns (lower, upper, mask) with mask the cells it applies to (q0
    strictly monotone between its neighbours, C inside the THINC_EPS band)."""
    qmin = np.minimum(qm, q1)
    dq = np.abs(q1 - qm)
    mono = (q1 - q0) * (q0 - qm) > 0.0
    safe = np.where(dq > 0.0, dq, 1.0)
    C = (q0 - qmin) / safe
    use = mono & (C > THINC_EPS) & (C < 1.0 - THINC_EPS)
    theta = np.where(q1 >= qm, 1.0, -1.0)
    B = np.exp(theta * beta * (2.0 * np.where(use, C, 0.5) - 1.0))
    tb = np.tanh(beta)
    A = (B / np.cosh(beta) - 1.0) / tb
    lower = qmin + 0.5 * dq * (1.0 + theta * A)
    upper = qmin + 0.5 * dq * (1.0 + theta * (tb + A) / (1.0 + A * tb))
    return lower, upper, use


def thinc_faces(q, beta):
    """THINC face states of a padded row q (..., n+4) for the n+1 faces:
    (left, right, use_left, use_right), the left state from the upper face
    of the cell below each face and the right state from the lower face of
    the cell above."""
    _, upper, uL = _thinc_cell(q[..., :-3], q[..., 1:-2], q[..., 2:-1], beta)
    lower, _, uR = _thinc_cell(q[..., 1:-2], q[..., 2:-1], q[..., 3:], beta)
    return upper, lower, uL, uR


def _critical(D, m, opts):
    tol = getattr(opts, "crit_rel_tol", None)
    return is_critical(D, m) if tol is None else is_critical(D, m, tol)


def _stress_band(m, opts):
    tol = getattr(opts, "crit_rel_tol", None)
    return stress_band(m) if tol is None else stress_band(m, tol)


def _pick(sel_pos, sel_neg, vL, vR):
    """Upwind choice: vL where sel_pos, vR where sel_neg, mean otherwise."""
    return np.where(sel_pos, vL, np.where(sel_neg, vR, 0.5 * (vL + vR)))


def _rec_rows(P, layout):
    """Cell-centre primitive rows that are reconstructed, with names."""
    L = layout
    rows, names = [], []
    for l in range(L.nm):
        rows.append(P.phi[l]); names.append(("phi", l))
    for l in range(L.nm):
        rows.append(P.rho_l[l]); names.append(("rho", l))
    for l in L.solids:
        rows.append(P.eps[l]); names.append(("eps", l))
        rows.append(P.D[l]); names.append(("D", l))
    for k in range(L.dim):
        rows.append(P.u[k]); names.append(("u", k))
    rows.append(P.p); names.append(("p", 0))
    for (i, j) in hencky_comps(L.dim):
        rows.append(P.H[i, j]); names.append(("H", (i, j)))
    for k, (i, j) in enumerate(L.vcomps):
        rows.append(P.V[i, j]); names.append(("V", (i, j)))
    return np.stack(rows), names


def _unpack(W, names, layout, shape):
    L = layout
    phi = np.zeros((L.nm,) + shape)
    rho = np.zeros((L.nm,) + shape)
    eps, D = {}, {}
    u = np.zeros((3,) + shape)
    H = np.zeros((3, 3) + shape)
    V = np.zeros((3, 3) + shape)
    p = None
    for r, (kind, key) in enumerate(names):
        if kind == "phi":
            phi[key] = W[r]
        elif kind == "rho":
            rho[key] = W[r]
        elif kind == "eps":
            eps[key] = W[r]
        elif kind == "D":
            D[key] = W[r]
        elif kind == "u":
            u[key] = W[r]
        elif kind == "p":
            p = W[r]
        elif kind == "H":
            i, j = key
            H[i, j] = W[r]
            H[j, i] = W[r]
        elif kind == "V":
            i, j = key
            V[i, j] = W[r]
    tr = (H[0, 0] + H[1, 1] + H[2, 2]) / 3.0
    for i in range(3):
        H[i, i] = H[i, i] - tr
    return phi, rho, eps, D, u, p, H, V


def _face_conserved(phi, rho_l, eps, D, u, rho, rhoE, layout):
    L = layout
    rows = [phi[l] * rho_l[l] for l in range(L.nm)]
    for l in L.solids:
        rows.append(phi[l] * rho_l[l] * eps[l])
        rows.append(phi[l] * rho_l[l] * D[l])
    for k in range(L.dim):
        rows.append(rho * u[k])
    rows.append(rhoE)
    return np.stack(rows)


def _phys_flux(Uc, un, u, t, layout):
    """Physical flux U u_n - (0, 0, sigma n, u . sigma n) (Section 2.1)."""
    L = layout
    F = Uc * un[None]
    base = L.nm + 2 * len(L.solids)
    for k in range(L.dim):
        F[base + k] = F[base + k] - t[k]
    F[-1] = F[-1] - np.sum(u * t, axis=0)
    return F


def hllc(sL, sR, a, layout):
    """Approximate Riemann flux with the contact's tangential state resolved.

    HLLC (Davis speeds S_L, S_R, contact speed S*) carries the normal
    structure: mass, histories, normal momentum and the normal-traction part
    of the energy.  A plain HLLC has no shear waves, so its star fluxes keep
    each side's own tangential traction and upwind it by the contact speed,
    a one-sided difference that lets shear waves grow.  Here the linearised
    shear waves on either side of the contact (impedance Z = sqrt(G rho))
    fix a common tangential velocity and traction at the contact,
      u_t** = (Z_L u_tL + Z_R u_tR + t_tR - t_tL) / (Z_L + Z_R),
      t_t** = t_tL + Z_L (u_t** - u_tL),
    (free slip, t_t** = 0, against a fluid) and the star-region flux is
      mass/history: chi_K U_K S*,  normal momentum: rho*_K S*^2 - t_n*,
      tangential momentum: rho*_K u_t** S* - t_t**,
      energy: E**_K S* - S* t_n* - u_t** . t_t**,
    with E**_K the HLLC star energy plus the kinetic-energy change of the
    tangential velocity.  The flux is consistent (F(U,U) = F(U)) and
    continuous through S* = 0.  Returns the flux, the face normal velocity,
    S*, the tie band and the face tangential velocity vector."""
    L = layout
    unL, unR = sL["u"][a], sR["u"][a]
    tnL, tnR = sL["t"][a], sR["t"][a]
    rL, rR = sL["rho"], sR["rho"]
    SL = np.minimum(unL - sL["c"], unR - sR["c"])
    SR = np.maximum(unL + sL["c"], unR + sR["c"])
    # grouped so that a mirrored pair of states gives exactly -S*
    num = (tnL - tnR) + (rL * unL * (SL - unL) - rR * unR * (SR - unR))
    den = rL * (SL - unL) - rR * (SR - unR)
    Ss = num / den
    tie = TIE_REL * np.maximum(np.abs(SL), np.abs(SR))
    FL = _phys_flux(sL["Uc"], unL, sL["u"], sL["t"], L)
    FR = _phys_flux(sR["Uc"], unR, sR["u"], sR["t"], L)
    tang = [k for k in range(3) if k != a]
    ZL = np.sqrt(sL["G"] * rL)
    ZR = np.sqrt(sR["G"] * rR)
    Zs = ZL + ZR
    pos = Zs > 0
    Zsafe = np.where(pos, Zs, 1.0)
    ut2 = np.zeros_like(sL["u"])
    tt2 = np.zeros_like(sL["u"])
    for k in tang:
        up = _pick(Ss > tie, Ss < -tie, sL["u"][k], sR["u"][k])
        ut2[k] = np.where(pos, (ZL * sL["u"][k] + ZR * sR["u"][k]
                                + (sR["t"][k] - sL["t"][k])) / Zsafe, up)
        tt2[k] = np.where(pos, sL["t"][k] + ZL * (ut2[k] - sL["u"][k]), 0.0)
    tn_star = 0.5 * ((tnL - rL * (SL - unL) * (Ss - unL))
                     + (tnR - rR * (SR - unR) * (Ss - unR)))
    work = sum(ut2[k] * tt2[k] for k in tang)
    base = L.nm + 2 * len(L.solids)

    def star(s, S, un, tn):
        chi = (S - un) / (S - Ss)
        rs = chi * s["rho"]
        Es = chi * (s["rhoE"] + (Ss - un) * (s["rho"] * Ss - tn / (S - un)))
        Ess = Es + 0.5 * rs * sum(ut2[k] ** 2 - s["u"][k] ** 2 for k in tang)
        F = s["Uc"] * (chi * Ss)[None]
        for k in range(L.dim):
            if k == a:
                F[base + k] = rs * Ss * Ss - tn_star
            else:
                F[base + k] = rs * ut2[k] * Ss - tt2[k]
        F[-1] = Ess * Ss - Ss * tn_star - work
        return F

    FsL = star(sL, SL, unL, tnL)
    FsR = star(sR, SR, unR, tnR)
    Fstar = np.where(Ss[None] > tie, FsL,
                     np.where(Ss[None] < -tie, FsR, 0.5 * (FsL + FsR)))
    F = np.where(SL[None] >= 0, FL, np.where(SR[None] <= 0, FR, Fstar))
    uface = np.where(SL > 0, unL, np.where(SR < 0, unR, Ss))
    uvec = np.where(SL[None] > 0, sL["u"], np.where(SR[None] < 0, sR["u"], ut2))
    uvec[a] = uface
    return F, uface, Ss, tie, uvec


def _side(W, names, layout, shape, mats):
    phi, rho_l, eps, D, u, p, H, V = _unpack(W, names, layout, shape)
    rho, rhoE, sig, c, G = face_state(phi, rho_l, eps, D, u, p, H, mats)
    Uc = _face_conserved(phi, rho_l, eps, D, u, rho, rhoE, layout)
    return dict(phi=phi, rho_l=rho_l, u=u, p=p, H=H, V=V, rho=rho,
                rhoE=rhoE, sig=sig, c=c, G=G, Uc=Uc)


def _vflux(V, uvec, a, comps):
    """Vbar flux along direction a: V_ij u_a - V_aj u_i (Section 2.1)."""
    return np.stack([V[i, j] * uvec[a] - V[a, j] * uvec[i] for (i, j) in comps])


def rhs(U, geom, layout, opts):
    """L(U) of the semi-discrete system and the outward boundary fluxes.

    Returns (dU (S, nz, ny, nx), bflux) where bflux[(k, side)] is the
    outward conserved-flux array (n_flux, transverse...) on boundary side
    `side` of direction k (absent for periodic sides)."""
    L = layout
    mats = L.mats
    dim = L.dim
    Up = pad(U, geom)
    P = cons_to_prim(Up, L)
    R, names = _rec_rows(P, L)
    dU = np.zeros_like(U)
    bflux = {}
    crit = np.zeros(P.p.shape, dtype=bool)
    tens_band = 0.0
    for l in L.solids:
        crit |= _critical(P.D[l], mats[l], opts)
        tens_band = max(tens_band, _stress_band(mats[l], opts))
    for a in range(dim):
        dxa = geom.dx[a]
        n = geom.n[a]
        Rs = _sweep_view(R, a, geom)                 # (nR, T.., n+4)
        s = van_leer(Rs[..., 1:-1] - Rs[..., :-2], Rs[..., 2:] - Rs[..., 1:-1])
        # s[..., m] is the slope at padded cell m+1, m = 0..n+1
        WL = Rs[..., 1:-2] + 0.5 * s[..., :-1]        # cells f+1, f = 0..n
        WR = Rs[..., 2:-1] - 0.5 * s[..., 1:]         # cells f+2
        beta = getattr(opts, "thinc_beta", 0.0)
        if beta > 0.0:
            for r, (kind, _) in enumerate(names):
                if kind != "phi":
                    continue
                tl, tr, ul, ur = thinc_faces(Rs[r], beta)
                WL[r] = np.where(ul, tl, WL[r])
                WR[r] = np.where(ur, tr, WR[r])
        fshape = WL.shape[1:]
        sL = _side(WL, names, L, fshape, mats)
        sR = _side(WR, names, L, fshape, mats)
        for sd in (sL, sR):
            sd["t"] = sd["sig"][:, a]
        F, uface, Ss, tie, uvec = hllc(sL, sR, a, L)
        up, un_ = uface > tie, uface < -tie
        phi_f = _pick(up, un_, sL["phi"], sR["phi"])
        V_f = _pick(up, un_, sL["V"], sR["V"])
        Xs = _sweep_view(P.X, a, geom)
        ext = geom.hi[a] - geom.lo[a]
        XfL, XfR = weno3_faces(Xs, opts.weno_eps * ext * ext)
        X_f = _pick(up, un_, XfL, XfR)
        # per-side (as seen from the left / right cell) geometric fluxes
        velL = uface.copy()
        velR = uface.copy()
        phiL = phi_f * uface[None]
        phiR = phiL.copy()
        XL = X_f * uface[None]
        XR = XL.copy()
        VfL = _vflux(V_f, uvec, a, L.vcomps)
        VfR = VfL.copy()
        rowL = V_f[a].copy()
        rowR = rowL.copy()
        # centre values of the two neighbours of each face
        cen = {}
        for key, arr in (("V", P.V), ("X", P.X), ("u", P.u),
                         ("sig", P.sigma[a, a]), ("crit", crit)):
            v = _sweep_view(arr, a, geom)
            cen[key] = (v[..., 1:-2], v[..., 2:-1])
        def closed_side(K, ustar, mask):
            """Overwrite side K's geometric fluxes with its own centre values
            and one-sided velocity where `mask`."""
            Vc, Xc, uc = cen["V"][K], cen["X"][K], cen["u"][K].copy()
            uc[a] = ustar
            vf = _vflux(Vc, uc, a, L.vcomps)
            xf = Xc * ustar[None]
            m = mask
            if K == 0:
                velL[m] = ustar[m]
                phiL[:, m] = 0.0
                XL[:, m] = xf[:, m]
                VfL[:, m] = vf[:, m]
                rowL[:, m] = Vc[a][:, m]
            else:
                velR[m] = ustar[m]
                phiR[:, m] = 0.0
                XR[:, m] = xf[:, m]
                VfR[:, m] = vf[:, m]
                rowR[:, m] = Vc[a][:, m]

        ustarL = sL["u"][a] - sL["t"][a] / (sL["rho"] * sL["c"])
        ustarR = sR["u"][a] + sR["t"][a] / (sR["rho"] * sR["c"])
        # the two free surfaces must separate (approaching sides are closing
        # the void and are in contact again)
        opened = ((cen["crit"][0] | cen["crit"][1])
                  & (cen["sig"][0] + cen["sig"][1] > tens_band)
                  & (ustarL <= ustarR))
        # boundary faces are handled below, never by the damage predicate
        if geom.bc[a][0] != "periodic":
            opened[..., 0] = False
            opened[..., -1] = False
        # an opened face is a free surface seen from each side: a side whose
        # one-sided velocity points through the face carries its material
        # (no traction) into the neighbour, otherwise void enters it
        outL = opened & (ustarL > 0)
        outR = opened & (ustarR < 0)
        Fo = (np.where(outL[None], sL["Uc"] * ustarL[None], 0.0)
              + np.where(outR[None], sR["Uc"] * ustarR[None], 0.0))
        F[:, opened] = Fo[:, opened]
        closed_side(0, ustarL, opened)
        closed_side(1, ustarR, opened)
        Po = (np.where(outL[None], sL["phi"] * ustarL[None], 0.0)
              + np.where(outR[None], sR["phi"] * ustarR[None], 0.0))
        phiL[:, opened] = Po[:, opened]
        phiR[:, opened] = Po[:, opened]
        # free-surface boundaries
        for side in (0, 1):
            if geom.bc[a][side] != "free":
                continue
            fi = 0 if side == 0 else n
            K = 1 if side == 0 else 0             # interior side
            sK = sR if K == 1 else sL
            ust = (ustarR if K == 1 else ustarL)[..., fi]
            outward = ust < 0 if side == 0 else ust > 0
            m = np.zeros(opened.shape, dtype=bool)
            # inflow of void: closed face
            m[..., fi] = ~outward
            F[:, m] = 0.0
            closed_side(K, ustarR if K == 1 else ustarL, m)
            # outflow of material at the free-surface velocity, no traction
            mo = np.zeros(opened.shape, dtype=bool)
            mo[..., fi] = outward
            us = ustarR if K == 1 else ustarL
            Fo = sK["Uc"] * us[None]
            F[:, mo] = Fo[:, mo]
            ufo = sK["u"].copy()
            ufo[a] = us
            XK = XfR if K == 1 else XfL
            vfo = _vflux(sK["V"], ufo, a, L.vcomps)
            if K == 0:
                velL[mo] = us[mo]
                phiL[:, mo] = (sK["phi"] * us[None])[:, mo]
                XL[:, mo] = (XK * us[None])[:, mo]
                VfL[:, mo] = vfo[:, mo]
                rowL[:, mo] = sK["V"][a][:, mo]
            else:
                velR[mo] = us[mo]
                phiR[:, mo] = (sK["phi"] * us[None])[:, mo]
                XR[:, mo] = (XK * us[None])[:, mo]
                VfR[:, mo] = vfo[:, mo]
                rowR[:, mo] = sK["V"][a][:, mo]
        # outward boundary fluxes for the conservation totals
        for side in (0, 1):
            if geom.bc[a][side] == "periodic":
                continue
            bflux[(a, side)] = (-F[..., 0] if side == 0 else F[..., n]).copy()
        # cell updates (cells i = 0..n-1 between faces i and i+1)
        inv = 1.0 / dxa
        div = (velL[..., 1:] - velR[..., :-1]) * inv
        contrib = np.zeros((L.S,) + div.shape)
        for r, row in enumerate(L.flux_rows):
            contrib[row] = -(F[r][..., 1:] - F[r][..., :-1]) * inv
        Pc = {}
        for key, arr in (("phi", P.phi), ("X", P.X), ("V", P.V), ("u", P.u)):
            v = _sweep_view(arr, a, geom)
            Pc[key] = v[..., 2:-2]
        for l in range(L.nm):
            contrib[L.phi[l]] = (-(phiL[l][..., 1:] - phiR[l][..., :-1]) * inv
                                 + Pc["phi"][l] * div)
        for k in range(dim):
            contrib[L.X[k]] = (-(XL[k][..., 1:] - XR[k][..., :-1]) * inv
                               + Pc["X"][k] * div)
        for q, (i, j) in enumerate(L.vcomps):
            beta_j = (rowL[j][..., 1:] - rowR[j][..., :-1]) * inv
            contrib[L.vbar[q]] = (-(VfL[q][..., 1:] - VfR[q][..., :-1]) * inv
                                  + (2.0 / 3.0) * Pc["V"][i, j] * div
                                  - Pc["u"][i] * beta_j)
        dU += _unsweep(contrib, a)
    return dU, bflux


def clamp_phi(U, layout, opts):
    U[layout.phi] = np.clip(U[layout.phi], opts.phi_floor, 1.0)
    return U


def dt_inverse(U, geom, layout):
    """Largest sum over directions of (|u_d| + c) / dx_d (the CFL
    reduction); the time step is CFL / dt_inverse."""
    P = cons_to_prim(U, layout)
    s = np.zeros_like(P.p)
    for k in range(layout.dim):
        s = s + (np.abs(P.u[k]) + P.c) / geom.dx[k]
    return float(np.max(s))

"""Lagrangian seeding into void -- oracle, FP64 (Section 3.2.1, the seeding
routine that follows the Lagrangian-coordinate update).

Applied once per time step after the source step, to every cell whose void
fraction nu = 1 - sum phi_l exceeds a threshold.  Readings of what the
routine leaves open:

  * threshold: a run option (the paper names nu_Thresh without a value); the
    workloads that use the routine take 0.99, so only cells holding less
    than 1% material are reseeded;
  * normal: n = grad(nu) / |grad(nu)| from central differences of the void
    fraction (one-sided at a domain side), pointing from the material into
    the void; a cell with grad(nu) = 0 (no material nearby) is left alone;
  * probe: from the cell centre c towards the material, p = c - 1.5 h n,
    with h the smallest cell size of the active directions -- the only
    direction in which the interpolated coordinates belong to material;
  * interpolation: multilinear in the cell-centred X, p clamped to the span
    of the cell centres (the same interpolation as the perturbation field);
  * update: X_new = X(p) - (p - c), from the coordinates before any cell of
    this step was reseeded.
For coordinates that are linear in space (a body in rigid translation,
X = x - d) the new value is exact: X(p) - (p - c) = c - d.
"""
import numpy as np

from .mixture import cons_to_prim, material_terms, pressure_from_energy
from .source import phi0_at


def seed_void(U, geom, layout, nu_thresh):
    """Reseed the Lagrangian coordinates of void cells (in place)."""
    L = layout
    dim = geom.dim
    phi = U[L.phi]
    nu = 1.0 - np.clip(np.sum(phi, axis=0), 0.0, 1.0)
    shape = nu.shape
    grad = np.zeros((3,) + shape)
    for k in range(dim):
        ax = nu.ndim - 1 - k
        n = shape[ax]
        if n < 2:
            continue
        d = np.zeros(shape)
        idx = lambda s: tuple(s if a == ax else slice(None) for a in range(nu.ndim))
        d[idx(slice(1, -1))] = ((nu[idx(slice(2, None))] - nu[idx(slice(None, -2))])
                                / (2.0 * geom.dx[k]))
        d[idx(slice(0, 1))] = (nu[idx(slice(1, 2))] - nu[idx(slice(0, 1))]) / geom.dx[k]
        d[idx(slice(-1, None))] = (nu[idx(slice(-1, None))] - nu[idx(slice(-2, -1))]) / geom.dx[k]
        grad[k] = d
    norm = np.sqrt(np.sum(grad * grad, axis=0))
    mask = (nu > nu_thresh) & (norm > 0.0)
    if not np.any(mask):
        return U
    h = min(geom.dx[k] for k in range(dim))
    nrm = np.where(norm > 0.0, norm, 1.0)
    centres = []
    for k in range(3):
        ax = 2 - k
        c = geom.lo[k] + (np.arange(geom.n[k]) + 0.5) * geom.dx[k]
        sh = [1, 1, 1]
        sh[ax] = geom.n[k]
        centres.append(np.broadcast_to(c.reshape(sh), shape))
    p = np.stack([centres[k] - 1.5 * h * grad[k] / nrm if k < dim else centres[k]
                  for k in range(3)])
    X = U[L.X]
    newX = []
    for k in range(dim):
        Xi = phi0_at(p[:dim], X[k], geom)
        newX.append(Xi - (p[k] - centres[k]))
    for k in range(dim):
        U[L.X[k]] = np.where(mask, newX[k], X[k])
    return U


RELAX_ITERS = 64


def relax_void(U, geom, layout, nu_thresh, phi_floor):
    """Void cells give up their pressure (a reading of the void treatment
    around Section 3.2.1's seeding, one solid only): a cell with mass whose
    void fraction exceeds the seeding threshold holds a film of material with
    void on its free side, and void carries no stress.  The film's density
    moves to the first density, scanning up from rho0 / 2 over
    [rho0 / 2, 2 rho0], at which the material's own pressure at the cell's
    specific internal energy e = rho_e / mass changes sign: the equation of
    state of the film alone (volume fraction one, energy rho_l e per film
    volume), so the closures of a trace never enter.  Bisection, RELAX_ITERS
    halvings, on whether the pressure at the midpoint has the sign it has at
    the lower end; without a sign change the film takes 2 rho0.  The volume
    fraction follows as mass / density (clamped to [phi_floor, 1]); mass,
    momentum, energy and histories are unchanged.  Returns a new array."""
    L = layout
    if len(L.mats) != 1:
        return U
    phi = U[L.phi[0]]
    mass = U[L.mass[0]]
    mask = ((1.0 - np.clip(phi, 0.0, 1.0)) > nu_thresh) & (mass > 0.0)
    if not np.any(mask):
        return U
    P = cons_to_prim(U, L)
    ms = np.where(mask, mass, 1.0)
    e = P.rho_e / ms
    rho0 = L.mats[0]["rho0"]
    one = np.ones((1,) + mass.shape)

    def positive(rl):
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            terms = material_terms(rl[None], P.D, P.J2, L.mats, one)
            return pressure_from_energy(one, terms, rl * e, L.mats) > 0.0

    lo = np.full(mass.shape, 0.5 * rho0)
    hi = np.full(mass.shape, 2.0 * rho0)
    slo = positive(lo)
    for _ in range(RELAX_ITERS):
        mid = 0.5 * (lo + hi)
        same = positive(mid) == slo
        lo = np.where(same, mid, lo)
        hi = np.where(same, hi, mid)
    rs = 0.5 * (lo + hi)
    out = U.copy()
    out[L.phi[0]] = np.where(mask, np.clip(ms / rs, phi_floor, 1.0), phi)
    return out

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

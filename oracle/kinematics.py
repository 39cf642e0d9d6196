"""Kinematics of the unimodular stretch (Sections 2.1, 2.2) -- oracle, FP64.

Vbar may lose symmetry under transport (its evolution equation carries the
velocity gradient on the left only); the stress depends only on
Bbar = Vbar Vbar^T, so the Hencky strain is taken as H = 1/2 ln(Bbar), which
equals ln(Vbar) for symmetric Vbar (the deviatoric Hencky strain definition of
Section 2.2).  The trace is removed, which restores det Vbar = 1.
"""
import numpy as np


def full_vbar(vals, comps, shape):
    """Assemble a (3, 3, ...) tensor from the stored components (the
    components that are not stored are zero)."""
    V = np.zeros((3, 3) + shape)
    for k, (i, j) in enumerate(comps):
        V[i, j] = vals[k]
    return V


def _to_last(T):
    """(3, 3, ...) -> (..., 3, 3)."""
    return np.moveaxis(np.moveaxis(T, 0, -1), 0, -1)


def _from_last(T):
    return np.moveaxis(np.moveaxis(T, -1, 0), -1, 0)


def hencky(V):
    """Deviatoric Hencky strain of the stretch V (3, 3, ...):
    eigendecomposition of Bbar = V V^T, H = Q diag(ln(lambda)/2) Q^T, trace
    removed.  Returns (H (3,3,...), eigenvalue logs h (3,...) after trace
    removal, eigenvectors Q (..., 3, 3))."""
    Vl = _to_last(V)
    B = Vl @ np.swapaxes(Vl, -1, -2)
    lam, Q = np.linalg.eigh(B)
    h = 0.5 * np.log(lam)
    h = h - h.mean(axis=-1, keepdims=True)
    H = (Q * h[..., None, :]) @ np.swapaxes(Q, -1, -2)
    return _from_last(H), np.moveaxis(h, -1, 0), Q


def stretch_from_log(h, Q):
    """Symmetric stretch Q diag(exp(h)) Q^T from eigenvalue logs h (3, ...)
    and eigenvectors Q (..., 3, 3)."""
    hl = np.moveaxis(h, 0, -1)
    V = (Q * np.exp(hl)[..., None, :]) @ np.swapaxes(Q, -1, -2)
    return _from_last(V)


def J2_of(H):
    """Second invariant of shear strain J^2 = tr(H H^T) (Section 2.2)."""
    return np.sum(H * H, axis=(0, 1))

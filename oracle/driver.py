"""Imposed-velocity driver of the expanding ring -- oracle, FP64
(Section 4.3, the U-Nb ring driven by the velocity profile of a driver ring).

The paper imposes the profile through a rigid body pushing the specimen from
inside, until an arrestor at r_max.  The rigid body is not part of this
build; the reading here keeps its kinematics: a driver surface about the z
axis starts at the ring's inner radius r_in and moves outward with

  v_r(t) = v0 t/t0 (t < t0),  v0 + (v1 - v0)(t - t0)/(t1 - t0) (t0 <= t < t1),
  v1 afterwards,

R_d(t) = r_in + the integral of v_r, while R_d < r_max.  After each step
(time t at its end), every cell holding a live solid (a volume fraction
above the trace threshold) whose centre lies at a radius r <= R_d and moves
outward slower than v_r takes the radial speed v_r (its other velocity
components kept); the kinetic energy it gains is added to the total energy
(the driver's work).  d = (r_in, v0, v1, t0, t1, r_max); r_max = 0 is off.
"""
import numpy as np

from .mixture import PHI_TRACE


def driver_speed(d, t):
    if t < d[3]:
        return d[1] * t / d[3]
    if t < d[4]:
        return d[1] + (d[2] - d[1]) * (t - d[3]) / (d[4] - d[3])
    return d[2]


def driver_radius(d, t):
    """r_in plus the integral of driver_speed from 0 to t (piecewise
    quadratic)."""
    r_in, v0, v1, t0, t1 = d[0], d[1], d[2], d[3], d[4]
    if t < t0:
        return r_in + 0.5 * v0 * t * t / t0
    a = r_in + 0.5 * v0 * t0
    if t < t1:
        s = t - t0
        return a + v0 * s + 0.5 * (v1 - v0) * s * s / (t1 - t0)
    return a + 0.5 * (v0 + v1) * (t1 - t0) + v1 * (t - t1)


def apply_driver(U, geom, layout, d, t):
    """Apply the driver to the state U (in place) at time t."""
    if d is None or d[5] <= 0.0 or geom.dim < 2:
        return U
    Rd = driver_radius(d, t)
    if Rd >= d[5]:
        return U
    L = layout
    vr = driver_speed(d, t)
    shape = U.shape[1:]
    cx = geom.lo[0] + (np.arange(geom.n[0]) + 0.5) * geom.dx[0]
    cy = geom.lo[1] + (np.arange(geom.n[1]) + 0.5) * geom.dx[1]
    x = np.broadcast_to(cx[None, None, :], shape)
    y = np.broadcast_to(cy[None, :, None], shape)
    r = np.sqrt(x * x + y * y)
    live = np.zeros(shape, dtype=bool)
    for l in L.solids:
        live |= U[L.phi[l]] >= PHI_TRACE
    rho = np.sum(np.maximum(U[L.mass], 0.0), axis=0)
    u = [U[L.mom[k]] / rho for k in range(geom.dim)]
    rs = np.where(r > 0.0, r, 1.0)
    ur = (u[0] * x + u[1] * y) / rs
    m = live & (r > 0.0) & (r <= Rd) & (ur < vr)
    if not np.any(m):
        return U
    du = vr - ur
    ke0 = sum(uk * uk for uk in u)
    un = list(u)
    un[0] = u[0] + du * x / rs
    un[1] = u[1] + du * y / rs
    ke1 = sum(uk * uk for uk in un)
    for k in range(2):
        U[L.mom[k]] = np.where(m, rho * un[k], U[L.mom[k]])
    U[L.energy] = np.where(m, U[L.energy] + 0.5 * rho * (ke1 - ke0), U[L.energy])
    return U

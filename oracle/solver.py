"""Time stepping driver -- oracle, FP64.

One step: dt from the CFL reduction on U^n (clamped to the end time), three
SSP-RK3 stages of the hyperbolic system (Shu-Osher form,
U1 = U + dt L(U), U2 = 3/4 U + 1/4 (U1 + dt L(U1)),
U^{n+1} = 1/3 U + 2/3 (U2 + dt L(U2))), then the source step.  The outward
boundary fluxes are accumulated with the matching weights 1/6, 1/6, 2/3.
"""
import numpy as np

from .layout import Layout
from .mixture import Options, prim_to_cons, cons_to_prim
from .scheme import Geometry, rhs, clamp_phi, dt_inverse
from .source import source_step
from .driver import apply_driver
from .seeding import relax_void, seed_void
from .totals import interior_totals, boundary_totals
from . import fragments as _frag


class Solver:
    def __init__(self, case, opts=None):
        self.case = case
        self.opts = opts or Options(cfl=case.cfl,
                                    seed_nu=getattr(case, "seed_nu", 0.0),
                                    thinc_beta=getattr(case, "thinc_beta", 0.0))
        self.layout = Layout(case.dim, case.mats)
        self.geom = Geometry(case.dim, case.n, case.lo, case.hi, case.bc)
        self.U = prim_to_cons(case.prim.copy(), self.layout, self.opts)
        self.phi0 = case.phi0
        self.t = 0.0
        self.steps = 0
        self.bacc = {}
        dx = self.geom.dx
        self.cell_volume = dx[0] * dx[1] * dx[2]
        self.face_areas = (dx[1] * dx[2], dx[0] * dx[2], dx[0] * dx[1])

    def dt_cfl(self):
        return self.opts.cfl / dt_inverse(self.U, self.geom, self.layout)

    def _accumulate(self, bflux, w):
        for key, arr in bflux.items():
            inc = w * arr
            if key in self.bacc:
                self.bacc[key] = self.bacc[key] + inc
            else:
                self.bacc[key] = inc

    def step(self, dt=None, t_end=None):
        if dt is None:
            dt = self.dt_cfl()
        if t_end is not None:
            dt = min(dt, t_end - self.t)
        if dt <= 0:
            return 0.0
        L, g, o = self.layout, self.geom, self.opts
        U0 = self.U
        k1, b1 = rhs(U0, g, L, o)
        U1 = clamp_phi(U0 + dt * k1, L, o)
        k2, b2 = rhs(U1, g, L, o)
        U2 = clamp_phi(0.75 * U0 + 0.25 * (U1 + dt * k2), L, o)
        k3, b3 = rhs(U2, g, L, o)
        U3 = clamp_phi(U0 / 3.0 + (2.0 / 3.0) * (U2 + dt * k3), L, o)
        self._accumulate(b1, dt / 6.0)
        self._accumulate(b2, dt / 6.0)
        self._accumulate(b3, dt * (2.0 / 3.0))
        self.U = source_step(U3, self.phi0, g, L, o, dt)
        self.U = apply_driver(self.U, g, L, getattr(self.case, "driver", None),
                              self.t + dt)
        if getattr(o, "seed_nu", 0.0) > 0.0:
            self.U = seed_void(self.U, g, L, o.seed_nu)
            self.U = relax_void(self.U, g, L, o.seed_nu, o.phi_floor)
        self.t += dt
        self.steps += 1
        return dt

    def run(self, t_end, max_steps=None):
        while self.t < t_end:
            if max_steps is not None and self.steps >= max_steps:
                break
            if self.step(t_end=t_end) <= 0:
                break
        return self

    def totals(self):
        inner = interior_totals(self.U, self.layout, self.cell_volume)
        outer = boundary_totals(self.bacc, self.layout, self.face_areas)
        return inner, outer

    def prim(self):
        return cons_to_prim(self.U, self.layout)

    def fragments(self, solid=0, cut=0.5):
        L = self.layout
        return _frag.fragments(self.U[L.phi[solid]], self.U[L.mass[solid]],
                               self.cell_volume, cut)

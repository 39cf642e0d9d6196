"""Seeded synthetic inputs for the fracture hot path.

This package is shared by the CPU oracle and the GPU library's callers and
therefore holds none of the method's arithmetic: it only lays out geometry
(volume fractions from sub-sampling), material constants, initial primitive
fields and the random yield-perturbation fields phi0.  Every array is produced
from a fixed numpy PCG64 seed.

Primitive layout (same field count S as the conserved state):
    [phi_l] * N, [rho_l] * N, [eps_p, D] * n_solid, [u_i] * d, p,
    [Vbar components] * nV, [X_i] * d
with arrays shaped (S, nz, ny, nx); x is the fastest index.  Volume fractions
are raw geometric fractions (absent materials are 0, the consumer applies its
own floor) and absent materials carry their reference density.
"""
from .configs import (  # noqa: F401
    COPPER, GAS, Case, make_case, uniform_case, config_member_draws,
    vbar_components,
    prim_field_names, CONFIG_SEEDS, mass_edges, DEGENERATE_GRIDS,
    degenerate_case, spall_strip, expanding_disk, STEEL_304L, STEEL_304L_JC,
    CUBE, AL_H32, al_cube_spall, UNB, unb_ring, UNB_DRIVER,
)
from .fields import (  # noqa: F401
    uniform_field, gaussian_field, lognormal_field, inclusion_field,
    correlated_normal,
)

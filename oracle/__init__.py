"""CPU oracle for the fracture hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 NumPy implementation of what the GPU path computes,
written from the paper (Sections 2 and 3) and the readings of the passages it
leaves open.  Only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import it; the product library never does, and it shares no
code with the HIP path (the seeded generators in `fvinputs` are the only
common input).

Modules:
  layout      field order of the conserved state (Section 2.1 equation order)
  closures    single-material EOS and damage closures (Sections 2.2, 2.3)
  kinematics  Hencky strain of the unimodular stretch (Section 2.2)
  mixture     mixture pressure, stress, sound speed; cons <-> prim
  scheme      reconstruction, HLLC flux with the void-opening modifier,
              SSP-RK3 update, CFL (Sections 3.1, 3.2.1)
  source      plastic return, Bonora damage by RK4, phi0 gather
              (Sections 2.1, 2.2, 3.1, 3.2.2)
  seeding     Lagrangian coordinates of void cells extrapolated from the
              material (Section 3.2.1 seeding routine)
  totals      correctly rounded conservation totals
  fragments   fragment labelling and masses (Section 4 fragment delineation)
  solver      time stepping driver

Functions whose result no independent pin fixes say "parity unpinned" in
their docstring.
"""
from .layout import Layout  # noqa: F401
from .solver import Solver  # noqa: F401

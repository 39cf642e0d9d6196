"""FP32-bulk form against the FP64 form on the GPU (both through the C ABI).

Bars (per-field L1 of the FP32 run relative to the FP64 field's L1; solid
cells for eps_p and D): density 1e-4, velocity 1e-3, eps_p 1e-3, damage
1e-2.  Conservation drift of the FP32 run: every stage rounds each stored
cell value to 2^-24, so after K steps the relative drift of mass and energy
is bounded by 3 K 2^-24; the measured drift is printed beside it."""
import numpy as np
import pytest

import fvinputs as F
from oracle.layout import Layout

pytestmark = pytest.mark.gpu

BARS = dict(rho=1e-4, u=1e-3, eps=1e-3, D=1e-2)


def _run(case, precision, steps):
    from paper_2210_04037_amd.solver import GpuSolver
    g = GpuSolver(case, precision=precision)
    t0, _ = g.totals()
    g.step(steps)
    t1, b1 = g.totals()
    W = g.primitive(0)
    t = g.time()[0]
    g.close()
    return W, t0[0], t1[0] + b1[0], t


def _l1(a, b, mask=None):
    if mask is not None:
        a, b = a[mask], b[mask]
    den = np.sum(np.abs(b))
    return np.sum(np.abs(a - b)) / den if den > 0 else np.sum(np.abs(a - b))


@pytest.mark.parametrize("which,steps", [("spall", 300), ("ring", 150)])
def test_fp32_bulk_within_bars(which, steps):
    case = F.make_case(1, n=400) if which == "spall" else F.make_case(2, n=256)
    print(f"[precision] {which} {case.n} {steps} steps", flush=True)
    W64, a0, a1, t64 = _run(case, "fp64", steps)
    W32, c0, c1, t32 = _run(case, "fp32", steps)
    L = Layout(case.dim, case.mats)
    rho64 = np.sum(W64[L.phi] * W64[L.mass], axis=0)
    rho32 = np.sum(W32[L.phi] * W32[L.mass], axis=0)
    sp64 = np.sqrt(np.sum(W64[L.mom] ** 2, axis=0))
    sp32 = np.sqrt(np.sum(W32[L.mom] ** 2, axis=0))
    solid = W64[L.phi[0]] > 0.5
    errs = dict(rho=_l1(rho32, rho64), u=_l1(sp32, sp64),
                eps=_l1(W32[L.eps[0]], W64[L.eps[0]], solid),
                D=_l1(W32[L.dmg[0]], W64[L.dmg[0]], solid))
    nm = len(case.mats)
    drift_mass = max(abs(c1[l] - c0[l]) / abs(c0[l]) for l in range(nm))
    drift_e = abs(c1[-1] - c0[-1]) / abs(c0[-1])
    bound = 3 * steps * 2.0 ** -24
    print("[precision]", which, {k: f"{v:.2e}" for k, v in errs.items()},
          f"mass drift {drift_mass:.2e} energy drift {drift_e:.2e} "
          f"(bound {bound:.1e})", "t64", t64, "t32", t32, flush=True)
    for k, v in errs.items():
        assert v <= BARS[k], (k, v)
    assert drift_mass <= bound and drift_e <= bound

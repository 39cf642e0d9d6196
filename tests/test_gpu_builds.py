"""The two builds of the 1D and 2D stage kernels give the same bits.

Runs that use no extended closure, THINC or driver take the build with those
branches compiled out.  An imposed-velocity driver of radius zero that never
moves (r_in = 0, v0 = v1 = 0) touches no cell (a cell is pushed only when
0 < r <= R_d), but it makes the library take the full build; the two runs
must agree bit for bit."""
import numpy as np
import pytest

import fvinputs as F

pytestmark = pytest.mark.gpu

NEUTRAL_DRIVER = (0.0, 0.0, 0.0, 1.0e-6, 2.0e-6, 1.0)


def _run(case, precision, steps):
    from paper_2210_04037_amd.solver import GpuSolver
    g = GpuSolver(case, precision=precision)
    g.step(steps)
    out = [g.state(0), g.time()]
    g.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["ring", "disk"])
def test_reduced_and_full_builds_agree(which, precision):
    case = F.make_case(2, n=160) if which == "ring" else F.expanding_disk(64)
    steps = 30
    print(f"[builds] {which} {precision} {steps} steps", flush=True)
    plain = _run(case, precision, steps)
    case.driver = NEUTRAL_DRIVER
    full = _run(case, precision, steps)
    assert np.array_equal(plain[0], full[0])
    assert np.array_equal(plain[1], full[1])

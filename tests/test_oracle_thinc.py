"""Pins of the THINC volume-fraction reconstruction of the oracle (CPU only).

THINC (Xiao, Honma and Kono, 2005) replaces the piecewise-linear profile of
a volume fraction in a cell by q_min + (dq/2)(1 + theta tanh(beta (x - x_c)))
over the unit cell, with x_c chosen so that the cell average is kept.  The
paper names it for its ring.  What the definition fixes independently of the
closed form the oracle uses:

  * the tanh profile through the returned lower-face value has its
    upper-face value at the returned upper-face value, and its average over
    the cell (numerical quadrature) equals the cell value;
  * the face values lie between the neighbours and keep the data's order;
  * a step at the cell centre (C = 1/2) gives q_min + (dq/2)(1 -/+ tanh(beta/2));
  * a material interface carried at a uniform velocity stays sharper than
    with MUSCL, and is still carried at that velocity.
"""
import numpy as np
import pytest
import scipy.integrate

import fvinputs as F
from oracle import Solver
from oracle.layout import Layout
from oracle.scheme import _thinc_cell


@pytest.mark.parametrize("beta", [1.2, 1.6, 2.3])
def test_face_values_belong_to_an_average_preserving_tanh_profile(beta):
    rng = np.random.default_rng(7)
    for _ in range(200):
        qm, q1 = rng.uniform(0, 1, 2)
        q0 = qm + rng.uniform(0.01, 0.99) * (q1 - qm)
        lo, up, use = _thinc_cell(np.array([qm]), np.array([q0]), np.array([q1]), beta)
        assert use[0]
        qmin, dq = min(qm, q1), abs(q1 - qm)
        th = 1.0 if q1 >= qm else -1.0
        # x_c from the lower-face value, H(0) = qmin + dq/2 (1 + th tanh(-beta x_c))
        t0 = th * (2.0 * (lo[0] - qmin) / dq - 1.0)
        xc = -np.arctanh(t0) / beta

        def H(x):
            return qmin + 0.5 * dq * (1.0 + th * np.tanh(beta * (x - xc)))
        assert H(1.0) == pytest.approx(up[0], rel=1e-11, abs=1e-13)
        avg, _ = scipy.integrate.quad(H, 0.0, 1.0, epsabs=1e-14, epsrel=1e-13)
        assert avg == pytest.approx(q0, rel=1e-10, abs=1e-12)
        assert min(qm, q1) <= lo[0] <= max(qm, q1)
        assert min(qm, q1) <= up[0] <= max(qm, q1)
        # increasing data: lower face below the average, upper face above
        assert (up[0] - lo[0]) * (q1 - qm) > 0


def test_centred_step_closed_form():
    beta = 1.6
    lo, up, use = _thinc_cell(np.array([0.0]), np.array([0.5]), np.array([1.0]), beta)
    assert lo[0] == pytest.approx(0.5 * (1 - np.tanh(beta / 2)), rel=1e-14)
    assert up[0] == pytest.approx(0.5 * (1 + np.tanh(beta / 2)), rel=1e-14)
    lo, up, use = _thinc_cell(np.array([1.0]), np.array([0.5]), np.array([0.0]), beta)
    assert lo[0] == pytest.approx(0.5 * (1 + np.tanh(beta / 2)), rel=1e-14)
    assert up[0] == pytest.approx(0.5 * (1 - np.tanh(beta / 2)), rel=1e-14)


def test_not_used_where_the_data_are_not_monotone():
    lo, up, use = _thinc_cell(np.array([0.2, 0.5, 0.3]), np.array([0.8, 0.5, 0.3]),
                              np.array([0.4, 0.9, 0.7]), 1.6)
    assert not use[0] and not use[1] and not use[2]


def _translated_interface(beta, steps=700):
    """Copper and gas in pressure equilibrium moving together at 200 m/s:
    the interface is carried without a pressure or velocity jump."""
    n = 100
    mats = [F.COPPER, F.GAS]
    case = F.uniform_case(1, (n, 1, 1), mats, [1.0, 0.0], [8930.0, 1.0],
                          [200.0], 1.0e5, bc="periodic")
    L = Layout(1, mats)
    x = (np.arange(n) + 0.5) / n
    solid = ((x > 0.3) & (x < 0.6)).astype(float)
    case.prim[L.phi[0]] = solid[None, None, :]
    case.prim[L.phi[1]] = 1.0 - solid[None, None, :]
    case.thinc_beta = beta
    o = Solver(case)
    for _ in range(steps):
        o.step()
    phi = o.U[L.phi[0]][0, 0]
    return phi, o.t, case


def test_interface_stays_sharper_and_is_carried_at_the_flow_velocity():
    phi_t, t, case = _translated_interface(1.6)
    phi_m, _, _ = _translated_interface(0.0)
    n = phi_t.size
    L = case.hi[0] - case.lo[0]
    x = case.lo[0] + (np.arange(n) + 0.5) * L / n
    # the exactly translated slab, as cell averages
    edges = case.lo[0] + np.arange(n + 1) * L / n
    a, b = 0.3 * L + 200.0 * t, 0.6 * L + 200.0 * t
    exact = np.clip(np.minimum(edges[1:], b) - np.maximum(edges[:-1], a), 0, None) / (L / n)
    err_t = np.sum(np.abs(phi_t - exact))
    err_m = np.sum(np.abs(phi_m - exact))
    assert 200.0 * t > 10 * L / n                    # carried over ten cells
    assert err_t < 0.6 * err_m
    c0 = 0.45 * L + case.lo[0]
    c = np.sum(phi_t * x) / np.sum(phi_t)
    assert c == pytest.approx(c0 + 200.0 * t, abs=0.5 * L / n)
    # the solid volume is kept
    assert np.sum(phi_t) == pytest.approx(0.3 * n, rel=1e-6)

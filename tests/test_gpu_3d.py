"""The 3D path (three passes per stage: primitives, faces per direction,
gather with update and source) against the oracle, through the C ABI.

Tolerance as for 2D: 1e-9 of each field's largest magnitude, except that
the components of a vector or tensor share one scale: the stretch (O(1)),
the momentum and the Lagrangian coordinates.  A component can be round-off
sized (off-diagonal stretch in a plate impact, axial momentum of a radially
expanding shell), and a per-component scale would compare rounding noise
with itself."""
import numpy as np
import pytest

import fvinputs as F
from oracle import Solver
from oracle import fragments as Fr
from oracle.layout import Layout
from oracle.totals import interior_totals

pytestmark = pytest.mark.gpu

TOL = 1e-9


def _gpu(cases, **kw):
    from paper_2210_04037_amd.solver import GpuSolver
    return GpuSolver(cases, **kw)


def _scales(ref, L):
    sc = np.max(np.abs(ref.reshape(ref.shape[0], -1)), axis=1)
    for group in (L.vbar, L.mom, L.X):
        v = max(sc[r] for r in group)
        for r in group:
            sc[r] = v
    return sc + 1e-300


def _assert_close(got, ref, L, tol=TOL, what=""):
    sc = _scales(ref, L)
    err = np.max(np.abs(got - ref).reshape(ref.shape[0], -1), axis=1) / sc
    assert err.max() < tol, (what, err)
    return err.max()


def _crop(case, nx, ny, nz, x0=0, y0=0, z0=0):
    """Box [x0, x0+nx) x [y0, y0+ny) x [z0, z0+nz) of a 3D case with its own
    geometry (ragged extents for the parity tests)."""
    d = case.dx
    lo = tuple(case.lo[k] + (x0, y0, z0)[k] * d[k] for k in range(3))
    hi = tuple(lo[k] + (nx, ny, nz)[k] * d[k] for k in range(3))
    return F.Case(case.name + "_crop", 3, (nx, ny, nz), lo, hi, case.bc,
                  case.mats,
                  np.ascontiguousarray(case.prim[:, z0:z0 + nz, y0:y0 + ny, x0:x0 + nx]),
                  np.ascontiguousarray(case.phi0[z0:z0 + nz, y0:y0 + ny, x0:x0 + nx]),
                  case.t_end)


def _case(which):
    if which == "shell":
        return F.make_case(3, n=20)
    if which == "impact":
        return F.make_case(5, n=14)
    return _crop(F.make_case(3, n=24), 21, 17, 13, x0=1, y0=3, z0=5)


@pytest.mark.parametrize("which", ["shell", "impact", "ragged"])
def test_3d_parity(which):
    case = _case(which)
    steps = 10
    print(f"[3d] {which} {case.n} {steps} steps", flush=True)
    g = _gpu(case)
    o = Solver(case)
    for _ in range(steps):
        o.step()
    g.step(steps)
    L = Layout(3, case.mats)
    e = _assert_close(g.state(0), o.U, L, what=which)
    assert g.time()[0] == pytest.approx(o.t, rel=1e-13)
    print(f"[3d] {which} worst {e:.2e}", flush=True)
    g.close()


def test_3d_uniform_state_preserved_bitwise():
    V = [[1.01, 0.004, -0.002], [0.003, 0.995, 0.001], [-0.001, 0.002, 1.0]]
    case = F.uniform_case(3, (20, 18, 16), [F.COPPER, F.GAS], [0.7, 0.3],
                          [8930.0, 1.0], [30.0, -20.0, 10.0], 2.0e8,
                          bc="periodic", vbar=V)
    g = _gpu(case)
    g.step(8)
    U = g.state(0)
    L = Layout(3, case.mats)
    for r in range(L.S):
        if r in L.X:
            continue
        assert np.all(U[r] == U[r].ravel()[0]), r
    g.close()


def test_3d_conservation():
    case = F.uniform_case(3, (24, 20, 16), [F.COPPER, F.GAS], [0.6, 0.4],
                          [8930.0, 1.0], [10.0, 5.0, -3.0], 1.0e8,
                          bc="periodic")
    L = Layout(3, case.mats)
    z, y, x = np.meshgrid(np.arange(16) / 16, np.arange(20) / 20,
                          np.arange(24) / 24, indexing="ij")
    bump = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) * np.cos(2 * np.pi * z)
    case.prim[L.phi[0]] = 0.6 + 0.3 * bump
    case.prim[L.phi[1]] = 1.0 - case.prim[L.phi[0]]
    case.prim[L.mom[2]] += 20.0 * bump
    case.prim[L.energy] += 5.0e8 * bump
    g = _gpu(case)
    t0, _ = g.totals()
    g.step(10)
    t1, b1 = g.totals()
    assert np.all(b1 == 0.0)
    U = g.state(0)
    dv = np.prod(case.dx)
    scale = [np.sum(np.abs(U[r])) * dv for r in L.mass + L.mom + [L.energy]]
    assert np.all(np.abs(t1[0] - t0[0]) <= 1e-13 * np.array(scale))
    g.close()


def test_3d_free_surface_outflow_matches_oracle():
    """Plate impact copy with free x-ends: interior and cumulative outflow
    totals against the oracle."""
    case = F.make_case(5, n=12)
    g = _gpu(case)
    o = Solver(case)
    for _ in range(40):
        o.step()
    g.step(40)
    inner, outer = o.totals()
    gi, go = g.totals()
    assert np.allclose(gi[0], inner, rtol=1e-9, atol=1e-12 * np.max(np.abs(inner)))
    assert np.allclose(go[0], outer, rtol=1e-7, atol=1e-9 * np.max(np.abs(inner)))
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_3d_totals_and_fragments_on_the_same_state(precision):
    """Totals and fragment labels of an evolved 3D shell equal the oracle's
    on the state the device holds (bit for bit)."""
    case = F.make_case(3, n=40)
    g = _gpu(case, precision=precision)
    g.step(20)
    U = g.state(0)
    L = Layout(3, case.mats)
    got, _ = g.totals()
    assert list(got[0]) == interior_totals(U, L, float(np.prod(case.dx)))
    lab, frags = g.fragments(0, 0.5)
    assert np.array_equal(lab.astype(np.int64), Fr.label(U[0], 0.5))
    ref = Fr.fragments(U[0], U[len(case.mats)], float(np.prod(case.dx)), 0.5)
    assert frags == [(a, b, c, d) for (a, b, c, d) in ref]
    print(f"[3d] shell 40^3 {precision}: {len(frags)} fragments", flush=True)
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_3d_shell_64_fragments_at_end_time(precision):
    """The shell's fragment check on its 64^3 copy at the end time (18 us):
    the device's labels, fragment list and totals equal the oracle's on the
    state the device holds, bit for bit.  At 0.625 mm cells the 1 mm shell
    is 1.6 cells thick, so the labelling is what this checks, not the
    physics of the fragments."""
    case = F.make_case(3, n=64)
    g = _gpu(case, precision=precision, use_graph=True)
    g.step(0, t_end=[case.t_end])
    steps = 0
    while g.time()[0] < case.t_end:
        g.step(100)
        steps += 100
        assert steps < 20000
    g.cfl_dt()                            # raises on the device flag
    U = g.state(0)
    L = Layout(3, case.mats)
    dv = float(np.prod(case.dx))
    got, _ = g.totals()
    assert list(got[0]) == interior_totals(U, L, dv)
    # the cut of the solid fraction at 0.5 and lower (the paper's void
    # cut-offs run from 0.25 to 0.75): the smeared 1.6-cell shell shows up
    # at the lower ones
    counts = {}
    for cut in (0.5, 0.25, 0.1):
        lab, frags = g.fragments(0, cut)
        assert np.array_equal(lab.astype(np.int64), Fr.label(U[0], cut)), cut
        ref = Fr.fragments(U[0], U[len(case.mats)], dv, cut)
        assert frags == [(a, b, c, d) for (a, b, c, d) in ref], cut
        counts[cut] = len(frags)
    print(f"[3d] shell 64^3 {precision}: t = {g.time()[0]:.3e} s after {steps} steps, "
          f"fragments by cut {counts}, max solid fraction {float(U[0].max()):.3f}", flush=True)
    assert max(counts.values()) >= 1
    g.close()


def _window(case, o0, w, halo):
    """Sub-case of a 3D case around the output box [o0, o0 + w)^3 with a
    dependence halo, clipped to the domain."""
    n = case.n
    a = [max(o0[k] - halo, 0) for k in range(3)]
    b = [min(o0[k] + w + halo, n[k]) for k in range(3)]
    sub = _crop(case, b[0] - a[0], b[1] - a[1], b[2] - a[2], a[0], a[1], a[2])
    sub.bc = case.bc
    return sub, tuple(o0[k] - a[k] for k in range(3))


def test_3d_full_size_shell_sampled_windows():
    """The 256^3 shell: two fixed steps on the GPU, compared on windows the
    oracle recomputes (2 x 3 x 2-cell dependence halo)."""
    case = F.make_case(3)
    dt = 5.0e-9
    steps = 2
    print("[3d] full-size shell 256^3, 2 steps", flush=True)
    g = _gpu(case)
    g.step(steps, dt=dt)
    U = g.state(0)
    g.close()
    L = Layout(3, case.mats)
    halo = 6 * steps
    w = 12
    r = 0.0155 / 0.04 * 256
    spots = [(0, 0, 0), (128 + int(r) - w // 2, 128 - w // 2, 128 - w // 2),
             (128 - w // 2, 128 - int(r) - w // 2, 200)]
    for o0 in spots:
        sub, off = _window(case, o0, w, halo)
        o = Solver(sub)
        for _ in range(steps):
            o.step(dt=dt)
        sl = (slice(None),) + tuple(slice(off[2 - k], off[2 - k] + w) for k in range(3))
        ref = o.U[sl]
        got = U[:, o0[2]:o0[2] + w, o0[1]:o0[1] + w, o0[0]:o0[0] + w]
        _assert_close(got, ref, L, what=str(o0))


@pytest.mark.parametrize("cfg,precision", [(3, "fp64"), (3, "fp32"),
                                           (5, "fp32")])
def test_3d_full_size_runs_stay_physical(cfg, precision):
    """30 steps of the 256^3 shell and of the 512^3 plate impact (FP32-bulk,
    10.7 GB per state copy) without a non-physical flag."""
    case = F.make_case(cfg)
    print(f"[3d] full size config {cfg} {case.n} {precision}", flush=True)
    g = _gpu(case, precision=precision)
    t0, _ = g.totals()
    g.step(30)
    dt = g.cfl_dt()                     # raises on the device flag
    t1, b1 = g.totals()
    if cfg == 3:
        W = g.primitive(0)
        assert np.isfinite(W).all()
    g.close()
    assert dt[0] > 0 and np.isfinite(t1).all()
    # mass of the solid conserved up to the outflow and the state rounding
    assert abs(t1[0][0] + b1[0][0] - t0[0][0]) <= 90 * 2.0 ** -24 * abs(t0[0][0])


@pytest.mark.parametrize("cfg,n,steps", [(5, 64, 150), (3, 64, 120)])
def test_3d_fp32_bulk_within_bars(cfg, n, steps):
    from paper_2210_04037_amd.abi import state_rows
    case = F.make_case(cfg, n=n)
    out = {}
    for prec in ("fp64", "fp32"):
        g = _gpu(case, precision=prec)
        t0, _ = g.totals()
        g.step(steps)
        t1, b1 = g.totals()
        out[prec] = (g.primitive(0), t0[0], t1[0] + b1[0])
        g.close()
    rows = state_rows(3, len(case.mats), [m["kind"] == "solid" for m in case.mats])
    W64, W32 = out["fp64"][0], out["fp32"][0]

    def l1(a, b, m=None):
        if m is not None:
            a, b = a[m], b[m]
        return np.sum(np.abs(a - b)) / max(np.sum(np.abs(b)), 1e-300)

    rho = lambda W: np.sum(W[rows["phi"]] * W[rows["mass"]], axis=0)
    spd = lambda W: np.sqrt(np.sum(W[rows["mom"]] ** 2, axis=0))
    solid = W64[rows["phi"][0]] > 0.5
    errs = dict(rho=l1(rho(W32), rho(W64)), u=l1(spd(W32), spd(W64)),
                eps=l1(W32[rows["eps"][0]], W64[rows["eps"][0]], solid),
                D=l1(W32[rows["dmg"][0]], W64[rows["dmg"][0]], solid))
    c0, c1 = out["fp32"][1], out["fp32"][2]
    drift = abs(c1[0] - c0[0]) / abs(c0[0])
    print(f"[3d precision] config {cfg} {n}^3 {steps} steps",
          {k: f"{v:.2e}" for k, v in errs.items()}, f"mass drift {drift:.2e}",
          flush=True)
    bars = dict(rho=1e-4, u=1e-3, eps=1e-3, D=1e-2)
    for k, v in errs.items():
        assert v <= bars[k], (k, v)
    assert drift <= 3 * steps * 2.0 ** -24

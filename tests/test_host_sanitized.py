"""The device kernels' phase functions (primitives, faces, gather, update,
source, CFL), stepped on the CPU by tests/host/phase_step.cpp under
AddressSanitizer and UndefinedBehaviorSanitizer, against the oracle.

The harness drives the same tile walk as the 2D stage kernel (halo loads,
face items, per-cell gather) and the same three passes as the 3D path, with
NaN-filled scratch and asserted indices, so an out-of-range access, a slot
read before it is written, or undefined arithmetic (signed overflow, bad
shifts, misaligned loads) ends the run; the state it produces must still
match the oracle to the FP64 parity bar (1e-9 of each field's largest
magnitude, vector and tensor components sharing one scale)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import fvinputs as F
from oracle import Solver
from oracle.layout import Layout

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "phase_step.cpp")
TOL = 1e-9


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("san") / "phase_step")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-Wall", "-Wno-unknown-pragmas", "-Werror", "-o", out, SRC]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def _write_input(path, case, steps, tile_x):
    from paper_2210_04037_amd import abi
    L = Layout(case.dim, case.mats)
    ncell = int(np.prod(case.n))
    with open(path, "wb") as f:
        f.write(bytes(abi.grid_struct(case)))
        f.write(np.int32(len(case.mats)).tobytes())
        f.write(bytes(abi.material_array(case.mats)))
        f.write(bytes(abi.options_struct("fp64", case.cfl,
                                         seed_nu=getattr(case, "seed_nu", 0.0),
                                         thinc_beta=getattr(case, "thinc_beta", 0.0),
                                         driver=getattr(case, "driver", None))))
        f.write(np.int64(L.S).tobytes())
        f.write(np.int64(ncell).tobytes())
        f.write(np.int32(steps).tobytes())
        f.write(np.int32(tile_x).tobytes())
        f.write(np.ascontiguousarray(case.prim, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(case.phi0, dtype=np.float64).tobytes())
    return L


def _run(exe, tmp_path, case, steps, tile_x=0):
    src, dst = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    L = _write_input(src, case, steps, tile_x)
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, src, dst], capture_output=True, text=True,
                       timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-6000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-6000:]
    raw = np.fromfile(dst, dtype=np.float64)
    t, flag = raw[0], raw[1]
    U = raw[2:].reshape(case.prim.shape)
    return t, flag, U, L


def _assert_matches_oracle(case, steps, t, flag, U, L):
    o = Solver(case)
    for _ in range(steps):
        o.step()
    assert flag == 0.0
    assert t == pytest.approx(o.t, rel=1e-13)
    sc = np.max(np.abs(o.U.reshape(L.S, -1)), axis=1)
    for group in (L.vbar, L.mom, L.X):
        v = max(sc[r] for r in group)
        for r in group:
            sc[r] = v
    err = np.max(np.abs(U - o.U).reshape(L.S, -1), axis=1) / (sc + 1e-300)
    assert err.max() < TOL, err


@pytest.mark.parametrize("which,steps", [
    ("spall1d", 12), ("ring2d", 4), ("ring2d_wide", 3), ("ring2d_spare", 3),
    ("ring2d_spare14", 3),
    ("shell3d", 2), ("shell3d_runs", 1),
    ("impact3d", 2), ("disk2d", 40), ("alcube1d", 120), ("alcube2d", 30),
    ("disk2d_jc", 30), ("ring2d_thinc", 6), ("spall1d_thinc", 40),
    ("unb2d", 3), ("unb3d", 4)])
def test_phase_functions_sanitized_match_oracle(exe, tmp_path, which, steps):
    tile_x = 0
    if which == "spall1d":
        case = F.make_case(1, n=45)            # 16-cell tiles, ragged tail
    elif which == "ring2d":
        case = F.make_case(2, n=22)            # 8 x 4 tiles, ragged both ways
    elif which == "ring2d_wide":
        case = F.make_case(2, n=40)            # 32 x 8 tiles
        tile_x = 32
    elif which == "ring2d_spare":
        case = F.make_case(2, n=37)            # 16 x 15 tiles on 256 threads
        tile_x = 16
    elif which == "ring2d_spare14":
        case = F.make_case(2, n=35)            # 16 x 14 tiles on 256 threads
        tile_x = 14
    elif which == "shell3d":
        case = F.make_case(3, n=10)
    elif which == "shell3d_runs":
        # x-face runs across rows, three marching runs along y and z with a
        # ragged last one
        case = F.make_case(3, n=34)
    elif which == "disk2d":
        case = F.expanding_disk(20)            # void around the disk: seeding
    elif which == "alcube1d":
        # two solids, Johnson-Cook hardening and rate terms (both), damage
        case = F.al_cube_spall(1, n=40, v=550.0)
    elif which == "alcube2d":
        case = F.al_cube_spall(2, n=20, ny=5, v=550.0)
    elif which == "ring2d_thinc":
        case = F.make_case(2, n=35)            # 16 x 14 tiles, THINC on
        case.thinc_beta = 1.6
        tile_x = 14
    elif which == "spall1d_thinc":
        case = F.make_case(1, n=45)
        case.thinc_beta = 1.6
    elif which == "unb2d":
        # Steinberg modulus, Burakovsky-Preston Grueneisen, Johnson-Cook with
        # thermal softening, the simplified damage law, the driver, seeding.
        # Later, cells the driver leaves at volume fractions just above the
        # trace threshold, at normal density, set the CFL step, and
        # rounding-order differences flip the trace switch there; next to
        # the relaxed void films they grow about fifty-fold a step from the
        # second step (2.4e-10 of the field scale at step 3, 1.3e-9 at 4).
        case = F.unb_ring(2, n=40)
    elif which == "unb3d":
        case = F.unb_ring(3, n=24, nz=4)
    elif which == "disk2d_jc":
        # Johnson-Cook with thermal softening (304L row)
        case = F.expanding_disk(20, mat=F.STEEL_304L_JC)
    else:
        case = F.make_case(5, n=9)
    t, flag, U, L = _run(exe, tmp_path, case, steps, tile_x)
    _assert_matches_oracle(case, steps, t, flag, U, L)


@pytest.mark.parametrize("dim,n,bc", F.DEGENERATE_GRIDS)
def test_degenerate_grids_sanitized_match_oracle(exe, tmp_path, dim, n, bc):
    """Grids of one to a few cells per direction, where the two-cell halo
    and the tile reach past the whole grid (a periodic one wraps more than
    once)."""
    case = F.degenerate_case(dim, n, bc)
    t, flag, U, L = _run(exe, tmp_path, case, 5)
    _assert_matches_oracle(case, 5, t, flag, U, L)


@pytest.fixture(scope="module")
def hencky_exe(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("hk") / "hencky_check")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-Wno-unknown-pragmas",
           "-Werror", "-o", out, os.path.join(HERE, "host", "hencky_check.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_hencky_of_strongly_sheared_stretch(hencky_exe, dim):
    """dev H = dev 1/2 ln(V V^T) of unimodular stretches with principal
    ratios up to 1e12 (the state of rarefied gas cells late in the ring
    runs): finite, and equal to the same strain from the singular values of
    V (which are the square roots of the eigenvalues of V V^T) to the
    rounding that the conditioning allows.  Formed from the entries of V V^T
    alone, the smallest eigenvalue is lost below about 1e8."""
    def stretch(s, th, c):
        R = np.array([[np.cos(th), -np.sin(th), 0.0],
                      [np.sin(th), np.cos(th), 0.0], [0.0, 0.0, 1.0]])
        return R @ np.diag([s, 1.0 / (s * c), c]) @ R.T

    cases = [(1.0001, 0.7, 1.0), (1e3, 0.3, 1.0), (3e3, 0.9, 0.02),
             (1e5, 2.0, 25.7), (1e6, 1.1, 0.5)]
    Vs = [stretch(*c) for c in cases]
    inp = f"{dim}\n" + "\n".join(" ".join(repr(float(x)) for x in V.ravel())
                                 for V in Vs) + "\n"
    r = subprocess.run([hencky_exe], input=inp, capture_output=True, text=True,
                       timeout=60)
    assert r.returncode == 0, r.stderr[-4000:]
    rows = r.stdout.strip().split("\n")
    assert len(rows) == len(Vs)
    for (s, _, _), V, row in zip(cases, Vs, rows):
        H = np.array([float(t) for t in row.split()]).reshape(3, 3)
        U, sig, _ = np.linalg.svd(V)
        h = np.log(sig)
        h -= h.mean()
        ref = (U * h) @ U.T
        assert np.isfinite(H).all(), s
        # the rounding of V itself moves the smallest singular value by
        # about eps * sigma_max, i.e. its log by eps * kappa
        kappa = sig.max() / sig.min()
        bound = (1e-11 + 4 * np.finfo(float).eps * kappa) * np.max(np.abs(ref))
        assert np.max(np.abs(H - ref)) <= bound, (s, np.max(np.abs(H - ref)), bound)


@pytest.fixture(scope="module")
def damage_exe(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("dm") / "damage_check")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-Wno-unknown-pragmas",
           "-Werror", "-o", out, os.path.join(HERE, "host", "damage_check.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def test_damage_closures_match_oracle(damage_exe):
    """The kernels' threshold strain and Bonora damage rate (Section 2.2),
    with the solid's derived constants formed as the library forms them,
    equal the oracle's to 1e-13 over the triaxialities, damage levels and
    strains the source step meets (R from 2/3 to 12, D up to just below
    D_crit, eps_p from 1e-4 to 2)."""
    from oracle import closures as Cl
    m = dict(F.COPPER)
    rng = np.random.default_rng(11)
    R = np.concatenate([[2.0 / 3.0, 1.0, 1.5, 12.0], rng.uniform(0.67, 12.0, 60)])
    D = np.concatenate([[0.0, 0.5, m["D_crit"] * (1 - 1e-9), 0.3],
                        rng.uniform(0.0, m["D_crit"] * 0.999, 60)])
    eps = np.concatenate([[1e-4, 0.08, 0.16, 2.0], 10 ** rng.uniform(-4, 0.3, 60)])
    head = " ".join(repr(float(m[k])) for k in
                    ("eps_th", "eps_c", "n_hard", "bonora_alpha", "D_crit", "D0",
                     "K0", "G0"))
    body = "\n".join(f"{float(a)!r} {float(b)!r} {float(c)!r}"
                      for a, b, c in zip(R, D, eps))
    r = subprocess.run([damage_exe], input=head + "\n" + body + "\n",
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr[-4000:]
    got = np.array([[float(t) for t in row.split()]
                    for row in r.stdout.strip().split("\n")])
    thr = np.array([Cl.eps_threshold(a, m) for a in R])
    rate = Cl.bonora_dD_deps(D, eps, R, m)
    assert np.allclose(got[:, 0], thr, rtol=1e-13, atol=0)
    assert np.allclose(got[:, 1], rate, rtol=1e-13, atol=0)
    # R = 1 reduces the threshold to eps_th itself
    assert got[1, 0] == pytest.approx(m["eps_th"], rel=1e-14)

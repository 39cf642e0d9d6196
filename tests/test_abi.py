"""Host-side checks of the C-ABI library (CPU only, no device calls): it
loads, exports every entry point declared in include/fv.h, sizes state and
workspace, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

import fvinputs as F
from paper_2210_04037_amd import abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(abi.LIB_PATH):
        pytest.skip("libfv.so not built (run __graft_entry__.build())")
    return abi.load()


def test_exports_match_header():
    lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "fv.h")).read()
    declared = set(re.findall(r"\b(fv_[a-z_0-9]+)\s*\(", hdr))
    assert declared == set(abi.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_state_fields_and_workspace():
    lib = _lib()
    c = F.make_case(2, n=64)
    mats = abi.material_array(c.mats)
    assert lib.fv_state_fields(2, 2, mats) == 16
    c1 = F.make_case(1, n=50)
    assert lib.fv_state_fields(1, 1, abi.material_array(c1.mats)) == 10
    g = (abi.FvGrid * 1)(abi.grid_struct(c))
    o = abi.options_struct("fp64")
    n = lib.fv_workspace_bytes(1, g, 2, mats, ctypes.byref(o))
    # two stage copies of the state at least
    assert n >= 2 * 16 * 64 * 64 * 8
    bad = abi.options_struct("fp64", cfl=1.5)
    assert lib.fv_workspace_bytes(1, g, 2, mats, ctypes.byref(bad)) == 0


def test_two_dimensional_field_size_limit():
    """In 1D and 2D one state field may hold up to 4 GiB: 2^29 cells in
    FP64, 2^30 in FP32-bulk; one row more is rejected."""
    lib = _lib()
    c = F.make_case(2, n=64)
    mats = abi.material_array(c.mats)
    for prec, rows in (("fp64", 1 << 14), ("fp32", 1 << 15)):
        o = abi.options_struct(prec)
        g = (abi.FvGrid * 1)(abi.grid_struct(c))
        g[0].n[0], g[0].n[1] = 1 << 15, rows
        assert lib.fv_workspace_bytes(1, g, 2, mats, ctypes.byref(o)) > 0
        g[0].n[1] = rows + 1
        assert lib.fv_workspace_bytes(1, g, 2, mats, ctypes.byref(o)) == 0
        ctx = ctypes.c_void_p()
        ptrs = (ctypes.c_void_p * 1)(ctypes.c_void_p(0x1000))
        rc = lib.fv_init(ctypes.byref(ctx), 1, g, 2, mats, ctypes.byref(o),
                         ptrs, ptrs, ctypes.c_void_p(0x1000), 1 << 30, None)
        assert rc == abi.FV_EINVAL
        assert b"4 GiB" in lib.fv_last_error(None)


def test_init_rejects_invalid_arguments():
    lib = _lib()
    c = F.make_case(2, n=32)
    mats = abi.material_array(c.mats)
    g = (abi.FvGrid * 1)(abi.grid_struct(c))
    o = abi.options_struct("fp64")
    ctx = ctypes.c_void_p()
    ptrs = (ctypes.c_void_p * 1)(ctypes.c_void_p(0x1000))
    # periodic on one side only
    g[0].bc[0][0] = abi.FV_BC["periodic"]
    rc = lib.fv_init(ctypes.byref(ctx), 1, g, 2, mats, ctypes.byref(o), ptrs,
                     ptrs, ctypes.c_void_p(0x1000), 1 << 30, None)
    assert rc == abi.FV_EINVAL
    assert b"periodic" in lib.fv_last_error(None)
    g[0].bc[0][0] = abi.FV_BC["transmissive"]
    # gas before solid
    rev = abi.material_array([c.mats[1], c.mats[0]])
    rc = lib.fv_init(ctypes.byref(ctx), 1, g, 2, rev, ctypes.byref(o), ptrs,
                     ptrs, ctypes.c_void_p(0x1000), 1 << 30, None)
    assert rc == abi.FV_EINVAL
    # null state pointer
    nulls = (ctypes.c_void_p * 1)()
    rc = lib.fv_init(ctypes.byref(ctx), 1, g, 2, mats, ctypes.byref(o), nulls,
                     ptrs, ctypes.c_void_p(0x1000), 1 << 30, None)
    assert rc == abi.FV_EINVAL
    lib.fv_destroy(None)


@pytest.mark.parametrize("cfg", [1, 2])
def test_state_rows_match_library_and_oracle_layout(cfg):
    """The binding's field map agrees with the library's field count and
    with the oracle's layout (written independently from the same order)."""
    from oracle.layout import Layout
    lib = _lib()
    c = F.make_case(cfg, n=16)
    rows = abi.state_rows(c.dim, len(c.mats),
                          [m["kind"] == "solid" for m in c.mats])
    assert rows["S"] == lib.fv_state_fields(c.dim, len(c.mats),
                                            abi.material_array(c.mats))
    L = Layout(c.dim, c.mats)
    assert rows["S"] == L.S
    assert rows["phi"] == L.phi and rows["mass"] == L.mass
    assert rows["eps"] == [L.eps[l] for l in L.solids]
    assert rows["dmg"] == [L.dmg[l] for l in L.solids]
    assert rows["mom"] == L.mom and rows["energy"] == L.energy
    assert rows["vbar"] == L.vbar and rows["X"] == L.X


def test_fragment_histogram_matches_oracle_definition():
    """fv_fragment_histogram is host code: checked here against the oracle's
    cumulative count on seeded lists (ties at an edge, unsorted edges)."""
    import numpy as np
    from oracle import fragments as Fr
    lib = _lib()
    rng = np.random.default_rng(11)
    for n in (0, 1, 7, 300):
        masses = np.round(rng.lognormal(-3, 2, n), 3)
        frags = [(i, 1, float(m), i % 2 == 0) for i, m in enumerate(masses)]
        arr = (abi.FvFragment * max(n, 1))()
        for i, (lab, nc, m, t) in enumerate(frags):
            arr[i].label, arr[i].n_cells, arr[i].mass = lab, nc, m
            arr[i].touches_boundary = int(t)
        edges = list(rng.permutation(np.concatenate(
            [masses[:5], np.geomspace(1e-6, 10.0, 15)])))
        e = (ctypes.c_double * len(edges))(*edges)
        out = (ctypes.c_int64 * len(edges))()
        assert lib.fv_fragment_histogram(arr, n, e, len(edges), out) == 0
        assert list(out) == Fr.mass_histogram(frags, edges)
    assert lib.fv_fragment_histogram(None, -1, None, 0, None) == abi.FV_EINVAL


def test_periodic_direction_needs_two_cells():
    """The two-cell halo wraps a periodic direction once, so a periodic
    direction of one cell is rejected before any device work (it would
    index outside the grid)."""
    lib = _lib()
    mats = [F.COPPER, F.GAS]
    o = abi.options_struct("fp64")
    for n, ok in (((1, 8, 1), False), ((2, 8, 1), True), ((8, 1, 1), False)):
        c = F.uniform_case(2, n, mats, [0.5, 0.5], [8930.0, 1.0], [0.0, 0.0],
                           1e5, bc="periodic")
        g = (abi.FvGrid * 1)(abi.grid_struct(c))
        nb = lib.fv_workspace_bytes(1, g, 2, abi.material_array(mats),
                                    ctypes.byref(o))
        assert (nb > 0) == ok, n

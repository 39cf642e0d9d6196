"""No entry point writes outside the buffers it is given: the workspace and
every state buffer are followed by canary bytes, and after loading,
stepping (eager and graph), the autotuner, totals, a checkpoint, a restore
and fragment labelling, in 1D, 2D, 3D and an ensemble, every canary byte is
unchanged."""
import ctypes

import numpy as np
import pytest

import fvinputs as F

pytestmark = pytest.mark.gpu

PAD = 1 << 16
CANARY = 0xA5


def _run(cases, precision):
    import torch
    from paper_2210_04037_amd import abi
    lib = abi.load()
    dev = torch.device("cuda:0")
    n = len(cases)
    c0 = cases[0]
    grids = (abi.FvGrid * n)(*[abi.grid_struct(c) for c in cases])
    mats = abi.material_array(c0.mats)
    opt = abi.options_struct(precision, c0.cfl, use_graph=True)
    S = lib.fv_state_fields(c0.dim, len(c0.mats), mats)
    dt = torch.float64 if precision == "fp64" else torch.float32
    elem = 8 if precision == "fp64" else 4
    nbytes = lib.fv_workspace_bytes(n, grids, len(c0.mats), mats, ctypes.byref(opt))
    assert nbytes > 0
    ws = torch.full((nbytes + PAD,), CANARY, dtype=torch.uint8, device=dev)
    raw = []
    for c in cases:
        ncell = int(np.prod(c.n))
        b = torch.full((S * ncell * elem + PAD,), CANARY, dtype=torch.uint8, device=dev)
        raw.append((b, S * ncell * elem))
    phi0 = [torch.as_tensor(np.ascontiguousarray(c.phi0), dtype=dt).to(dev) for c in cases]
    sp = (ctypes.c_void_p * n)(*[b.data_ptr() for b, _ in raw])
    pp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in phi0])
    ctx = ctypes.c_void_p()
    stream = torch.cuda.current_stream(dev)
    rc = lib.fv_init(ctypes.byref(ctx), n, grids, len(c0.mats), mats, ctypes.byref(opt),
                     sp, pp, ctypes.c_void_p(ws.data_ptr()), nbytes,
                     ctypes.c_void_p(stream.cuda_stream))
    assert rc == 0, lib.fv_last_error(None)
    ok = lambda r: r == 0 or pytest.fail(lib.fv_last_error(ctx).decode())
    for i, c in enumerate(cases):
        prim = torch.as_tensor(np.ascontiguousarray(c.prim), dtype=torch.float64).to(dev)
        ok(lib.fv_load_primitive(ctx, i, ctypes.c_void_p(prim.data_ptr())))
    ok(lib.fv_step(ctx, None, 3, None))
    tiles = (ctypes.c_int32 * 96)()
    ms = (ctypes.c_float * 32)()
    ok(lib.fv_autotune(ctx, 2, 32, tiles, ms, None, None))
    ok(lib.fv_step(ctx, None, 2, None))
    nt = len(c0.mats) + c0.dim + 1
    out = (ctypes.c_double * (n * 2 * nt))()
    ok(lib.fv_totals(ctx, out))
    ck_n = lib.fv_checkpoint_bytes(ctx)
    ck = torch.full((ck_n + PAD,), CANARY, dtype=torch.uint8, device=dev)
    ok(lib.fv_checkpoint(ctx, ctypes.c_void_p(ck.data_ptr())))
    ok(lib.fv_restore(ctx, ctypes.c_void_p(ck.data_ptr())))
    ok(lib.fv_step(ctx, None, 2, None))
    dts = (ctypes.c_double * n)()
    ok(lib.fv_cfl_dt(ctx, dts))
    frag = []
    for i, c in enumerate(cases):
        ncell = int(np.prod(c.n))
        cap = ncell // 2 + 1
        fb = lib.fv_fragment_workspace_bytes(ctx, i, cap)
        fws = torch.full((fb + PAD,), CANARY, dtype=torch.uint8, device=dev)
        lab = torch.full((ncell * 4 + PAD,), CANARY, dtype=torch.uint8, device=dev)
        res = (abi.FvFragment * cap)()
        nf = ctypes.c_int64()
        ok(lib.fv_fragments(ctx, i, 0.5, ctypes.c_void_p(lab.data_ptr()),
                            ctypes.c_void_p(fws.data_ptr()), fb, cap, ctypes.byref(nf), res))
        frag.append((fws, fb, lab, ncell * 4))
    lib.fv_destroy(ctx)
    torch.cuda.synchronize()
    assert bool((ws[nbytes:] == CANARY).all()), "workspace overrun"
    assert bool((ck[ck_n:] == CANARY).all()), "checkpoint overrun"
    for i, (b, used) in enumerate(raw):
        assert bool((b[used:] == CANARY).all()), f"state {i} overrun"
    for i, (fws, fb, lab, lb) in enumerate(frag):
        assert bool((fws[fb:] == CANARY).all()), f"fragment workspace {i} overrun"
        assert bool((lab[lb:] == CANARY).all()), f"labels {i} overrun"


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["1d", "2d", "3d", "ensemble"])
def test_no_writes_outside_given_buffers(which, precision):
    if which == "1d":
        cases = [F.make_case(1, n=130)]
    elif which == "2d":
        cases = [F.make_case(2, n=70)]
    elif which == "3d":
        cases = [F.make_case(3, n=20)]
    else:
        cases = [F.make_case(4, member=m, n=n) for m, n in ((0, 40), (1, 57))]
    print(f"[bounds] {which} {precision}", flush=True)
    _run(cases, precision)

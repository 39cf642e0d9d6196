"""Torch-backed driver of the C ABI: allocates the caller-owned device
buffers (state, phi0, workspace) with PyTorch, passes raw pointers and the
current HIP stream to libfv, and converts host arrays.  No arithmetic of the
method happens here."""
import ctypes

import numpy as np

from . import abi


def _check(lib, ctx, rc):
    if rc != abi.FV_OK:
        msg = lib.fv_last_error(ctx)
        raise abi.FvError(rc, msg.decode() if msg else "")


class GpuSolver:
    """One context over one or more instances (an ensemble shares dimension,
    materials and options)."""

    def __init__(self, cases, precision="fp64", device="cuda:0", cfl=None,
                 phi_floor=1e-8, weno_eps=1e-6, phi_fp64_cut=1e-6, load=True,
                 tile=None, use_graph=False):
        import torch
        if not isinstance(cases, (list, tuple)):
            cases = [cases]
        self.torch = torch
        self.lib = lib = abi.load()
        self.cases = list(cases)
        self.n_inst = len(cases)
        self.device = torch.device(device)
        c0 = cases[0]
        self.dim = c0.dim
        self.mats = c0.mats
        self.grids = (abi.FvGrid * self.n_inst)(
            *[abi.grid_struct(c) for c in cases])
        self.mat_arr = abi.material_array(self.mats)
        self.opt = abi.options_struct(precision, cfl or c0.cfl, phi_floor,
                                      weno_eps, phi_fp64_cut, tile, use_graph,
                                      getattr(c0, "seed_nu", 0.0),
                                      getattr(c0, "thinc_beta", 0.0),
                                      getattr(c0, "driver", None))
        self.S = lib.fv_state_fields(self.dim, len(self.mats), self.mat_arr)
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.states, self.phi0s = [], []
        for c in cases:
            nx, ny, nz = c.n
            self.states.append(torch.empty((self.S, nz, ny, nx),
                                           dtype=self.dtype, device=self.device))
            self.phi0s.append(torch.as_tensor(
                np.ascontiguousarray(c.phi0), dtype=self.dtype).to(self.device))
        nbytes = lib.fv_workspace_bytes(self.n_inst, self.grids, len(self.mats),
                                        self.mat_arr, ctypes.byref(self.opt))
        if nbytes == 0:
            raise abi.FvError(abi.FV_EINVAL, lib.fv_last_error(None) or b"")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8,
                                     device=self.device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        sp = (ctypes.c_void_p * self.n_inst)(
            *[t.data_ptr() for t in self.states])
        pp = (ctypes.c_void_p * self.n_inst)(
            *[t.data_ptr() for t in self.phi0s])
        self.ctx = ctypes.c_void_p()
        rc = lib.fv_init(ctypes.byref(self.ctx), self.n_inst, self.grids,
                         len(self.mats), self.mat_arr, ctypes.byref(self.opt),
                         sp, pp, ctypes.c_void_p(self.workspace.data_ptr()),
                         nbytes, ctypes.c_void_p(self.stream.cuda_stream))
        _check(lib, None, rc)
        if load:
            for i, c in enumerate(cases):
                self.load_primitive(i, c.prim)

    def _c(self, rc):
        _check(self.lib, self.ctx, rc)

    def load_primitive(self, i, prim):
        t = self.torch.as_tensor(np.ascontiguousarray(prim),
                                 dtype=self.torch.float64).to(self.device)
        self._c(self.lib.fv_load_primitive(self.ctx, i, ctypes.c_void_p(t.data_ptr())))

    def reset(self):
        self._c(self.lib.fv_reset(self.ctx))

    def step(self, n=1, dt=None, t_end=None):
        dtp = None
        tep = None
        if dt is not None:
            dtp = (ctypes.c_double * self.n_inst)(*np.broadcast_to(dt, self.n_inst))
        if t_end is not None:
            tep = (ctypes.c_double * self.n_inst)(*np.broadcast_to(t_end, self.n_inst))
        self._c(self.lib.fv_step(self.ctx, dtp, int(n), tep))

    def cfl_dt(self):
        out = (ctypes.c_double * self.n_inst)()
        self._c(self.lib.fv_cfl_dt(self.ctx, out))
        return np.array(out[:])

    def time(self):
        out = (ctypes.c_double * self.n_inst)()
        self._c(self.lib.fv_time(self.ctx, out))
        return np.array(out[:])

    def totals(self):
        nt = len(self.mats) + self.dim + 1
        out = (ctypes.c_double * (self.n_inst * 2 * nt))()
        self._c(self.lib.fv_totals(self.ctx, out))
        a = np.array(out[:]).reshape(self.n_inst, 2, nt)
        return a[:, 0], a[:, 1]

    def primitive(self, i=0):
        t = self.torch.empty(self.states[i].shape, dtype=self.torch.float64,
                             device=self.device)
        self._c(self.lib.fv_primitive(self.ctx, i, ctypes.c_void_p(t.data_ptr())))
        self.torch.cuda.synchronize(self.device)
        return t.cpu().numpy()

    def state(self, i=0):
        self.torch.cuda.synchronize(self.device)
        return self.states[i].double().cpu().numpy()

    def checkpoint(self):
        """Copies of the state buffers and the context's own state (time,
        CFL state, boundary outflow, step count), all on the device."""
        n = self.lib.fv_checkpoint_bytes(self.ctx)
        blob = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        self._c(self.lib.fv_checkpoint(self.ctx, ctypes.c_void_p(blob.data_ptr())))
        return [t.clone() for t in self.states], blob

    def restore(self, ck):
        """Continue from a checkpoint of a context with the same grids,
        materials and options (bit for bit)."""
        states, blob = ck
        for t, s in zip(self.states, states):
            t.copy_(s)
        self.torch.cuda.synchronize(self.device)
        self._c(self.lib.fv_restore(self.ctx, ctypes.c_void_p(blob.data_ptr())))

    def autotune(self, reps=20):
        """Time every compiled tile shape under every block schedule, keep
        the fastest; returns (chosen (tx, ty, schedule),
        {(tx, ty, schedule): ms per launch})."""
        cap = 64
        tiles = (ctypes.c_int32 * (3 * cap))()
        ms = (ctypes.c_float * cap)()
        nv, ch = ctypes.c_int32(), ctypes.c_int32()
        self._c(self.lib.fv_autotune(self.ctx, int(reps), cap, tiles, ms,
                                     ctypes.byref(nv), ctypes.byref(ch)))
        n = min(nv.value, cap)
        key = lambda v: tuple(tiles[3 * v:3 * v + 3])
        return key(ch.value), {key(v): ms[v] for v in range(n)}

    def fragments(self, i=0, cut=0.5, cap=None):
        """Fragment labels (nz, ny, nx) int32 (-1 outside material) and the
        fragment list [(label, n_cells, mass, touches_boundary)] in label
        order, from the library's device labelling."""
        torch = self.torch
        c = self.cases[i]
        ncell = int(np.prod(c.n))
        cap = ncell // 2 + 1 if cap is None else int(cap)
        nbytes = self.lib.fv_fragment_workspace_bytes(self.ctx, i, cap)
        if nbytes == 0:
            raise abi.FvError(abi.FV_EINVAL, "fragment workspace size")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        labels = torch.empty(ncell, dtype=torch.int32, device=self.device)
        out = (abi.FvFragment * max(cap, 1))()
        nf = ctypes.c_int64()
        self._c(self.lib.fv_fragments(
            self.ctx, i, float(cut), ctypes.c_void_p(labels.data_ptr()),
            ctypes.c_void_p(ws.data_ptr()), nbytes, cap, ctypes.byref(nf), out))
        nx, ny, nz = c.n
        lab = labels.cpu().numpy().reshape(nz, ny, nx)
        frags = [(int(f.label), int(f.n_cells), float(f.mass),
                  bool(f.touches_boundary)) for f in out[:nf.value]]
        return lab, frags

    def fragments_noalloc(self, i=0, cut=0.5, cap=4096):
        """As fragments(), through fv_fragments_noalloc: the library's static
        scratch replaces the workspace (only the label buffer is the
        caller's)."""
        torch = self.torch
        c = self.cases[i]
        ncell = int(np.prod(c.n))
        labels = torch.empty(ncell, dtype=torch.int32, device=self.device)
        out = (abi.FvFragment * max(int(cap), 1))()
        nf = ctypes.c_int64()
        self._c(self.lib.fv_fragments_noalloc(
            self.ctx, i, float(cut), ctypes.c_void_p(labels.data_ptr()),
            int(cap), ctypes.byref(nf), out))
        nx, ny, nz = c.n
        lab = labels.cpu().numpy().reshape(nz, ny, nx)
        frags = [(int(f.label), int(f.n_cells), float(f.mass),
                  bool(f.touches_boundary)) for f in out[:nf.value]]
        return lab, frags

    def mass_histogram(self, frags, edges):
        """Cumulative fragment count at each mass edge (entry k: fragments of
        mass >= edges[k]) from the library's fv_fragment_histogram."""
        n = len(frags)
        arr = (abi.FvFragment * max(n, 1))()
        for k, (lab, nc, m, t) in enumerate(frags):
            arr[k].label, arr[k].n_cells, arr[k].mass = lab, nc, m
            arr[k].touches_boundary = int(t)
        e = (ctypes.c_double * len(edges))(*[float(v) for v in edges])
        out = (ctypes.c_int64 * len(edges))()
        self._c(self.lib.fv_fragment_histogram(arr, n, e, len(edges), out))
        return list(out)

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.fv_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

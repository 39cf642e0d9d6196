"""ctypes binding of include/fv.h: the C structs, status codes and the
library loader.  Argument marshalling only; every step of the method runs in
the HIP kernels of libfv.so."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfv.so")

FV_OK, FV_EINVAL, FV_ENOMEM, FV_EDEVICE, FV_ENONPHYS, FV_ESTATE = 0, -1, -2, -3, -4, -5
FV_FRAGMENT_SCRATCH_BYTES = 64 << 20
FV_BC = {"transmissive": 0, "free": 1, "periodic": 2}
FV_MAT = {"solid": 0, "gas": 1}
FV_FP64, FV_FP32_BULK = 0, 1
PRECISIONS = {"fp64": FV_FP64, "fp32": FV_FP32_BULK}

EXPORTS = ["fv_state_fields", "fv_workspace_bytes", "fv_init",
           "fv_load_primitive", "fv_reset", "fv_primitive", "fv_cfl_dt",
           "fv_step", "fv_time", "fv_totals", "fv_checkpoint_bytes",
           "fv_checkpoint", "fv_restore", "fv_autotune",
           "fv_fragment_workspace_bytes",
           "fv_fragments", "fv_fragments_noalloc", "fv_fragment_histogram",
           "fv_last_error",
           "fv_destroy"]


class FvGrid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("bc", (ctypes.c_int32 * 2) * 3)]


class FvMaterial(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32)] + [
        (n, ctypes.c_double) for n in (
            "rho0", "K0", "alpha", "G0", "beta", "Gamma0", "yield_", "D_crit",
            "D0", "eps_th", "eps_c", "bonora_alpha", "n_hard", "p_gate",
            "jc_B", "jc_C", "jc_m", "T_melt", "C_V",
            "G_p", "Gamma1", "Gamma2", "gamma_bp", "Ddot0")]


class FvOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("cfl", ctypes.c_double),
                ("phi_floor", ctypes.c_double), ("weno_eps", ctypes.c_double),
                ("phi_fp64_cut", ctypes.c_double),
                ("tile", ctypes.c_int32 * 3), ("use_graph", ctypes.c_int32),
                ("seed_nu", ctypes.c_double), ("thinc_beta", ctypes.c_double),
                ("driver", ctypes.c_double * 6)]


class FvFragment(ctypes.Structure):
    _fields_ = [("label", ctypes.c_int64), ("n_cells", ctypes.c_int64),
                ("mass", ctypes.c_double), ("touches_boundary", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class FvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libfv status {code}: {msg}")
        self.code = code


_lib = None


def load(path=LIB_PATH):
    """Load libfv.so; raises if it has not been built (there is no
    fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with "
            "`python -m paper_2210_04037_amd.build` (no CPU fallback exists)")
    try:
        # one HIP runtime per process: a ROCm build of torch brings its own,
        # which must be the one libfv binds to when both are used
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    P = ctypes.POINTER
    lib.fv_state_fields.argtypes = [i32, i32, P(FvMaterial)]
    lib.fv_state_fields.restype = i32
    lib.fv_workspace_bytes.argtypes = [i32, P(FvGrid), i32, P(FvMaterial), P(FvOptions)]
    lib.fv_workspace_bytes.restype = ctypes.c_size_t
    lib.fv_init.argtypes = [P(vp), i32, P(FvGrid), i32, P(FvMaterial), P(FvOptions),
                            P(vp), P(vp), vp, ctypes.c_size_t, vp]
    lib.fv_init.restype = i32
    lib.fv_load_primitive.argtypes = [vp, i32, vp]
    lib.fv_load_primitive.restype = i32
    lib.fv_reset.argtypes = [vp]
    lib.fv_reset.restype = i32
    lib.fv_primitive.argtypes = [vp, i32, vp]
    lib.fv_primitive.restype = i32
    lib.fv_cfl_dt.argtypes = [vp, P(dbl)]
    lib.fv_cfl_dt.restype = i32
    lib.fv_checkpoint_bytes.argtypes = [vp]
    lib.fv_checkpoint_bytes.restype = ctypes.c_size_t
    lib.fv_checkpoint.argtypes = [vp, vp]
    lib.fv_checkpoint.restype = i32
    lib.fv_restore.argtypes = [vp, vp]
    lib.fv_restore.restype = i32
    lib.fv_autotune.argtypes = [vp, i32, i32, P(i32), P(ctypes.c_float), P(i32), P(i32)]
    lib.fv_autotune.restype = i32
    lib.fv_fragment_workspace_bytes.argtypes = [vp, i32, ctypes.c_int64]
    lib.fv_fragment_workspace_bytes.restype = ctypes.c_size_t
    lib.fv_fragments.argtypes = [vp, i32, dbl, vp, vp, ctypes.c_size_t,
                                 ctypes.c_int64, P(ctypes.c_int64), P(FvFragment)]
    lib.fv_fragments.restype = i32
    lib.fv_fragments_noalloc.argtypes = [vp, i32, dbl, vp, ctypes.c_int64,
                                         P(ctypes.c_int64), P(FvFragment)]
    lib.fv_fragments_noalloc.restype = i32
    lib.fv_fragment_histogram.argtypes = [vp, ctypes.c_int64, P(dbl), i32,
                                          P(ctypes.c_int64)]
    lib.fv_fragment_histogram.restype = i32
    lib.fv_step.argtypes = [vp, P(dbl), i32, P(dbl)]
    lib.fv_step.restype = i32
    lib.fv_time.argtypes = [vp, P(dbl)]
    lib.fv_time.restype = i32
    lib.fv_totals.argtypes = [vp, P(dbl)]
    lib.fv_totals.restype = i32
    lib.fv_last_error.argtypes = [vp]
    lib.fv_last_error.restype = ctypes.c_char_p
    lib.fv_destroy.argtypes = [vp]
    lib.fv_destroy.restype = None
    _lib = lib
    return lib


def grid_struct(case):
    g = FvGrid()
    g.dim = case.dim
    for k in range(3):
        g.n[k] = int(case.n[k])
        g.lo[k] = float(case.lo[k])
        g.hi[k] = float(case.hi[k])
        for s in range(2):
            g.bc[k][s] = FV_BC[case.bc[k][s]]
    return g


def material_array(mats):
    arr = (FvMaterial * len(mats))()
    for l, m in enumerate(mats):
        a = arr[l]
        a.kind = FV_MAT[m["kind"]]
        for key in ("rho0", "K0", "alpha", "G0", "beta", "Gamma0", "D_crit",
                    "D0", "eps_th", "eps_c", "bonora_alpha", "n_hard",
                    "p_gate"):
            setattr(a, key, float(m[key]))
        a.yield_ = float(m["yield_stress"])
        for key in ("jc_B", "jc_C", "jc_m", "T_melt", "C_V",
                    "G_p", "Gamma1", "Gamma2", "gamma_bp", "Ddot0"):
            setattr(a, key, float(m.get(key, 0.0)))
    return arr


def options_struct(precision="fp64", cfl=0.6, phi_floor=1e-8, weno_eps=1e-6,
                   phi_fp64_cut=1e-6, tile=None, use_graph=False, seed_nu=0.0,
                   thinc_beta=0.0, driver=None):
    o = FvOptions()
    o.precision = PRECISIONS[precision]
    o.cfl = cfl
    o.phi_floor = phi_floor
    o.weno_eps = weno_eps
    o.phi_fp64_cut = phi_fp64_cut
    if tile is not None:
        # (x, y) or (x, y, block schedule)
        for k, v in enumerate(tile):
            o.tile[k] = int(v)
    o.use_graph = 1 if use_graph else 0
    o.seed_nu = float(seed_nu)
    o.thinc_beta = float(thinc_beta)
    if driver is not None:
        for k, v in enumerate(driver):
            o.driver[k] = float(v)
    return o


def state_rows(dim, n_mat, solid):
    """Row indices of the state (and primitive) fields in the layout that
    include/fv.h documents: volume fractions, phasic masses, (eps_p, D) of
    each solid, momentum, energy, stored stretch components, Lagrangian
    coordinates.  `solid` flags which materials are solids."""
    k = 0
    rows = {"phi": list(range(k, k + n_mat))}
    k += n_mat
    rows["mass"] = list(range(k, k + n_mat))
    k += n_mat
    rows["eps"], rows["dmg"] = [], []
    for l in range(n_mat):
        if solid[l]:
            rows["eps"].append(k)
            rows["dmg"].append(k + 1)
            k += 2
    rows["mom"] = list(range(k, k + dim))
    k += dim
    rows["energy"] = k
    k += 1
    nv = {1: 3, 2: 5, 3: 9}[dim]
    rows["vbar"] = list(range(k, k + nv))
    k += nv
    rows["X"] = list(range(k, k + dim))
    k += dim
    rows["S"] = k
    return rows


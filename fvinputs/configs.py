"""Synthetic workloads: materials, geometry and initial primitive fields.

The five workloads follow the inert problems of the paper's validation
section (plate-impact spallation, expanding ring, expanding shell), built on a
copper-like solid whose constants are stated below.  Where the workloads leave
a detail open these readings fill it: free-surface ends for the plate
impacts, gas at atmospheric pressure around rings and shells, gate pressure
-1.5 GPa for plate impacts and 0 otherwise.
"""
from dataclasses import dataclass, field
import numpy as np

from .fields import (uniform_field, gaussian_field, lognormal_field,
                     inclusion_field)

# Base seed: workload k uses CONFIG_SEEDS[k] for its phi0 field and draws.
CONFIG_SEEDS = {k: 221004037 + k for k in range(1, 6)}
ENSEMBLE_MEMBER_SEED0 = 4000

# Copper-like solid: rho0 8930 kg/m^3, bulk sound speed 3940 m/s
# (K0 = rho0 * 3940^2), shear modulus 45 GPa, yield 90 MPa.  Romenskii
# exponents and Grueneisen constant from the CuBe row of the paper's
# Romenskii table; Bonora constants from its CuBe damage row with the
# critical damage 0.9; hardening exponent from its Johnson-Cook CuBe row.
COPPER = dict(
    kind="solid", rho0=8930.0, K0=8930.0 * 3940.0 ** 2, alpha=1.0, G0=45.0e9,
    beta=3.0, Gamma0=2.0, yield_stress=90.0e6, D_crit=0.9, D0=0.0,
    eps_th=0.08, eps_c=0.16, bonora_alpha=0.631, n_hard=0.31, p_gate=0.0,
)
# Low-density ideal gas, gamma = 1.4 (Grueneisen constant gamma - 1).
GAS = dict(
    kind="gas", rho0=1.0, K0=0.0, alpha=1.0, G0=0.0, beta=0.0, Gamma0=0.4,
    yield_stress=0.0, D_crit=1.0, D0=0.0, eps_th=0.0, eps_c=0.0,
    bonora_alpha=1.0, n_hard=1.0, p_gate=0.0,
)
P_ATM = 1.0e5

# 304L stainless steel of the expanding disk, all from the paper's Appendix A
# rows: Romenskii table (rho0, K0, G0, alpha, beta, Gamma0), the Johnson-Cook
# table's initial yield c1 (hardening, rate and thermal terms are not part
# of this build: the yield is constant) and hardening exponent n, and the
# Bonora table's expanding-disk row (D_crit, eps_thresh, eps_crit, alpha).
STEEL_304L = dict(
    kind="solid", rho0=8000.0, K0=158.3e9, alpha=0.569, G0=73.1e9, beta=2.437,
    Gamma0=1.84, yield_stress=0.253e9, D_crit=0.3, D0=0.0, eps_th=0.002,
    eps_c=0.5, bonora_alpha=0.5, n_hard=0.313, p_gate=0.0,
)

# The two solids of the paper's spallation test (Section 4.1), all from its
# Appendix A rows: the Romenskii table (rho0, K0, G0, alpha, beta, Gamma0),
# the Johnson-Cook table (c1 the yield, c2 = jc_B, c3 = jc_C, n; neither
# material has thermal terms there) and, for the damageable CuBe target, the
# Bonora table (D_crit, eps_thresh, eps_crit, alpha).  The aluminium flyer
# does not damage (the paper damages the copper only): its damage gate never
# opens.  The CuBe gate is the plate impacts' -1.5 GPa.
CUBE = dict(
    kind="solid", rho0=8370.0, K0=131.3e9, alpha=1.0, G0=53.6e9, beta=3.0,
    Gamma0=2.0, yield_stress=1.041e9, jc_B=0.0, jc_C=0.025, n_hard=0.31,
    D_crit=0.85, D0=0.0, eps_th=0.08, eps_c=0.16, bonora_alpha=0.631,
    p_gate=-1.5e9,
)
AL_H32 = dict(
    kind="solid", rho0=2670.0, K0=72.2e9, alpha=0.627354, G0=25.8e9,
    beta=2.28816, Gamma0=1.48389, yield_stress=0.275e9, jc_B=0.114e9,
    jc_C=0.002, n_hard=0.42, D_crit=0.99, D0=0.0, eps_th=0.08, eps_c=0.16,
    bonora_alpha=1.0, p_gate=-1.0e30,
)
# 304L with the full Johnson-Cook row of the paper's plasticity table
# (hardening, rate and thermal softening), for the Johnson-Cook variant of
# the expanding disk.
STEEL_304L_JC = dict(STEEL_304L, jc_B=0.685e9, jc_C=0.097, jc_m=2.044,
                     T_melt=1689.0, C_V=468.6)

# U-Nb of the paper's expanding ring (Section 4.3), from its Appendix A rows:
# the Romenskii-Steinberg table (rho0, K0, G0, G_p, alpha and the
# Burakovsky-Preston Gamma0 (in the role of Gamma_infinity), Gamma1, Gamma2,
# gamma), the Johnson-Cook table (c1..C_V) and the simplified damage law of
# the ring section (Ddot0 = 0.15, D_crit = 0.1).  beta, the Romenskii shear
# exponent, is not used by the Steinberg modulus; the Bonora constants are
# placeholders the simplified law does not read.
UNB = dict(
    kind="solid", rho0=17411.0, K0=111.27e9, alpha=1.105, G0=26.34e9,
    beta=0.0, Gamma0=0.5, G_p=1.1226, Gamma1=1.056, Gamma2=1.068,
    gamma_bp=3.843, yield_stress=0.780e9, jc_B=0.253e9, jc_C=0.012,
    n_hard=0.22, jc_m=1.0, T_melt=1710.0, C_V=115.0, D_crit=0.1, D0=0.0,
    Ddot0=0.15, eps_th=0.08, eps_c=0.16, bonora_alpha=1.0, p_gate=0.0,
)


# The driver profile of the paper's ring (Section 4.3): 210 m/s reached at
# 17.5 us, 160 m/s at 35 us, arrested at 20 mm.
UNB_RING_R = (17.185e-3, 17.945e-3)
UNB_DRIVER = (UNB_RING_R[0], 210.0, 160.0, 17.5e-6, 35.0e-6, 20.0e-3)


def unb_ring(dim=2, n=300, nz=8, t_end=50.0e-6, corr_len=0.2e-3, seed=None,
             thinc_beta=0.0, mat=None, driver=UNB_DRIVER):
    """The paper's expanding U-Nb ring (Section 4.3) without AMR: a ring of
    radii 17.185-17.945 mm about the z axis in void, at rest and at zero
    pressure, driven by the imposed-velocity driver (UNB_DRIVER), CFL 0.3,
    50 us, Gaussian yield perturbation of mean 1 and std 0.167, transmissive
    sides, Lagrangian seeding of void cells.  dim 3 is the paper's slab
    [-30, 30]^2 x [-0.8, 0.8] mm with a square cross-section (|z| <= 0.38
    mm) on n x n x nz cells; dim 2 the plane cross-section on n x n cells.
    The paper gives no correlation length for the perturbation: 0.2 mm
    here, as for the copper rings.  `mat` replaces U-Nb and `driver` the
    driver (None: off)."""
    r0, r1 = UNB_RING_R
    lo = (-0.03, -0.03, -0.0008 if dim == 3 else 0.0)
    hi = (0.03, 0.03, 0.0008 if dim == 3 else 1.0)
    grid = (n, n, nz if dim == 3 else 1)
    mats = [dict(UNB if mat is None else mat)]

    def ind(X, Y, Z):
        r = np.sqrt(X * X + Y * Y)
        inside = (r >= r0) & (r <= r1)
        return inside & (np.abs(Z) <= 0.38e-3) if dim == 3 else inside

    def vel(X, Y, Z):
        return [np.zeros_like(X) for _ in range(dim)]

    frac, u = _subsample(dim, grid, lo, hi, ind, vel, mats[0]["rho0"], 1.0e-30)
    prim = _assemble(dim, mats, frac, u, 0.0, grid, lo, hi)
    d = (hi[0] - lo[0]) / n
    shp = (grid[2], grid[1], grid[0])
    sd = CONFIG_SEEDS[2] + 500 + dim if seed is None else seed
    dxs = (((hi[2] - lo[2]) / grid[2]) if dim == 3 else 1.0, d, d)
    phi0 = gaussian_field(shp, dxs, corr_len, 0.167, sd)
    bc = (("transmissive",) * 2,) * 3
    return Case(f"unbring{dim}d", dim, grid, lo, hi, bc, mats, prim, phi0,
                t_end, cfl=0.3, seed_nu=0.99, thinc_beta=thinc_beta,
                driver=driver)


def al_cube_spall(dim=1, n=None, flyer=2.0e-3, v=400.0, a=0.05, t_end=5.0e-6,
                  seed=None, ny=None):
    """The paper's spallation test (Section 4.1): an Al-H32 flyer strikes a
    CuBe target on [0, 11] mm (the paper's domain, CFL 0.4, 5 us).  The
    initial-condition figure is not available: the flyer here is the first
    `flyer` metres, moving at `v` m/s, the rest of the domain is the target
    at rest, both at zero pressure, with free x-ends.  The CuBe yield is
    perturbed by a field uniform in [1 - a, 1 + a] per cell (the paper's
    perturbation study).  dim 2 gives the paper's quasi-one-dimensional
    square (n x n cells unless ny is given, transmissive in y)."""
    nx = n or (110 if dim == 1 else 800)
    nyy = 1 if dim == 1 else (ny or nx)
    lo = (0.0, 0.0, 0.0)
    hi = (0.011, 0.011 if dim == 2 else 1.0, 1.0)
    grid = (nx, nyy, 1)
    mats = [dict(CUBE), dict(AL_H32)]
    dx = (hi[0] - lo[0]) / nx
    xl = lo[0] + np.arange(nx) * dx
    # exact target fraction of each cell (the interface is a plane x = flyer)
    frac_x = np.clip((xl + dx - flyer) / dx, 0.0, 1.0)
    shp = (1, nyy, nx)
    frac = np.broadcast_to(frac_x, shp).copy()
    mc, ma = frac * mats[0]["rho0"], (1.0 - frac) * mats[1]["rho0"]
    u = [ma * v / (mc + ma)] + [np.zeros(shp)] * (dim - 1)
    prim = _assemble(dim, mats, frac, u, 0.0, grid, lo, hi)
    sd = CONFIG_SEEDS[1] + 300 + dim if seed is None else seed
    phi0 = uniform_field(shp, a, sd)
    bc = (("free", "free"), ("transmissive",) * 2, ("transmissive",) * 2)
    return Case(f"alcube{dim}d", dim, grid, lo, hi, bc, mats, prim, phi0, t_end,
                cfl=0.4)


def vbar_components(dim):
    """Stored (i, j) components of the unimodular stretch, row-major:
    1D uniaxial strain keeps Vbar diagonal; 2D plane strain keeps the xy block
    and the zz entry; 3D stores all nine."""
    if dim == 1:
        return [(0, 0), (1, 1), (2, 2)]
    if dim == 2:
        return [(0, 0), (0, 1), (1, 0), (1, 1), (2, 2)]
    return [(i, j) for i in range(3) for j in range(3)]


def prim_field_names(dim, mats):
    n = len(mats)
    solids = [l for l, m in enumerate(mats) if m["kind"] == "solid"]
    names = [f"phi{l}" for l in range(n)] + [f"rho{l}" for l in range(n)]
    for l in solids:
        names += [f"eps{l}", f"D{l}"]
    names += ["u", "v", "w"][:dim] + ["p"]
    names += [f"V{i + 1}{j + 1}" for i, j in vbar_components(dim)]
    names += ["X", "Y", "Z"][:dim]
    return names


@dataclass
class Case:
    name: str
    dim: int
    n: tuple            # (nx, ny, nz)
    lo: tuple           # (x, y, z) lower corner; unused dims span [0, 1]
    hi: tuple
    bc: tuple           # ((xlo, xhi), (ylo, yhi), (zlo, zhi)) names
    mats: list
    prim: np.ndarray    # (S, nz, ny, nx)
    phi0: np.ndarray    # (nz, ny, nx)
    t_end: float
    cfl: float = 0.6
    meta: dict = field(default_factory=dict)
    # void-fraction threshold of the Lagrangian seeding (0: off)
    seed_nu: float = 0.0
    # THINC steepness of the volume-fraction reconstruction (0: MUSCL)
    thinc_beta: float = 0.0
    # imposed-velocity driver (r_in, v0, v1, t0, t1, r_max) or None
    driver: tuple = None

    @property
    def dx(self):
        return tuple((self.hi[k] - self.lo[k]) / self.n[k] for k in range(3))

    @property
    def n_cells(self):
        return int(self.n[0] * self.n[1] * self.n[2])


def _centres(n, lo, hi, sub=1):
    """Cell-centre (sub=1) or sub-sample coordinates per axis."""
    out = []
    for k in range(3):
        d = (hi[k] - lo[k]) / n[k]
        if sub == 1:
            out.append(lo[k] + (np.arange(n[k]) + 0.5) * d)
        else:
            off = (np.arange(sub) + 0.5) / sub
            out.append(lo[k] + (np.arange(n[k])[:, None] + off[None, :]) * d)
    return out


def _subsample(dim, n, lo, hi, indicator, velocity, rho_in, rho_out, sub=4,
               may_hold=None):
    """Volume fraction of the solid region and the mass-weighted velocity of
    each cell from sub^dim sub-samples.  `indicator(x, y, z)` -> bool array,
    `velocity(x, y, z)` -> list of d arrays (solid velocity).  `may_hold(x,
    y, z, reach)`, if given, marks the cells whose centre lies within `reach`
    (half the cell diagonal) of the solid region; the others hold no solid
    sub-sample and are skipped (same values, computed only where needed)."""
    nx, ny, nz = n
    frac = np.zeros((nz, ny, nx))
    mom = np.zeros((dim, nz, ny, nx))
    mass = np.zeros((nz, ny, nx))
    subs = [sub if k < dim else 1 for k in range(3)]
    d = [(hi[k] - lo[k]) / n[k] for k in range(3)]
    cnt = float(np.prod(subs))
    if may_hold is None:
        cells = None
    else:
        cx, cy, cz = _centres(n, lo, hi)
        Zc, Yc, Xc = np.meshgrid(cz, cy, cx, indexing="ij")
        reach = 0.5 * float(np.sqrt(sum(d[k] ** 2 for k in range(dim))))
        cells = np.nonzero(may_hold(Xc, Yc, Zc, reach).ravel())[0]
        del Xc, Yc, Zc
        iz, iy, ix = np.unravel_index(cells, (nz, ny, nx))
        mass.ravel()[:] = rho_out * cnt        # no solid sub-sample
    for sz in range(subs[2]):
        for sy in range(subs[1]):
            for sx in range(subs[0]):
                if cells is None:
                    zc = lo[2] + (np.arange(nz) + (sz + 0.5) / subs[2]) * d[2]
                    yc = lo[1] + (np.arange(ny) + (sy + 0.5) / subs[1]) * d[1]
                    xc = lo[0] + (np.arange(nx) + (sx + 0.5) / subs[0]) * d[0]
                    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
                    ins = indicator(X, Y, Z)
                    frac += ins
                    rho = np.where(ins, rho_in, rho_out)
                    mass += rho
                    vel = velocity(X, Y, Z)
                    for k in range(dim):
                        mom[k] += np.where(ins, rho * vel[k], 0.0)
                    continue
                Z = lo[2] + (iz + (sz + 0.5) / subs[2]) * d[2]
                Y = lo[1] + (iy + (sy + 0.5) / subs[1]) * d[1]
                X = lo[0] + (ix + (sx + 0.5) / subs[0]) * d[0]
                ins = indicator(X, Y, Z)
                rho = np.where(ins, rho_in, rho_out)
                f = frac.ravel()
                f[cells] = f[cells] + ins
                if sz == 0 and sy == 0 and sx == 0:
                    mass.ravel()[cells] = 0.0
                mv = mass.ravel()
                mv[cells] = mv[cells] + rho
                vel = velocity(X, Y, Z)
                for k in range(dim):
                    mk = mom[k].ravel()
                    mk[cells] = mk[cells] + np.where(ins, rho * vel[k], 0.0)
    frac /= cnt
    u = mom / mass[None]
    return frac, u


def _assemble(dim, mats, frac_solid, u, p, n, lo, hi):
    """Primitive array (S, nz, ny, nx) from the solid volume fraction, the
    velocity and a uniform pressure.  Material 0 is the solid; if a second
    material is present it fills the remainder."""
    nx, ny, nz = n
    shp = (nz, ny, nx)
    nm = len(mats)
    rows = []
    if nm == 1:
        rows.append(frac_solid)
    else:
        rows += [frac_solid, 1.0 - frac_solid]
    rows += [np.full(shp, m["rho0"]) for m in mats]
    for m in mats:
        if m["kind"] == "solid":
            rows += [np.zeros(shp), np.zeros(shp)]
    rows += [u[k] for k in range(dim)]
    rows.append(np.full(shp, p))
    for (i, j) in vbar_components(dim):
        rows.append(np.full(shp, 1.0 if i == j else 0.0))
    cx, cy, cz = _centres(n, lo, hi)
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    rows += [X, Y, Z][:dim]
    return np.stack(rows).astype(np.float64)


def config_member_draws(n_members=64):
    """Ensemble draws: grid edge in {256, 384, 512, 768} and ring speed in
    U(100, 250) m/s per member."""
    rng = np.random.Generator(np.random.PCG64(CONFIG_SEEDS[4]))
    sizes = rng.choice(np.array([256, 384, 512, 768]), size=n_members)
    vels = rng.uniform(100.0, 250.0, size=n_members)
    return [int(s) for s in sizes], [float(v) for v in vels]


def _copper(p_gate):
    m = dict(COPPER)
    m["p_gate"] = p_gate
    return m


def _ring(name, nedge, v_out, phi0_seed, t_end, with_phi0=True):
    lo = (-0.03, -0.03, 0.0)
    hi = (0.03, 0.03, 1.0)
    n = (nedge, nedge, 1)
    r_in, r_out = 0.025, 0.0265
    mats = [_copper(0.0), dict(GAS)]

    def ind(X, Y, Z):
        r = np.sqrt(X * X + Y * Y)
        return (r >= r_in) & (r <= r_out)

    def vel(X, Y, Z):
        # u = v_out (r / r_out) rhat = v_out / r_out * (x, y)
        s = v_out / r_out
        return [s * X, s * Y]

    frac, u = _subsample(2, n, lo, hi, ind, vel, mats[0]["rho0"],
                         mats[1]["rho0"])
    prim = _assemble(2, mats, frac, u, P_ATM, n, lo, hi)
    dxs = (1.0, (hi[1] - lo[1]) / n[1], (hi[0] - lo[0]) / n[0])
    phi0 = (gaussian_field((1, nedge, nedge), dxs, 0.2e-3, 0.05, phi0_seed)
            if with_phi0 else np.ones((1, nedge, nedge)))
    bc = (("transmissive",) * 2, ("transmissive",) * 2, ("transmissive",) * 2)
    return Case(name, 2, n, lo, hi, bc, mats, prim, phi0, t_end,
                meta=dict(v_out=v_out))


def make_case(config, n=None, member=None, t_end=None):
    """Build workload `config` (1..5).  `n` overrides the grid edge (a scaled
    copy of the same geometry); `member` selects an ensemble member of
    workload 4."""
    if config == 1:
        nx = n or 400
        lo, hi = (0.0, 0.0, 0.0), (0.01, 1.0, 1.0)
        mats = [_copper(-1.5e9)]
        grid = (nx, 1, 1)

        def ind(X, Y, Z):
            return np.ones_like(X, dtype=bool)

        def vel(X, Y, Z):
            return [np.where(X < 0.002, 200.0, 0.0)]

        frac, u = _subsample(1, grid, lo, hi, ind, vel, mats[0]["rho0"], 1.0)
        prim = _assemble(1, mats, frac, u, P_ATM, grid, lo, hi)
        phi0 = uniform_field((1, 1, nx), 0.05, CONFIG_SEEDS[1])
        bc = (("free", "free"), ("transmissive",) * 2, ("transmissive",) * 2)
        return Case("spall1d", 1, grid, lo, hi, bc, mats, prim, phi0,
                    t_end if t_end is not None else 2.0e-6)
    if config == 2:
        c = _ring("ring2d", n or 1024, 150.0, CONFIG_SEEDS[2],
                  t_end if t_end is not None else 40.0e-6)
        return c
    if config == 3:
        ne = n or 256
        lo, hi = (-0.02, -0.02, -0.02), (0.02, 0.02, 0.02)
        grid = (ne, ne, ne)
        mats = [_copper(0.0), dict(GAS)]

        def ind(X, Y, Z):
            r = np.sqrt(X * X + Y * Y)
            return (r >= 0.015) & (r <= 0.016) & (np.abs(Z) <= 0.015)

        def vel(X, Y, Z):
            r = np.sqrt(X * X + Y * Y)
            r = np.where(r > 0, r, 1.0)
            return [200.0 * X / r, 200.0 * Y / r, np.zeros_like(X)]

        def near(X, Y, Z, reach):
            r = np.sqrt(X * X + Y * Y)
            return (np.abs(r - 0.0155) <= 0.0005 + reach) & (np.abs(Z) <= 0.015 + reach)

        frac, u = _subsample(3, grid, lo, hi, ind, vel, mats[0]["rho0"],
                             mats[1]["rho0"], may_hold=near)
        prim = _assemble(3, mats, frac, u, P_ATM, grid, lo, hi)
        d = (hi[0] - lo[0]) / ne
        phi0 = lognormal_field((ne, ne, ne), (d, d, d), 0.3e-3, 0.05,
                               CONFIG_SEEDS[3])
        bc = (("transmissive",) * 2,) * 3
        return Case("shell3d", 3, grid, lo, hi, bc, mats, prim, phi0,
                    t_end if t_end is not None else 18.0e-6)
    if config == 4:
        sizes, vels = config_member_draws()
        m = 0 if member is None else member
        ne = n or sizes[m]
        c = _ring(f"ensemble_m{m}", ne, vels[m], ENSEMBLE_MEMBER_SEED0 + m,
                  t_end if t_end is not None else 40.0e-6)
        c.meta["member"] = m
        return c
    if config == 5:
        ne = n or 512
        lo, hi = (0.0, 0.0, 0.0), (0.02, 0.02, 0.02)
        grid = (ne, ne, ne)
        mats = [_copper(-1.5e9)]

        def ind(X, Y, Z):
            return np.ones_like(X, dtype=bool)

        def vel(X, Y, Z):
            return [np.where(X < 0.004, 400.0, 0.0)]

        # The plate is uniform in y and z: sub-sample the x profile only.
        frac1, u1 = _subsample(1, (ne, 1, 1), lo, (hi[0], 1.0, 1.0), ind, vel,
                               mats[0]["rho0"], 1.0)
        frac = np.broadcast_to(frac1, (ne, ne, ne))
        u = np.zeros((3, ne, ne, ne))
        u[0] = u1[0]
        prim = _assemble(3, mats, frac, u, P_ATM, grid, lo, hi)
        phi0 = inclusion_field(grid, lo, hi, (0.004, 0.0, 0.0),
                               (0.02, 0.02, 0.02), 1000, 0.1e-3, 0.3e-3, 0.7,
                               CONFIG_SEEDS[5])
        bc = (("free", "free"), ("transmissive",) * 2, ("transmissive",) * 2)
        return Case("impact3d", 3, grid, lo, hi, bc, mats, prim, phi0,
                    t_end if t_end is not None else 3.0e-6)
    raise ValueError(f"unknown workload {config}")


def expanding_disk(n=400, t_end=200.0e-6, corr_len=1.0e-3, seed=221004043,
                   mat=None):
    """The expanding disk of the paper's validation section: a 304L disk of
    radius 10 cm centred in a [-13, 13]^2 cm domain of void, radial velocity
    u = 2000 r (1/s), Gaussian phi0 (mean 1, std 0.1, rectified), CFL 0.4,
    200 us, transmissive sides, Lagrangian seeding into cells of void
    fraction above 0.99.  The paper leaves the correlation length of phi0
    open: 1 mm here (1.5 cells at 400^2).  `mat` replaces the constant-yield
    304L (STEEL_304L_JC: its full Johnson-Cook row).  Void cells hold the solid at the
    volume-fraction floor, at its reference density and zero pressure."""
    lo, hi = (-0.13, -0.13, 0.0), (0.13, 0.13, 1.0)
    grid = (n, n, 1)
    mats = [dict(STEEL_304L if mat is None else mat)]

    def ind(X, Y, Z):
        return X * X + Y * Y <= 0.1 * 0.1

    def vel(X, Y, Z):
        return [2000.0 * X, 2000.0 * Y]

    frac, u = _subsample(2, grid, lo, hi, ind, vel, mats[0]["rho0"], 1.0e-30)
    prim = _assemble(2, mats, frac, u, 0.0, grid, lo, hi)
    d = (hi[0] - lo[0]) / n
    phi0 = gaussian_field((1, n, n), (1.0, d, d), corr_len, 0.1, seed)
    bc = (("transmissive",) * 2,) * 3
    return Case("disk2d", 2, grid, lo, hi, bc, mats, prim, phi0, t_end,
                cfl=0.4, seed_nu=0.99)


def spall_strip(dim, n_long=100, n_trans=8, bump=0.5e-3, v=200.0, seed=None,
                t_end=3.0e-6):
    """Plate impact on a 2D or 3D strip, for fracture checks off the 1D line:
    the 1D spall workload (10 mm, copper with gate pressure -1.5 GPa, free
    x-ends, phi0 ~ U(0.95, 1.05) per cell) widened to n_trans cells of the
    same size in y (and z), periodic there.  The flyer's impact face is
    curved, x < 2 mm + bump cos(2 pi y / W) (cos of y and z in 3D), so the
    spall plane and the faces it opens vary across the strip."""
    dx = 0.01 / n_long
    W = n_trans * dx
    lo = (0.0, 0.0, 0.0)
    hi = (0.01, W if dim >= 2 else 1.0, W if dim >= 3 else 1.0)
    grid = (n_long, n_trans if dim >= 2 else 1, n_trans if dim >= 3 else 1)
    mats = [_copper(-1.5e9)]

    def face(Y, Z):
        c = np.cos(2 * np.pi * Y / W)
        if dim >= 3:
            c = 0.5 * (c + np.cos(2 * np.pi * Z / W))
        return 0.002 + bump * c

    def ind(X, Y, Z):
        return np.ones_like(X, dtype=bool)

    def vel(X, Y, Z):
        out = [np.where(X < face(Y, Z), v, 0.0)]
        out += [np.zeros_like(X)] * (dim - 1)
        return out

    frac, u = _subsample(dim, grid, lo, hi, ind, vel, mats[0]["rho0"], 1.0)
    prim = _assemble(dim, mats, frac, u, P_ATM, grid, lo, hi)
    sd = CONFIG_SEEDS[1] + 100 * dim if seed is None else seed
    phi0 = uniform_field((grid[2], grid[1], grid[0]), 0.05, sd)
    bc = (("free", "free"),) + tuple(
        ("periodic", "periodic") if k < dim else ("transmissive",) * 2
        for k in (1, 2))
    return Case(f"spall{dim}d_strip", dim, grid, lo, hi, bc, mats, prim, phi0,
                t_end)


def uniform_case(dim, n, mats, phi, rho, u, p, bc="periodic", vbar=None,
                 phi0=1.0, lo=None, hi=None, t_end=1.0):
    """A spatially uniform primitive state (used for invariance checks)."""
    nx, ny, nz = n
    lo = lo or (0.0, 0.0, 0.0)
    hi = hi or tuple(1e-3 * n[k] if k < dim else 1.0 for k in range(3))
    shp = (nz, ny, nx)
    solids = [l for l, m in enumerate(mats) if m["kind"] == "solid"]
    rows = [np.full(shp, v) for v in phi] + [np.full(shp, v) for v in rho]
    for _ in solids:
        rows += [np.zeros(shp), np.zeros(shp)]
    rows += [np.full(shp, u[k]) for k in range(dim)]
    rows.append(np.full(shp, p))
    comps = vbar_components(dim)
    for (i, j) in comps:
        val = (1.0 if i == j else 0.0) if vbar is None else vbar[i][j]
        rows.append(np.full(shp, val))
    cx, cy, cz = _centres(n, lo, hi)
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    rows += [X, Y, Z][:dim]
    prim = np.stack(rows).astype(np.float64)
    bcs = tuple((bc, bc) if k < dim else ("transmissive", "transmissive")
                for k in range(3))
    return Case("uniform", dim, tuple(n), lo, hi, bcs, mats, prim,
                np.full(shp, float(phi0)), t_end)


def mass_edges(lo=1.0e-6, hi=10.0, per_decade=4):
    """Log-spaced fragment-mass edges (kg per metre of depth in 2D) for the
    cumulative fragment-mass histograms of the ring workloads."""
    n = int(round(np.log10(hi / lo) * per_decade)) + 1
    return [float(v) for v in np.geomspace(lo, hi, n)]


# tiny and one-cell-wide grids: (dim, cells, boundary kind)
DEGENERATE_GRIDS = [(2, (1, 9, 1), "transmissive"), (2, (9, 1, 1), "free"),
                    (2, (3, 3, 1), "transmissive"), (2, (2, 5, 1), "periodic"),
                    (1, (1, 1, 1), "transmissive"), (1, (3, 1, 1), "free"),
                    (3, (1, 1, 6), "transmissive"), (3, (2, 3, 2), "periodic")]


def degenerate_case(dim, n, bc, seed=5):
    """Copper/gas mixture on a tiny grid with a seeded velocity and
    volume-fraction field."""
    c = uniform_case(dim, n, [COPPER, GAS], [0.7, 0.3], [8930.0, 1.0],
                     [0.0] * dim, 1e5, bc=bc)
    rng = np.random.default_rng(seed)
    nm = len(c.mats)
    shape = c.prim[0].shape
    mom0 = 2 * nm + 2                       # first velocity row (one solid)
    c.prim[mom0] = 50.0 * rng.standard_normal(shape)
    c.prim[0] = 0.7 + 0.2 * rng.random(shape)
    c.prim[1] = 1.0 - c.prim[0]
    return c

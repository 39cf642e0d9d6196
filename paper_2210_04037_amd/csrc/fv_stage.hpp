// One SSP-RK3 stage of the hyperbolic update on an LDS tile, plus the source
// step and CFL reduction fused into the third stage.
//
// A block owns a TX x TY tile of output cells.  Phases (barriers between):
//   1 load   : every tile cell and its two-cell halo is read from HBM once,
//              converted to primitives and stored in LDS (structure of
//              arrays, one row per variable);
//   2 faces  : per direction, every face of the tile is computed exactly once
//              (MUSCL + HLLC + void-opening modifier) into an LDS face buffer;
//   3 gather : each thread adds the two faces of its own cell in that
//              direction to its update accumulator (registers);
//   4 finish : RK combination, volume-fraction clamp, and in stage 3 the
//              plastic/damage source step, the non-physical check and the
//              block maximum of the CFL wave-speed sum.
// The phases are written as per-thread functions so that the same code can
// be stepped on the CPU; on the GPU they run inside stage_kernel.
#pragma once

#include "fv_core.hpp"

namespace fv {

enum { BC_TRANSMISSIVE = 0, BC_FREE = 1, BC_PERIODIC = 2 };

// relative band of a stationary contact, per arithmetic precision
constexpr double TIE_REL64 = 1.0e-12;
constexpr double TIE_REL32 = 1.0e-6;

// Brick traversal of the 3D y- and z-face passes: a block of 256 threads
// covers 64 positions along x by 4 along the other transverse direction, and
// consecutive block numbers step along the face direction first, so the cell
// planes a brick's stencil reaches are still in the XCD's L2 for the next
// block (a 256^2 plane of primitives is larger than one XCD's L2).
constexpr int BRX = 64, BRY = 4;
FV_HD int64_t brick_blocks(int n_t, int n_u, int n_s) {
  // n_t: cells along x, n_u: along the other transverse direction,
  // n_s: positions along the stepping direction
  return (int64_t)((n_t + BRX - 1) / BRX) * ((n_u + BRY - 1) / BRY) * n_s;
}
// position of thread tid of brick block b: x, transverse u, step s;
// false past the domain
FV_HD bool brick_pos(int64_t b, int tid, int n_t, int n_u, int n_s, int& x, int& u, int& s) {
  s = (int)(b % n_s);
  const int64_t br = b / n_s;
  const int nbx = (n_t + BRX - 1) / BRX;
  x = (int)(br % nbx) * BRX + tid % BRX;
  u = (int)(br / nbx) * BRY + tid / BRX;
  return x < n_t && u < n_u;
}

// Per-instance descriptor (device memory).
struct Inst {
  void* U;          // state (caller-owned), in/out
  void* U1;         // stage-1 result (workspace)
  void* U2;         // stage-2 result (workspace)
  const void* phi0; // perturbation field on the initial mesh
  double* bacc;     // outward boundary flux accumulators
  void* Wb;         // 3D: primitives of every cell (workspace)
  void* Acc;        // 3D: per-cell divergence summed by the face passes (workspace)
  double* dts;      // dt state, see DTS_* below
  int n[3];
  int tiles[3];
  int bc[3][2];
  int nblocks;
  int bacc_off[6];  // offset (in doubles) of each boundary side's slots
  double lo[3];
  double dx[3];
  int64_t ncell;
};

// dt state of an instance (doubles).  First line: t[2] (DTS_T), t_end,
// dt_fixed, flags.  The CFL inverse of each parity is the maximum of
// DTS_NSLOT partial maxima, each on a 128-byte line of its own: a block
// folds its maximum into the slot of the XCD it runs on with an integer
// atomicMax on the bits (an unsigned max of non-negative doubles is their
// floating max).  A single address would take the atomics of every block of
// a launch one after another.
enum { DTS_T = 2, DTS_TEND = 4, DTS_DTFIX = 5, DTS_FLAG = 6, DTS_NSLOT = 8,
       DTS_LINE = 16, DTS_SIZE = DTS_LINE * (1 + 2 * DTS_NSLOT) };
// slot k of parity q
FV_HD int dts_slot(int q, int k) { return DTS_LINE * (1 + q * DTS_NSLOT + k); }
// CFL inverse of parity q
FV_HD double dts_dtinv(const double* dts, int q) {
  double m = dts[dts_slot(q, 0)];
  for (int k = 1; k < DTS_NSLOT; ++k) m = m > dts[dts_slot(q, k)] ? m : dts[dts_slot(q, k)];
  return m;
}
// The words of parity q a stage launch reads: its time, its CFL inverse, the
// fixed dt and the end time.  Earlier launches wrote them and a launch writes
// only parity 1 - q and the flag, so on the device they are read as
// wave-uniform global words, which the compiler turns into scalar loads.
FV_HD void read_dt_state(const double* dts, int q, double& t, double& dtinv, double& dtfix,
                         double& tend) {
#if defined(__HIP_DEVICE_COMPILE__)
  using GD = __attribute__((address_space(1))) const double;
  GD* d = (GD*)wave_uniform(dts);
#else
  const double* d = dts;
#endif
  t = d[DTS_T + q];
  dtinv = d[dts_slot(q, 0)];
  for (int k = 1; k < DTS_NSLOT; ++k) dtinv = dtinv > d[dts_slot(q, k)] ? dtinv : d[dts_slot(q, k)];
  dtfix = d[DTS_DTFIX];
  tend = d[DTS_TEND];
}
// the slots of parity q hold v (first slot) and nothing else
FV_HD void dts_set_dtinv(double* dts, int q, double v) {
  for (int k = 0; k < DTS_NSLOT; ++k) dts[dts_slot(q, k)] = k == 0 ? v : 0.0;
}
enum { FLAG_NONPHYS = 1 };

// A tile of TX x TY cells worked on by NTH threads (NTH >= TX * TY): thread
// tid < TX * TY owns interior cell tid; every thread takes face items, so a
// thread count at or above the face count of each direction computes a
// direction's faces in one pass.
template <int DIM, int TX, int TY, int NTH = TX * TY>
struct Tile {
  static_assert(NTH >= TX * TY, "a tile needs a thread per interior cell");
  static constexpr int HX = TX + 4;
  static constexpr int HY = DIM >= 2 ? TY + 4 : 1;
  static constexpr int NCELL = HX * HY;
  static constexpr int NT = NTH;
  static constexpr int NOWN = TX * TY;
  static constexpr int NFX = (TX + 1) * TY;
  static constexpr int NFY = DIM >= 2 ? TX * (TY + 1) : 0;
  static constexpr int NFACE = NFX > NFY ? NFX : NFY;
  // halo ring: tile cells outside the TX x TY interior
  static constexpr int NHALO = NCELL - NOWN;
  FV_HD static int cell(int hx, int hy) { return hy * HX + hx; }
  // tile cell of halo index h (rows below and above the interior first, then
  // the two columns on each side of every interior row)
  FV_HD static int halo_cell(int h) {
    if (DIM == 1) return h < 2 ? h : TX + h;
    if (h < 2 * HX) return h;
    if (h < 4 * HX) return cell(h % HX, TY + 2 + (h - 2 * HX) / HX);
    const int r = h - 4 * HX, c = r % 4;
    return cell(c < 2 ? c : TX + c, 2 + r / 4);
  }
  // tile cell of the interior cell owned by thread tid
  FV_HD static int own(int tid) {
    return DIM >= 2 ? cell(tid % TX + 2, tid / TX + 2) : tid + 2;
  }
};

// EXT 0: the build for runs without the extended closures (Steinberg,
// Burakovsky-Preston, Johnson-Cook, the simplified damage law), THINC and the
// driver, whose branches are compiled out; results are the same bits.
template <int DIM, int NM, int NS, class T, class C, int TX, int TY, int NTH = TX * TY,
          int EXT = 1>
struct Stage {
  static constexpr bool kExt = EXT != 0;
  using L = Lay<DIM, NM, NS>;
  using TL = Tile<DIM, TX, TY, NTH>;
  static constexpr int S = L::S;
  static constexpr int NW = L::NW;
  static constexpr int NQ = L::NQ;
  static constexpr int NC = L::NC;

  // LDS layout: W[NW][NCELL] then FB[NQ][NFACE] (both of type C)
  static constexpr size_t smem_elems() {
    return (size_t)NW * TL::NCELL + (size_t)NQ * TL::NFACE;
  }
  static constexpr size_t smem_bytes() { return smem_elems() * sizeof(C); }

  struct Ctx {
    const Inst* I;
    Params P;
    int stage;      // 1, 2, 3
    bool dry;       // timing run: no boundary accumulation
    int parity;     // step & 1
    int bx, by;     // tile coordinates
    C dt;
    double tn;      // time at the end of the step (t + dt)
    const T* src;   // stage input
    const T* base;  // U^n
    T* out;         // stage output
  };

  // critical-damage level: the advected ratio (phi rho D)/(phi rho)
  // returns D_crit only to the rounding of the storage precision T
  FV_HD static double crit_level(const MatP& m) {
    return sizeof(T) == 8 ? m.Dcrit_eff : m.Dcrit_bulk;
  }

  // FP64 island of the FP32-bulk policy: the mixture pressure inversion of a
  // cell holding a trace volume fraction, with the phasic masses, energy and
  // the sums in double (reference terms from the FP32 closures).
  FV_HD static C island_pressure(const Params& P, const C* U, const Mix<NM, NS, C>& mx) {
    double rho = 0, xi = 0;
#pragma unroll
    for (int l = 0; l < NM; ++l) {
      rho += m_max((double)U[L::MASS + l], 0.0);
      xi += (double)U[L::PHI + l] * (kExt && P.mat[l].bp ? (double)mx.t[l].invG : P.mat[l].invGamma);
    }
    double m2 = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) m2 += (double)U[L::MOM + k] * (double)U[L::MOM + k];
    double th = (double)U[L::ENE] - 0.5 * m2 / rho, cold = 0;
#pragma unroll
    for (int l = 0; l < NM; ++l) {
      const double ph = (double)U[L::PHI + l];
      th = th - ph * (double)mx.t[l].rho_eref;
      cold = cold + ph * (double)mx.t[l].pref *
                        (kExt && P.mat[l].bp ? (double)mx.t[l].invG : P.mat[l].invGamma);
    }
    return (C)((m_max(th, 0.0) + cold) / xi);
  }

  // Cell index along a direction of n cells for any g: the face stencils
  // reach two cells past each side, and a tile wider than a small grid
  // reaches further, so a periodic direction wraps modulo n.
  FV_HD static int map_index(int g, int n, int bclo, int bchi) {
    if (g < 0) return bclo == BC_PERIODIC ? (n - 1) - (-g - 1) % n : 0;
    if (g >= n) return bchi == BC_PERIODIC ? g % n : n - 1;
    return g;
  }

  // ---------------------------------------------------------------- phase 1
  // global cell of tile cell tc (ghost cells mapped by the boundary kind)
  FV_HD static int64_t tile_global(const Ctx& cx, int tc) {
    const Inst& I = *cx.I;
    const int hx = tc % TL::HX;
    const int hy = tc / TL::HX;
    const int gx = map_index(cx.bx * TX + hx - 2, I.n[0], I.bc[0][0], I.bc[0][1]);
    int gy = 0;
    if (DIM >= 2) gy = map_index(cx.by * TY + hy - 2, I.n[1], I.bc[1][0], I.bc[1][1]);
    return (int64_t)gy * I.n[0] + gx;
  }

  // Element g of field f of an instance's state.  In 1D and 2D a field holds
  // at most 4 GiB (checked when a context is made), so the cell's byte offset
  // within it fits 32 bits.  On the device the field's base is then made a
  // wave-uniform global address: each access is a global load or store with
  // a scalar base and a 32-bit lane offset, not a flat access with a 64-bit
  // address per lane.
  static constexpr bool OFF32 = DIM <= 2;
  FV_HD static T ld(const T* base, int f, int64_t ncell, int64_t g) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (OFF32) {
      using GB = __attribute__((address_space(1))) const char;
      GB* fb = (GB*)wave_uniform(base + (int64_t)f * ncell);
      return *(__attribute__((address_space(1))) const T*)(fb + (uint32_t)g * (uint32_t)sizeof(T));
    }
#endif
    return base[(int64_t)f * ncell + g];
  }
  FV_HD static void st(T* base, int f, int64_t ncell, int64_t g, T v) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (OFF32) {
      using GB = __attribute__((address_space(1))) char;
      GB* fb = (GB*)wave_uniform(base + (int64_t)f * ncell);
      *(__attribute__((address_space(1))) T*)(fb + (uint32_t)g * (uint32_t)sizeof(T)) = v;
      return;
    }
#endif
    base[(int64_t)f * ncell + g] = v;
  }

  FV_HD static void load_state(const Ctx& cx, const T* src, int64_t g, C* U) {
    const Inst& I = *cx.I;
#pragma unroll
    for (int f = 0; f < S; ++f) U[f] = (C)ld(src, f, I.ncell, g);
  }

  FV_HD static void load_cell(const Ctx& cx, C* sm, int tc) {
    cell_prims<int>(cx, tile_global(cx, tc), sm, TL::NCELL, tc);
  }

  // Primitive and derived values of cell g of the stage input, stored at
  // W[v * wstride + tc] (an LDS tile, or a full-grid buffer in HBM).
  // VXS (the 3D passes): the stretch and coordinate rows are not copied;
  // the faces read them from the stage-input state, which holds the same
  // values
  template <class IDX, bool VXS = false>
  FV_HD static void cell_prims(const Ctx& cx, int64_t g, C* sm, IDX wstride, IDX tc) {
    C U[S];
    load_state(cx, cx.src, g, U);
    prims_of<IDX, VXS>(cx, U, sm, wstride, tc);
  }

  // the same from the cell's stage-input values already in registers
  template <class IDX, bool VXS = false>
  FV_HD static void prims_of(const Ctx& cx, const C* U, C* sm, IDX wstride, IDX tc) {
    C* W = sm;
    C phi[NM], rho_l[NM], mass[NM], D[NS > 0 ? NS : 1], eps[NS > 0 ? NS : 1];
    C rho = 0;
#pragma unroll
    for (int l = 0; l < NM; ++l) {
      phi[l] = U[L::PHI + l];
      mass[l] = m_max(U[L::MASS + l], (C)0);
      rho_l[l] = mass[l] / phi[l];
      rho += mass[l];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const C ms = U[L::MASS + s];
      eps[s] = ms > (C)0 ? U[L::HIST + 2 * s] / ms : (C)0;
      D[s] = ms > (C)0 ? U[L::HIST + 2 * s + 1] / ms : (C)0;
    }
    C u[3] = {0, 0, 0};
    C ke = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) { u[k] = U[L::MOM + k] / rho; ke += u[k] * u[k]; }
    const C rho_e = U[L::ENE] - (C)0.5 * rho * ke;
    C V[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int q = 0; q < L::NV; ++q) V[vb_i<DIM>(q)][vb_j<DIM>(q)] = U[L::VB + q];
    C H[3][3];
    hencky<DIM, C>(V, H);
    const C J2 = J2_of<DIM, C>(H);
    Mix<NM, NS, C> mx;
    mix_terms<NM, NS, C, kExt>(cx.P, phi, rho_l, D, J2, mx);
    C p;
    bool island = false;
    if (sizeof(C) == 4) {
#pragma unroll
      for (int l = 0; l < NM; ++l) island = island || phi[l] < cst<C>(cx.P.phi_fp64_cut, cx.P.f_phi_fp64_cut);
    }
    if (island) p = island_pressure(cx.P, U, mx);
    else p = mix_pressure<NM, NS, C>(cx.P, phi, mx, rho_e);
    C Gmix = 0;
#pragma unroll
    for (int l = 0; l < NM; ++l) Gmix += phi[l] * mx.t[l].G;
    const C sf = solid_frac<NM, C>(phi);
    C crit = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (D[s] >= cst<C>(crit_level(cx.P.mat[s]), cx.P.mat[s].f_Dcrit_eff)) crit = 1;
    const IDX NCELL = wstride;
#pragma unroll
    for (int l = 0; l < NM; ++l) {
      W[(L::R_PHI + l) * NCELL + tc] = phi[l];
      W[(L::R_RHO + l) * NCELL + tc] = rho_l[l];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      W[(L::R_HIST + 2 * s) * NCELL + tc] = eps[s];
      W[(L::R_HIST + 2 * s + 1) * NCELL + tc] = D[s];
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) W[(L::R_U + k) * NCELL + tc] = u[k];
    W[L::R_P * NCELL + tc] = p;
#pragma unroll
    for (int q = 0; q < L::NH; ++q) W[(L::R_H + q) * NCELL + tc] = H[hk_i<DIM>(q)][hk_j<DIM>(q)];
#pragma unroll
    for (int q = 0; q < L::NV; ++q)
      if (!VXS) W[(L::R_V + q) * NCELL + tc] = U[L::VB + q];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      if (!VXS) W[(L::W_X + k) * NCELL + tc] = U[L::XC + k];
      W[(L::W_SIG + k) * NCELL + tc] = (C)2 * Gmix * H[k][k] - sf * p;
    }
    W[L::W_CRIT * NCELL + tc] = crit;
  }

  // ---------------------------------------------------------------- phase 2
  struct Side {
    C phi[NM], rho_l[NM], eps[NS > 0 ? NS : 1], D[NS > 0 ? NS : 1];
    C u[3], p, H[3][3];
    C rho, rhoE, c, G, t[3];
    C Uc[NC];
  };

  FV_HD static void unpack_side(const Params& P, const C* w, int a, Side& s) {
#pragma unroll
    for (int l = 0; l < NM; ++l) { s.phi[l] = w[L::R_PHI + l]; s.rho_l[l] = w[L::R_RHO + l]; }
#pragma unroll
    for (int q = 0; q < NS; ++q) { s.eps[q] = w[L::R_HIST + 2 * q]; s.D[q] = w[L::R_HIST + 2 * q + 1]; }
    s.u[0] = s.u[1] = s.u[2] = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) s.u[k] = w[L::R_U + k];
    s.p = w[L::R_P];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) s.H[i][j] = 0;
#pragma unroll
    for (int q = 0; q < L::NH; ++q) {
      const int i = hk_i<DIM>(q), j = hk_j<DIM>(q);
      s.H[i][j] = w[L::R_H + q];
      s.H[j][i] = w[L::R_H + q];
    }
    const C tr = (s.H[0][0] + s.H[1][1] + s.H[2][2]) / (C)3;
    s.H[0][0] -= tr; s.H[1][1] -= tr; s.H[2][2] -= tr;
    // face EOS: energy from the reconstructed pressure
    const C J2 = J2_of<DIM, C>(s.H);
    Mix<NM, NS, C> mx;
    mix_terms<NM, NS, C, kExt>(P, s.phi, s.rho_l, s.D, J2, mx);
    C rho = 0;
#pragma unroll
    for (int l = 0; l < NM; ++l) rho += s.phi[l] * s.rho_l[l];
    s.rho = rho;
    const C rho_e = mix_energy<NM, NS, C>(P, s.phi, mx, s.p);
    s.rhoE = rho_e + (C)0.5 * rho * (s.u[0] * s.u[0] + s.u[1] * s.u[1] + s.u[2] * s.u[2]);
    C Gmix;
    s.c = mix_sound<NM, NS, C>(P, s.phi, mx, s.p, rho, Gmix);
    s.G = Gmix;
    const C sf = solid_frac<NM, C>(s.phi);
#pragma unroll
    for (int i = 0; i < 3; ++i) s.t[i] = (C)2 * Gmix * s.H[i][a] - (i == a ? sf * s.p : (C)0);
#pragma unroll
    for (int l = 0; l < NM; ++l) s.Uc[l] = s.phi[l] * s.rho_l[l];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      s.Uc[NM + 2 * q] = s.phi[q] * s.rho_l[q] * s.eps[q];
      s.Uc[NM + 2 * q + 1] = s.phi[q] * s.rho_l[q] * s.D[q];
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) s.Uc[L::C_MOM + k] = rho * s.u[k];
    s.Uc[L::C_ENE] = s.rhoE;
  }

  // physical flux U u_n - (0, 0, sigma n, u . sigma n)  (Section 2.1)
  FV_HD static void phys_flux(const Side& s, int a, C* F) {
    const C un = s.u[a];
#pragma unroll
    for (int q = 0; q < NC; ++q) F[q] = s.Uc[q] * un;
#pragma unroll
    for (int k = 0; k < DIM; ++k) F[L::C_MOM + k] -= s.t[k];
    F[L::C_ENE] -= s.u[0] * s.t[0] + s.u[1] * s.t[1] + s.u[2] * s.t[2];
  }

  // Star-region flux of side K with the contact's tangential state resolved
  // (see compute_face): mass/history chi U S*, normal momentum
  // rho* S*^2 - t_n*, tangential momentum rho* u_t** S* - t_t**, energy
  // E** S* - S* t_n* - u_t** . t_t**.
  FV_HD static void star_flux(const Side& s, int a, C SK, C Ss, C tn_star,
                              const C* ut2, const C* tt2, C work, C* Fs) {
    const C un = s.u[a];
    const C chi = (SK - un) / (SK - Ss);
    const C rs = chi * s.rho;
    const C Es = chi * (s.rhoE + (Ss - un) * (s.rho * Ss - s.t[a] / (SK - un)));
    C dke = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (k != a) dke += ut2[k] * ut2[k] - s.u[k] * s.u[k];
    const C Ess = Es + (C)0.5 * rs * dke;
#pragma unroll
    for (int q = 0; q < L::C_MOM; ++q) Fs[q] = s.Uc[q] * (chi * Ss);
#pragma unroll
    for (int k = 0; k < DIM; ++k)
      Fs[L::C_MOM + k] = k == a ? rs * Ss * Ss - tn_star : rs * ut2[k] * Ss - tt2[k];
    Fs[L::C_ENE] = Ess * Ss - Ss * tn_star - work;
  }

  // Face a of the tile: W pointers of the four stencil cells (cm, c0 | c1, c2)
  // and the face's position relative to the domain boundary.
  template <class IDX, bool VXS = false>
  FV_HD static void compute_face(const Ctx& cx, const C* sm, IDX wstride, int a, IDX cm,
                                 IDX c0, IDX c1, IDX c2, int gface, IDX fslot, IDX fstride,
                                 int64_t bslot, C* fb) {
    const Inst& I = *cx.I;
    const Params& P = cx.P;
    const IDX NCELL = wstride;
    const C* W = sm;
    // stretch and coordinate rows: the primitives', or (VXS) the stage
    // input's rows of the same cells and stride
    static_assert(!VXS || sizeof(T) == sizeof(C), "state and compute types differ");
    const C* VX = VXS ? (const C*)cx.src : sm;
    constexpr int RV = VXS ? L::VB : L::R_V, RX = VXS ? L::XC : L::W_X;
    // the rows the face states need; the stretch rows (the last NV) are
    // reconstructed below, only on the side the face takes them from
    C wl[L::NR], wr[L::NR];
#pragma unroll
    for (int v = 0; v < L::R_V; ++v) {
      const C qm = W[v * NCELL + cm], q0 = W[v * NCELL + c0];
      const C q1 = W[v * NCELL + c1], q2 = W[v * NCELL + c2];
      wl[v] = q0 + (C)0.5 * van_leer(q0 - qm, q1 - q0);
      wr[v] = q1 - (C)0.5 * van_leer(q1 - q0, q2 - q1);
    }
    // THINC sharpening of the volume fractions (the first NM rows): the
    // upper face of the cell below and the lower face of the cell above
    if (kExt && P.thinc_beta > 0.0) {
      const C beta = cst<C>(P.thinc_beta, P.f_thinc_beta);
      const C tb = cst<C>(P.thinc_tb, P.f_thinc_tb), sh = cst<C>(P.thinc_sech, P.f_thinc_sech);
#pragma unroll
      for (int v = 0; v < NM; ++v) {
        const C qm = W[v * NCELL + cm], q0 = W[v * NCELL + c0];
        const C q1 = W[v * NCELL + c1], q2 = W[v * NCELL + c2];
        C t;
        if (thinc_cell<C>(qm, q0, q1, beta, tb, sh, nullptr, &t)) wl[v] = t;
        if (thinc_cell<C>(q0, q1, q2, beta, tb, sh, &t, nullptr)) wr[v] = t;
      }
    }
    Side sL, sR;
    unpack_side(P, wl, a, sL);
    unpack_side(P, wr, a, sR);
    const C unL = sL.u[a], unR = sR.u[a];
    const C SL = m_min(unL - sL.c, unR - sR.c);
    const C SR = m_max(unL + sL.c, unR + sR.c);
    const C num = (sL.t[a] - sR.t[a]) +
                  (sL.rho * unL * (SL - unL) - sR.rho * unR * (SR - unR));
    const C den = sL.rho * (SL - unL) - sR.rho * (SR - unR);
    const C Ss = num / den;
    // contact and face speeds below TIE_REL of the largest signal speed are
    // stationary: the upwind choices take the mean of the two sides (the star
    // fluxes differ by the tangential-traction jump at a zero contact speed)
    const C tie = (C)(sizeof(C) == 8 ? TIE_REL64 : TIE_REL32) * m_max(m_abs(SL), m_abs(SR));
    // Contact tangential state from the linearised shear waves on either
    // side (impedance Z = sqrt(G rho)); free slip against a fluid.  Without
    // it the star fluxes would take one side's tangential traction,
    // upwinded by S*, which lets shear waves grow.
    const C ZL = m_sqrt(sL.G * sL.rho), ZR = m_sqrt(sR.G * sR.rho);
    const C Zs = ZL + ZR;
    C ut2[3] = {0, 0, 0}, tt2[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k == a) continue;
      if (Zs > (C)0) {
        ut2[k] = (ZL * sL.u[k] + ZR * sR.u[k] + (sR.t[k] - sL.t[k])) / Zs;
        tt2[k] = sL.t[k] + ZL * (ut2[k] - sL.u[k]);
      } else {
        ut2[k] = Ss > tie ? sL.u[k] : (Ss < -tie ? sR.u[k] : (C)0.5 * (sL.u[k] + sR.u[k]));
      }
    }
    const C tn_star = (C)0.5 * ((sL.t[a] - sL.rho * (SL - unL) * (Ss - unL)) +
                                (sR.t[a] - sR.rho * (SR - unR) * (Ss - unR)));
    C work = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (k != a) work += ut2[k] * tt2[k];
    C F[NC];
    if (SL >= (C)0) {
      phys_flux(sL, a, F);
    } else if (SR <= (C)0) {
      phys_flux(sR, a, F);
    } else if (Ss > tie) {
      star_flux(sL, a, SL, Ss, tn_star, ut2, tt2, work, F);
    } else if (Ss < -tie) {
      star_flux(sR, a, SR, Ss, tn_star, ut2, tt2, work, F);
    } else {
      C FsL[NC], FsR[NC];
      star_flux(sL, a, SL, Ss, tn_star, ut2, tt2, work, FsL);
      star_flux(sR, a, SR, Ss, tn_star, ut2, tt2, work, FsR);
#pragma unroll
      for (int q = 0; q < NC; ++q) F[q] = (C)0.5 * (FsL[q] + FsR[q]);
    }
    C uf = SL > (C)0 ? unL : (SR < (C)0 ? unR : Ss);
    C ut[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) ut[k] = SL > (C)0 ? sL.u[k] : (SR < (C)0 ? sR.u[k] : ut2[k]);
    // upwinded geometric face values: the volume fractions here; the
    // stretch and the coordinates once the side they come from is known
    const bool up = uf > tie, dn = uf < -tie;
    C phif[NM], Vf[L::NV], Xf[DIM];
#pragma unroll
    for (int l = 0; l < NM; ++l)
      phif[l] = up ? sL.phi[l] : (dn ? sR.phi[l] : (C)0.5 * (sL.phi[l] + sR.phi[l]));
    // side of the stretch and coordinate values: 0 left, 1 right, 2 the
    // mean of both, 3 none (an opened or closed face, whose neighbours use
    // their own centre values)
    int pick = up ? 0 : (dn ? 1 : 2);
    // one-sided free-surface velocities
    const C usL = unL - sL.t[a] / (sL.rho * sL.c);
    const C usR = unR + sR.t[a] / (sR.rho * sR.c);
    C os = 0;
    const int n = I.n[a];
    const bool lo_b = gface == 0, hi_b = gface == n;
    const bool periodic = I.bc[a][0] == BC_PERIODIC;
    if ((!lo_b && !hi_b) || periodic) {
      // void-opening modifier (Section 3.1): next to a critically damaged
      // cell, when the pair is in tension
      const bool crit = W[L::W_CRIT * NCELL + c0] > (C)0 || W[L::W_CRIT * NCELL + c1] > (C)0;
      const C tens = W[(L::W_SIG + a) * NCELL + c0] + W[(L::W_SIG + a) * NCELL + c1];
      // open only while the two free surfaces separate
      const C band = (C)(sizeof(T) == 8 ? cx.P.tens_band : cx.P.tens_band_bulk);
      if (crit && tens > band && usL <= usR) {
        // no traction; a side whose one-sided velocity points through the
        // face carries its material into the neighbour, else void enters it
        os = 1;
        const C oL = usL > (C)0 ? usL : (C)0;
        const C oR = usR < (C)0 ? usR : (C)0;
#pragma unroll
        for (int q = 0; q < NC; ++q) F[q] = sL.Uc[q] * oL + sR.Uc[q] * oR;
        // opened faces store the shared volume-fraction flux in Q_PHI
#pragma unroll
        for (int l = 0; l < NM; ++l) phif[l] = sL.phi[l] * oL + sR.phi[l] * oR;
        pick = 3;
      }
    } else if ((lo_b && I.bc[a][0] == BC_FREE) || (hi_b && I.bc[a][1] == BC_FREE)) {
      const Side& sK = lo_b ? sR : sL;
      const C us = lo_b ? usR : usL;
      const bool outward = lo_b ? us < (C)0 : us > (C)0;
      if (outward) {
        // material leaves at the free-surface velocity, no traction
#pragma unroll
        for (int q = 0; q < NC; ++q) F[q] = sK.Uc[q] * us;
        uf = us;
#pragma unroll
        for (int k = 0; k < 3; ++k) ut[k] = sK.u[k];
#pragma unroll
        for (int l = 0; l < NM; ++l) phif[l] = sK.phi[l];
        pick = lo_b ? 1 : 0;
      } else {
        os = 1;
#pragma unroll
        for (int q = 0; q < NC; ++q) F[q] = 0;
#pragma unroll
        for (int l = 0; l < NM; ++l) phif[l] = 0;
        pick = 3;
      }
    }
    // The left value of a stencil (qm, q0 | q1, q2) is q0 + vl(q0-qm, q1-q0)/2
    // and the right one q1 - vl(q1-q0, q2-q1)/2; van Leer's mean is
    // symmetric and odd, so the right value is the left formula on the
    // mirrored stencil (q2, q1, q0), bit for bit, and one pass over the
    // picked stencil serves either side.  The mean takes the right side in
    // a second pass.
    {
      const bool rt = pick == 1;
      const IDX ia = rt ? c2 : cm, ib = rt ? c1 : c0, ic = rt ? c0 : c1;
      const C ext = (C)(I.dx[a] * I.n[a]);
      const C weps = cst<C>(P.weno_eps, P.f_weno_eps) * ext * ext;
#pragma unroll
      for (int q = 0; q < L::NV; ++q) Vf[q] = 0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) Xf[k] = 0;
      if (pick != 3) {
#pragma unroll
        for (int q = 0; q < L::NV; ++q) {
          const C qa = VX[(RV + q) * NCELL + ia], qb = VX[(RV + q) * NCELL + ib];
          const C qc = VX[(RV + q) * NCELL + ic];
          Vf[q] = qb + (C)0.5 * van_leer(qb - qa, qc - qb);
        }
#pragma unroll
        for (int k = 0; k < DIM; ++k)
          Xf[k] = weno3_left(VX[(RX + k) * NCELL + ia], VX[(RX + k) * NCELL + ib],
                             VX[(RX + k) * NCELL + ic], weps);
      }
      if (pick == 2) {
#pragma unroll
        for (int q = 0; q < L::NV; ++q) {
          const C q0 = VX[(RV + q) * NCELL + c0], q1 = VX[(RV + q) * NCELL + c1];
          const C q2 = VX[(RV + q) * NCELL + c2];
          Vf[q] = (C)0.5 * (Vf[q] + (q1 - (C)0.5 * van_leer(q1 - q0, q2 - q1)));
        }
#pragma unroll
        for (int k = 0; k < DIM; ++k)
          Xf[k] = (C)0.5 * (Xf[k] + weno3_left(VX[(RX + k) * NCELL + c2],
                                                VX[(RX + k) * NCELL + c1],
                                                VX[(RX + k) * NCELL + c0], weps));
      }
    }
    // outward boundary flux accumulation, RK3 weights 1/6, 1/6, 2/3
    if (!periodic && (lo_b || hi_b) && !cx.dry) {
      // the weights in double, as the cell update applies them
      const double wdt = (cx.stage == 3 ? 2.0 / 3.0 : 1.0 / 6.0) * (double)cx.dt;
      const double sgn = lo_b ? -1.0 : 1.0;
      double* acc = I.bacc + I.bacc_off[2 * a + (hi_b ? 1 : 0)] + (int64_t)bslot * NC;
#pragma unroll
      for (int q = 0; q < NC; ++q) acc[q] += wdt * (sgn * (double)F[q]);
    }
    // store
    const IDX NF = fstride;
#pragma unroll
    for (int q = 0; q < NC; ++q) fb[(L::Q_F + q) * NF + fslot] = F[q];
    fb[L::Q_UF * NF + fslot] = uf;
    {
      int k2 = 0;
#pragma unroll
      for (int k = 0; k < DIM; ++k)
        if (k != a) { fb[(L::Q_UT + k2) * NF + fslot] = ut[k]; ++k2; }
    }
#pragma unroll
    for (int l = 0; l < NM; ++l) fb[(L::Q_PHI + l) * NF + fslot] = phif[l];
#pragma unroll
    for (int k = 0; k < DIM; ++k) fb[(L::Q_X + k) * NF + fslot] = Xf[k];
#pragma unroll
    for (int q = 0; q < L::NV; ++q) fb[(L::Q_V + q) * NF + fslot] = Vf[q];
    fb[L::Q_OS * NF + fslot] = os;
    fb[L::Q_USL * NF + fslot] = usL;
    fb[L::Q_USR * NF + fslot] = usR;
  }

  // Face item -> stencil and slot.  Returns false if the face lies outside
  // the domain (partial tiles).
  FV_HD static bool face_item(const Ctx& cx, int a, int item, int& cm, int& c0,
                              int& c1, int& c2, int& gface, int& fslot,
                              int& bslot) {
    const Inst& I = *cx.I;
    if (a == 0) {
      const int fx = item % (TX + 1), ty = item / (TX + 1);
      if (ty >= TY) return false;
      gface = cx.bx * TX + fx;
      const int gy = cx.by * TY + ty;
      if (gface > I.n[0] || (DIM >= 2 && gy >= I.n[1])) return false;
      const int hy = DIM >= 2 ? ty + 2 : 0;
      cm = TL::cell(fx, hy); c0 = TL::cell(fx + 1, hy);
      c1 = TL::cell(fx + 2, hy); c2 = TL::cell(fx + 3, hy);
      fslot = ty * (TX + 1) + fx;
      bslot = DIM >= 2 ? gy : 0;
      return true;
    }
    const int tx = item % TX, fy = item / TX;
    if (fy > TY) return false;
    gface = cx.by * TY + fy;
    const int gx = cx.bx * TX + tx;
    if (gface > I.n[1] || gx >= I.n[0]) return false;
    const int hx = tx + 2;
    cm = TL::cell(hx, fy); c0 = TL::cell(hx, fy + 1);
    c1 = TL::cell(hx, fy + 2); c2 = TL::cell(hx, fy + 3);
    fslot = fy * TX + tx;
    bslot = gx;
    return true;
  }

  FV_HD static int face_items(int a) { return a == 0 ? TL::NFX : TL::NFY; }

  // ---------------------------------------------------------------- phase 3
  // contribution of one face to the owning cell (side 0: the cell is the
  // face's left neighbour, side 1: its right neighbour)
  struct FaceC {
    C F[NC];
    C vel;
    C phif[NM];
    C Xfl[DIM];
    C Vfl[L::NV];
    C row[3];
  };

  template <class IDX>
  FV_HD static void face_contrib(const C* fb, IDX fslot, IDX fstride, int a, int side,
                                 const C* Xc, const C Vc[3][3], const C* uc,
                                 FaceC& o) {
    const IDX NF = fstride;
#pragma unroll
    for (int q = 0; q < NC; ++q) o.F[q] = fb[(L::Q_F + q) * NF + fslot];
    const C os = fb[L::Q_OS * NF + fslot];
    C uv[3];
    C Vm[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    if (os == (C)0) {
      const C uf = fb[L::Q_UF * NF + fslot];
      o.vel = uf;
      uv[0] = uv[1] = uv[2] = 0;
      int k2 = 0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        if (k == a) uv[k] = uf;
        else { uv[k] = fb[(L::Q_UT + k2) * NF + fslot]; ++k2; }
      }
#pragma unroll
      for (int l = 0; l < NM; ++l) o.phif[l] = fb[(L::Q_PHI + l) * NF + fslot] * uf;
#pragma unroll
      for (int k = 0; k < DIM; ++k) o.Xfl[k] = fb[(L::Q_X + k) * NF + fslot] * uf;
#pragma unroll
      for (int q = 0; q < L::NV; ++q) Vm[vb_i<DIM>(q)][vb_j<DIM>(q)] = fb[(L::Q_V + q) * NF + fslot];
    } else {
      const C us = fb[(side == 0 ? L::Q_USL : L::Q_USR) * NF + fslot];
      o.vel = us;
      uv[0] = uc[0]; uv[1] = uc[1]; uv[2] = uc[2];
      uv[a] = us;
#pragma unroll
      for (int l = 0; l < NM; ++l) o.phif[l] = fb[(L::Q_PHI + l) * NF + fslot];
#pragma unroll
      for (int k = 0; k < DIM; ++k) o.Xfl[k] = Xc[k] * us;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Vm[i][j] = Vc[i][j];
    }
#pragma unroll
    for (int q = 0; q < L::NV; ++q) {
      const int i = vb_i<DIM>(q), j = vb_j<DIM>(q);
      o.Vfl[q] = Vm[i][j] * uv[a] - Vm[a][j] * uv[i];
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) o.row[j] = Vm[a][j];
  }

  // own cell of this thread inside the tile
  FV_HD static bool own_cell(const Ctx& cx, int tid, int& tx, int& ty, int64_t& g) {
    const Inst& I = *cx.I;
    if (NTH > TL::NOWN && tid >= TL::NOWN) return false;
    tx = tid % TX;
    ty = tid / TX;
    const int gx = cx.bx * TX + tx;
    const int gy = cx.by * TY + ty;
    if (gx >= I.n[0]) return false;
    if (DIM >= 2 && gy >= I.n[1]) return false;
    g = DIM >= 2 ? (int64_t)gy * I.n[0] + gx : gx;
    return true;
  }

  FV_HD static void gather(const Ctx& cx, const C* sm, const C* fb, int a,
                           int tx, int ty, C* acc) {
    const int NCELL = TL::NCELL;
    const C* W = sm;
    const int hx = tx + 2, hy = DIM >= 2 ? ty + 2 : 0;
    const int cc = TL::cell(hx, hy);
    C Xc[DIM], uc[3] = {0, 0, 0}, phic[NM];
    C Vc[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int k = 0; k < DIM; ++k) { Xc[k] = W[(L::W_X + k) * NCELL + cc]; uc[k] = W[(L::R_U + k) * NCELL + cc]; }
#pragma unroll
    for (int l = 0; l < NM; ++l) phic[l] = W[(L::R_PHI + l) * NCELL + cc];
#pragma unroll
    for (int q = 0; q < L::NV; ++q) Vc[vb_i<DIM>(q)][vb_j<DIM>(q)] = W[(L::R_V + q) * NCELL + cc];
    int fm, fp;
    if (a == 0) { fm = ty * (TX + 1) + tx; fp = fm + 1; }
    else { fm = ty * TX + tx; fp = fm + TX; }
    FaceC m, p;
    face_contrib<int>(fb, fm, TL::NFACE, a, 1, Xc, Vc, uc, m);
    face_contrib<int>(fb, fp, TL::NFACE, a, 0, Xc, Vc, uc, p);
    gather_dir(cx, a, m, p, Xc, uc, phic, Vc, acc);
  }

  // accumulate the divergence of direction a from its two faces (m: the
  // lower face, p: the upper one) and the cell's own values
  FV_HD static void gather_dir(const Ctx& cx, int a, const FaceC& m, const FaceC& p,
                               const C* Xc, const C* uc, const C* phic,
                               const C Vc[3][3], C* acc) {
    const C inv = (C)1 / (C)cx.I->dx[a];
    const C div = (p.vel - m.vel) * inv;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      int f;
      if (q < NM) f = L::MASS + q;
      else if (q < NM + 2 * NS) f = L::HIST + (q - NM);
      else if (q < L::C_ENE) f = L::MOM + (q - L::C_MOM);
      else f = L::ENE;
      acc[f] += -(p.F[q] - m.F[q]) * inv;
    }
#pragma unroll
    for (int l = 0; l < NM; ++l)
      acc[L::PHI + l] += -(p.phif[l] - m.phif[l]) * inv + phic[l] * div;
#pragma unroll
    for (int k = 0; k < DIM; ++k)
      acc[L::XC + k] += -(p.Xfl[k] - m.Xfl[k]) * inv + Xc[k] * div;
#pragma unroll
    for (int q = 0; q < L::NV; ++q) {
      const int i = vb_i<DIM>(q), j = vb_j<DIM>(q);
      const C beta = (p.row[j] - m.row[j]) * inv;
      acc[L::VB + q] += -(p.Vfl[q] - m.Vfl[q]) * inv + (C)(2.0 / 3.0) * Vc[i][j] * div - uc[i] * beta;
    }
  }

  // ------------------------------------------------------- 3D face passes
  // The 3D stage takes its faces direction by direction from the primitives
  // of every cell (W, stride ncell) and sums each cell's divergence in Acc
  // (S fields, stride ncell); no face data goes through HBM.  Each face is
  // computed once (x) or once plus one face per run of MARCH cells (y, z).
  //
  // x: the faces in row order (f = row * (nx + 1) + i), in runs of XRUN + 1
  // faces that overlap by one, so that both faces of every cell fall in one
  // run.  Phase 1: face f = b * XRUN + t into slot t of fb (stride XRUN + 1).
  static constexpr int XRUN = 255;
  FV_HD static int64_t xrun_count(const Inst& I) {
    const int64_t nf = I.ncell / I.n[0] * (I.n[0] + 1);
    return (nf - 1 + XRUN - 1) / XRUN;
  }
  FV_HD static void xrun_face(const Ctx& cx, const C* W, int64_t b, int t, C* fb) {
    const Inst& I = *cx.I;
    const int nx = I.n[0];
    const int64_t nf = I.ncell / nx * (nx + 1);
    const int64_t f = b * XRUN + t;
    if (t > XRUN || f >= nf) return;
    const int i = (int)(f % (nx + 1));
    const int64_t row = f / (nx + 1);
    int64_t st[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      st[k] = row * nx + map_index(i - 2 + k, nx, I.bc[0][0], I.bc[0][1]);
    compute_face<int64_t, true>(cx, W, I.ncell, 0, st[0], st[1], st[2], st[3], i, (int64_t)t,
                          (int64_t)(XRUN + 1), row, fb);
  }
  // Phase 2: the cell between faces t and t + 1 of run b, if they bound one;
  // its x divergence starts its sum in Acc.
  FV_HD static void xrun_cell(const Ctx& cx, const C* W, int64_t b, int t, const C* fb,
                              C* accb) {
    const Inst& I = *cx.I;
    const int nx = I.n[0];
    const int64_t nc = I.ncell;
    const int64_t nf = nc / nx * (nx + 1);
    const int64_t f = b * XRUN + t;
    if (t >= XRUN || f + 1 >= nf) return;
    const int i = (int)(f % (nx + 1));
    if (i == nx) return;
    const int64_t g = f / (nx + 1) * nx + i;
    C Xc[3], uc[3], phic[NM];
    C Vc[3][3];
    own_values(cx, W, nc, g, Xc, uc, phic, Vc);
    FaceC m, p;
    face_contrib<int>(fb, t, XRUN + 1, 0, 1, Xc, Vc, uc, m);
    face_contrib<int>(fb, t + 1, XRUN + 1, 0, 0, Xc, Vc, uc, p);
    C acc[S];
#pragma unroll
    for (int q = 0; q < S; ++q) acc[q] = 0;
    gather_dir(cx, 0, m, p, Xc, uc, phic, Vc, acc);
#pragma unroll
    for (int q = 0; q < S; ++q) accb[q * nc + g] = acc[q];
  }

  // y, z: one thread per transverse position (x, u) (u = z for y, y for z)
  // and run s of MARCH cells along a.  It walks the faces s * MARCH ..
  // min(s * MARCH + MARCH, n_a) in order, keeping the lower face's record,
  // and adds each cell's divergence along a to its sum in Acc.
  static constexpr int MARCH = 16;
  FV_HD static int march_runs(const Inst& I, int a) { return (I.n[a] + MARCH - 1) / MARCH; }
  FV_HD static void march_cells(const Ctx& cx, const C* W, int a, int x, int u, int s, C* accb) {
    const Inst& I = *cx.I;
    const int nx = I.n[0], ny = I.n[1], na = I.n[a];
    const int64_t nc = I.ncell;
    const int i0 = s * MARCH, i1 = m_min(i0 + MARCH, na);
    const int64_t sa = a == 1 ? (int64_t)nx : (int64_t)nx * ny;
    const int64_t g0 = a == 1 ? (int64_t)u * nx * ny + x : (int64_t)u * nx + x;
    const int64_t bslot = (int64_t)u * nx + x;
    C lo[L::NQ], up[L::NQ];
    for (int i = i0; i <= i1; ++i) {
      int64_t st[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        st[k] = g0 + (int64_t)map_index(i - 2 + k, na, I.bc[a][0], I.bc[a][1]) * sa;
      compute_face<int64_t, true>(cx, W, nc, a, st[0], st[1], st[2], st[3], i, (int64_t)0,
                                  (int64_t)1,
                            bslot, up);
      if (i > i0) {
        const int64_t g = g0 + (int64_t)(i - 1) * sa;
        C Xc[3], uc[3], phic[NM];
        C Vc[3][3];
        own_values(cx, W, nc, g, Xc, uc, phic, Vc);
        FaceC m, p;
        face_contrib<int>(lo, 0, 1, a, 1, Xc, Vc, uc, m);
        face_contrib<int>(up, 0, 1, a, 0, Xc, Vc, uc, p);
        C acc[S];
#pragma unroll
        for (int q = 0; q < S; ++q) acc[q] = accb[q * nc + g];
        gather_dir(cx, a, m, p, Xc, uc, phic, Vc, acc);
#pragma unroll
        for (int q = 0; q < S; ++q) accb[q * nc + g] = acc[q];
      }
#pragma unroll
      for (int q = 0; q < L::NQ; ++q) lo[q] = up[q];
    }
  }

  // the centre values a cell's gather takes from the 3D primitives
  // (the coordinates and the stretch from the stage input, as the 3D faces
  // read them)
  FV_HD static void own_values(const Ctx& cx, const C* W, int64_t nc, int64_t g, C* Xc, C* uc,
                               C* phic, C Vc[3][3]) {
    const C* Us = (const C*)cx.src;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Xc[k] = Us[(L::XC + k) * nc + g];
      uc[k] = W[(L::R_U + k) * nc + g];
    }
#pragma unroll
    for (int l = 0; l < NM; ++l) phic[l] = W[(L::R_PHI + l) * nc + g];
#pragma unroll
    for (int q = 0; q < L::NV; ++q) Vc[vb_i<3>(q)][vb_j<3>(q)] = Us[(L::VB + q) * nc + g];
  }

  // ---------------------------------------------------------------- phase 4
  // Source step on the new state of one cell (FP64), Section 2.4 / 3.1 /
  // 3.2.2 readings: phi0 gather, radial return, Bonora RK4, Vbar rebuild.
  FV_HD static double phi0_gather(const Inst& I, const double* X) {
    return gather_field(I, (const T*)I.phi0, X);
  }

  // Multilinear interpolation of a cell-centred field f (one field of
  // ncell values) at position X, clamped to the span of the cell centres;
  // nested linear interpolations, x first, so a constant field is returned
  // exactly.
  FV_HD static double gather_field(const Inst& I, const T* f, const double* X) {
    int i0[3] = {0, 0, 0};
    double w[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const int nk = I.n[k];
      double s = (X[k] - (I.lo[k] + 0.5 * I.dx[k])) / I.dx[k];
      // clamped to the initial cell-centre span; a NaN coordinate (a state
      // the non-physical check flags after this step) maps to the first
      // centre, so the index below is always defined and in range
      s = s >= 0.0 ? (s > (double)(nk - 1) ? (double)(nk - 1) : s) : 0.0;
      double fl = floor(s);
      const double top = nk >= 2 ? (double)(nk - 2) : 0.0;
      if (fl > top) fl = top;
      i0[k] = (int)fl;
      w[k] = s - fl;
    }
    auto at = [&](int dx_, int dy_, int dz_) -> double {
      const int x = m_min(i0[0] + dx_, I.n[0] - 1);
      const int y = DIM >= 2 ? m_min(i0[1] + dy_, I.n[1] - 1) : 0;
      const int z = DIM >= 3 ? m_min(i0[2] + dz_, I.n[2] - 1) : 0;
      return (double)f[((int64_t)z * I.n[1] + y) * I.n[0] + x];
    };
    auto lerp = [](double a, double b, double t) { return a + t * (b - a); };
    if (DIM == 1) return lerp(at(0, 0, 0), at(1, 0, 0), w[0]);
    const double f0 = lerp(at(0, 0, 0), at(1, 0, 0), w[0]);
    const double f1 = lerp(at(0, 1, 0), at(1, 1, 0), w[0]);
    if (DIM == 2) return lerp(f0, f1, w[1]);
    const double g0 = lerp(f0, f1, w[1]);
    const double f2 = lerp(at(0, 0, 1), at(1, 0, 1), w[0]);
    const double f3 = lerp(at(0, 1, 1), at(1, 1, 1), w[0]);
    return lerp(g0, lerp(f2, f3, w[1]), w[2]);
  }

  // Lagrangian seeding of cell g (Section 3.2.1 seeding routine) from the
  // state U after the step: if the cell's void fraction exceeds seed_nu and
  // the void fraction has a gradient there (central differences, one-sided at
  // a domain side), its coordinates are extrapolated from the point probed
  // 1.5 cells towards the material, X(p) - (p - c); otherwise they are kept.
  // Xn: the cell's coordinates after seeding (DIM values).
  FV_HD static void seed_cell(const Params& P, const Inst& I, const T* U, int64_t g,
                              double* Xn) {
    const int64_t nc = I.ncell;
    int ix[3];
    {
      int64_t r = g;
      ix[0] = (int)(r % I.n[0]);
      r /= I.n[0];
      ix[1] = (int)(r % I.n[1]);
      ix[2] = (int)(r / I.n[1]);
    }
    auto nu_at = [&](int64_t h) -> double {
      double sphi = 0.0;
#pragma unroll
      for (int l = 0; l < NM; ++l) sphi += (double)U[(int64_t)(L::PHI + l) * nc + h];
      sphi = sphi < 0.0 ? 0.0 : (sphi > 1.0 ? 1.0 : sphi);
      return 1.0 - sphi;
    };
#pragma unroll
    for (int k = 0; k < DIM; ++k) Xn[k] = (double)U[(int64_t)(L::XC + k) * nc + g];
    if (!(nu_at(g) > P.seed_nu)) return;
    const int64_t stride[3] = {1, (int64_t)I.n[0], (int64_t)I.n[0] * I.n[1]};
    double grad[3] = {0.0, 0.0, 0.0}, n2 = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const int nk = I.n[k];
      if (nk < 2) continue;
      if (ix[k] == 0) grad[k] = (nu_at(g + stride[k]) - nu_at(g)) / I.dx[k];
      else if (ix[k] == nk - 1) grad[k] = (nu_at(g) - nu_at(g - stride[k])) / I.dx[k];
      else grad[k] = (nu_at(g + stride[k]) - nu_at(g - stride[k])) / (2.0 * I.dx[k]);
      n2 += grad[k] * grad[k];
    }
    if (!(n2 > 0.0)) return;
    const double nrm = sqrt(n2);
    double h = I.dx[0];
#pragma unroll
    for (int k = 1; k < DIM; ++k) h = I.dx[k] < h ? I.dx[k] : h;
    double c[3] = {0.0, 0.0, 0.0}, p[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      c[k] = I.lo[k] + (ix[k] + 0.5) * I.dx[k];
      p[k] = c[k] - 1.5 * h * grad[k] / nrm;
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k)
      Xn[k] = gather_field(I, U + (int64_t)(L::XC + k) * nc, p) - (p[k] - c[k]);
  }

  // Returns the cell's CFL sum  sum_a (|u_a| + c)/dx_a  after the source step.
  FV_HD static double source_and_cfl(const Params& P, const Inst& I, double* U, double dt,
                                     int64_t g, double tn) {
    double phi[NM], mass[NM], rho_l[NM], eps[NS > 0 ? NS : 1], D[NS > 0 ? NS : 1];
    double rho = 0;
#pragma unroll
    for (int l = 0; l < NM; ++l) {
      phi[l] = U[L::PHI + l];
      mass[l] = U[L::MASS + l] > 0.0 ? U[L::MASS + l] : 0.0;
      rho_l[l] = mass[l] / phi[l];
      rho += mass[l];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double ms = U[L::MASS + s];
      eps[s] = ms > 0.0 ? U[L::HIST + 2 * s] / ms : 0.0;
      D[s] = ms > 0.0 ? U[L::HIST + 2 * s + 1] / ms : 0.0;
    }
    double u[3] = {0, 0, 0}, ke = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) { u[k] = U[L::MOM + k] / rho; ke += u[k] * u[k]; }
    const double rho_e = U[L::ENE] - 0.5 * rho * ke;
    double V[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int q = 0; q < L::NV; ++q) V[vb_i<DIM>(q)][vb_j<DIM>(q)] = U[L::VB + q];
    double H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double Dn[NS > 0 ? NS : 1];
    // A cell whose solids are all traces has no shear stiffness: its
    // distortion is dropped (the stretch becomes the identity, on which
    // the stress does not depend) and it does no plastic work, so the
    // histories stand.  The Hencky strain, the perturbation gather and
    // the return are skipped there (most of a gas- or void-filled grid).
    bool live = false;
#pragma unroll
    for (int s = 0; s < NS; ++s) live = live || phi[s] >= PHI_TRACE;
    if (live) {
      // 3D: the eigen-decomposition of V V^T is kept, so that the return (a
      // scaling of dev H) rebuilds the stretch from the same eigenvectors
      double Qe[3][3], he[3];
      if constexpr (DIM == 3) {
        double B[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j)
            B[i][j] = V[i][0] * V[j][0] + V[i][1] * V[j][1] + V[i][2] * V[j][2];
        sym3_eig(B, Qe);
        half_log_eigs3<double>(V, B, he);
        const double mm = (he[0] + he[1] + he[2]) / 3.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) he[k] -= mm;
        sym3_compose(Qe, he, H);
      } else {
        hencky<DIM, double>(V, H);
      }
      const double J2 = J2_of<DIM, double>(H);
      Mix<NM, NS, double> mx;
      mix_terms<NM, NS, double, kExt>(P, phi, rho_l, D, J2, mx);
      const double p = mix_pressure<NM, NS, double>(P, phi, mx, rho_e);
      double X[3] = {0, 0, 0};
#pragma unroll
      for (int k = 0; k < DIM; ++k) X[k] = U[L::XC + k];
      const double pert = phi0_gather(I, X);
      // radial return of dev H to the perturbed mixture yield surface; trace
      // solids have no stiffness and take no part; with no mixture modulus the
      // distortion carries no stress and is dropped, with no plastic work
      double Ymix = 0, Gm = 0;
      bool jc = false;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const MatP& m = P.mat[s];
        if (!(phi[s] >= PHI_TRACE)) continue;
        const double w = 1.0 - D[s];
        Gm += phi[s] * w * shear_modulus_undamaged<double, kExt>(m, rho_l[s]);
        const double sy = D[s] < crit_level(m) ? pert * m.yield : 0.0;
        Ymix += phi[s] * w * sy;
        jc = jc || (kExt && m.jc);
      }
      const double J = DIM == 3 ? sqrt(he[0] * he[0] + he[1] * he[1] + he[2] * he[2]) : sqrt(J2);
      double scale = 1.0, deps = 0.0;
      // phase temperatures of the entering state, frozen over the return
      double Tl[NS > 0 ? NS : 1];
#pragma unroll
      for (int s = 0; s < NS; ++s)
        Tl[s] = jc ? jc_temperature(P.mat[s], p, mx.t[s].pref, rho_l[s]) : JC_T_REF;
      if (!jc) {
        const double Jmax = Gm > 0.0 ? Ymix / (sqrt(6.0) * Gm) : 0.0;
        if (J > Jmax) {
          scale = Jmax / J;
          if (Gm > 0.0) deps = sqrt(2.0 / 3.0) * (J - Jmax);
        }
      } else if (Gm > 0.0) {
        // Johnson-Cook: solve sqrt6 G (J - sqrt(3/2) d) = Y_mix(d), the yield
        // at the end of the step (strain eps + d, rate d/dt).  The residual
        // falls in d; at the constant-yield increment it is already <= 0, so
        // the root lies in [0, that increment]: Newton steps kept inside
        // the bracket, bisection where one would leave it.
        auto ymix = [&](double dg, double* dY) {
          double y = 0.0, dy = 0.0;
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const MatP& m = P.mat[s];
            if (!(phi[s] >= PHI_TRACE) || !(D[s] < crit_level(m))) continue;
            double d1;
            const double f = phi[s] * (1.0 - D[s]) * pert;
            y += f * jc_yield(m, eps[s], dg, dt, Tl[s], &d1);
            dy += f * d1;
          }
          *dY = dy;
          return y;
        };
        double dY0;
        const double Y0 = ymix(0.0, &dY0);
        const double s6G = sqrt(6.0) * Gm;
        if (s6G * J > Y0) {
          // converged when the residual is at the rounding of the stress
          // scale sqrt6 G J or the bracket at that of its bound; a small
          // Newton step alone is no test (the hardening term's derivative
          // grows without bound as eps_p + d goes to zero)
          double lo = 0.0, hi = sqrt(2.0 / 3.0) * (J - Y0 / s6G), x = hi;
          const double fscale = 1e-14 * s6G * J;
          for (int it = 0; it < 200; ++it) {
            double dY;
            const double f = s6G * (J - sqrt(1.5) * x) - ymix(x, &dY);
            if (fabs(f) <= fscale) break;
            if (f > 0.0) lo = x; else hi = x;
            if (hi - lo <= 1e-15 * hi) { x = 0.5 * (lo + hi); break; }
            double xn = x - f / (-3.0 * Gm - dY);
            if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
            x = xn;
          }
          deps = x;
          scale = (J - sqrt(1.5) * x) / J;
        }
      } else if (J > 0.0) {
        scale = 0.0;
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) H[i][j] *= scale;
      double Vn[3][3];
      if constexpr (DIM == 3) {
        double e[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) e[k] = exp(scale * he[k]);
        sym3_compose(Qe, e, Vn);
      } else {
        stretch_from_log<DIM, double>(H, Vn);
      }
#pragma unroll
      for (int q = 0; q < L::NV; ++q) U[L::VB + q] = Vn[vb_i<DIM>(q)][vb_j<DIM>(q)];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const MatP& m = P.mat[s];
        // a trace solid does no plastic work: its histories stand
        const double dl = phi[s] >= PHI_TRACE ? deps : 0.0;
        const double seq = (1.0 - D[s]) * pert *
                         (jc ? jc_yield(m, eps[s], dl, dt, Tl[s], nullptr) : m.yield);
        // the simplified law has no gate: any plastic increment of a live
        // solid below D_crit
        const bool simple = kExt && m.Ddot0 > 0.0;
        const double pg = m.pgate - (sizeof(T) == 8 ? m.sbnd : m.sbnd_bulk);
        bool gate = (simple || p < pg) && (dl > 0.0) && (D[s] < crit_level(m));
        const bool ok = seq > 0.0;
        const double R = ok ? triaxiality(m, p, seq, closure_density(m, phi[s], rho_l[s])) : 1.0;
        if (gate && !simple) {
          const double thr = eps_threshold(m, R);
          gate = (eps[s] > thr) || !ok;
        }
        Dn[s] = D[s];
        if (gate) Dn[s] = (ok || simple) ? damage_rk4<kExt>(m, D[s], eps[s], dl, R) : m.Dcrit;
        const double ms = U[L::MASS + s];
        U[L::HIST + 2 * s] = ms * (eps[s] + dl);
        U[L::HIST + 2 * s + 1] = ms * Dn[s];
      }
    } else {
#pragma unroll
      for (int q = 0; q < L::NV; ++q)
        U[L::VB + q] = vb_i<DIM>(q) == vb_j<DIM>(q) ? 1.0 : 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) Dn[s] = D[s];
    }
    // imposed-velocity driver (Section 4.3): a live solid behind the driver
    // surface moves outward at least at the driver's speed; the kinetic
    // energy this adds is the driver's work
    if constexpr (kExt && DIM >= 2) {
      if (P.drv[5] > 0.0 && live) {
        const double Rd = driver_radius(P.drv, tn);
        if (Rd < P.drv[5]) {
          const int64_t ix = g % I.n[0], iy = (g / I.n[0]) % I.n[1];
          const double x = I.lo[0] + ((double)ix + 0.5) * I.dx[0];
          const double y = I.lo[1] + ((double)iy + 0.5) * I.dx[1];
          const double r = sqrt(x * x + y * y);
          const double vr = driver_speed(P.drv, tn);
          if (r > 0.0 && r <= Rd) {
            const double ur = (u[0] * x + u[1] * y) / r;
            if (ur < vr) {
              const double du = vr - ur;
              const double ke0 = ke;
              u[0] += du * x / r;
              u[1] += du * y / r;
              ke = 0.0;
#pragma unroll
              for (int k = 0; k < DIM; ++k) { U[L::MOM + k] = rho * u[k]; ke += u[k] * u[k]; }
              U[L::ENE] += 0.5 * rho * (ke - ke0);
            }
          }
        }
      }
    }
    // CFL sum on the new state, in the policy precision C
    C phic[NM], rlc[NM], Dc[NS > 0 ? NS : 1];
#pragma unroll
    for (int l = 0; l < NM; ++l) { phic[l] = (C)phi[l]; rlc[l] = (C)rho_l[l]; }
#pragma unroll
    for (int s = 0; s < NS; ++s) Dc[s] = (C)Dn[s];
    const C J2n = (C)J2_of<DIM, double>(H);
    Mix<NM, NS, C> mx2;
    mix_terms<NM, NS, C, kExt>(P, phic, rlc, Dc, J2n, mx2);
    bool isl = false;
#pragma unroll
    for (int l = 0; l < NM; ++l) isl = isl || phic[l] < cst<C>(P.phi_fp64_cut, P.f_phi_fp64_cut);
    C p2;
    if (sizeof(C) == 8 || !isl) {
      p2 = mix_pressure<NM, NS, C>(P, phic, mx2, (C)rho_e);
    } else {
      // FP64 island, as in the stages: the inversion of a trace cell in double
      double xi = 0, th = rho_e, cold = 0;
#pragma unroll
      for (int l = 0; l < NM; ++l) {
        const double ig = kExt && P.mat[l].bp ? (double)mx2.t[l].invG : P.mat[l].invGamma;
        xi += phi[l] * ig;
        th -= phi[l] * (double)mx2.t[l].rho_eref;
        cold += phi[l] * (double)mx2.t[l].pref * ig;
      }
      p2 = (C)((m_max(th, 0.0) + cold) / xi);
    }
    C Gmix;
    const C c = mix_sound<NM, NS, C>(P, phic, mx2, p2, (C)rho, Gmix);
    double sum = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) sum += (fabs(u[k]) + (double)c) / I.dx[k];
    return sum;
  }

  // Void relaxation of one cell after seeding (one solid, seed_nu > 0): a
  // cell with mass whose void fraction exceeds seed_nu holds a film of
  // material with void on its free side, and void carries no stress.  The
  // film's density moves to the first density, scanning up from rho0/2 over
  // [rho0/2, 2 rho0], at which the material's own pressure at the cell's
  // specific internal energy e = rho_e / mass changes sign (the film alone:
  // volume fraction one, energy rho_l e per film volume, no trace closures);
  // RELAX_ITERS halvings on whether the pressure at the midpoint has the
  // sign it has at the lower end; without a sign change the film takes
  // 2 rho0.  phi = mass / density, clamped to [phi_floor, 1]; nothing else
  // changes.  U: the cell's state (double), phi updated in place.
  FV_HD static void relax_void_cell(const Params& P, double* U) {
    if constexpr (NM == 1 && NS == 1) {
      const double phi = U[L::PHI], ms = U[L::MASS];
      if (!(1.0 - m_clamp(phi, 0.0, 1.0) > P.seed_nu) || !(ms > 0.0)) return;
      double u2 = 0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        const double uk = U[L::MOM + k] / ms;
        u2 += uk * uk;
      }
      const double e = (U[L::ENE] - 0.5 * ms * u2) / ms;
      double D[1] = {U[L::HIST + 1] / ms};
      double V[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
      for (int q = 0; q < L::NV; ++q) V[vb_i<DIM>(q)][vb_j<DIM>(q)] = U[L::VB + q];
      double H[3][3];
      hencky<DIM, double>(V, H);
      const double J2 = J2_of<DIM, double>(H);
      // the root in the closure precision C: float closures and 32 halvings
      // (a bracket of 1.5 rho0 / 2^32, far below float storage) in the
      // FP32-bulk form; in double the halvings stop once the midpoint is an
      // end of the bracket, after which they could not move it
      const C ec = (C)e, J2c = (C)J2;
      C Dc[1] = {(C)D[0]};
      auto positive = [&](C rl) {
        C one = (C)1;
        Mix<1, 1, C> mr;
        mix_terms<1, 1, C, kExt>(P, &one, &rl, Dc, J2c, mr);
        return mix_pressure<1, 1, C>(P, &one, mr, rl * ec) > (C)0;
      };
      const C rho0 = cst<C>(P.mat[0].rho0, P.mat[0].f_rho0);
      C lo = (C)0.5 * rho0, hi = (C)2 * rho0;
      const bool slo = positive(lo);
      const int iters = sizeof(C) == 8 ? RELAX_ITERS : RELAX_ITERS / 2;
      for (int it = 0; it < iters; ++it) {
        const C mid = (C)0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (positive(mid) == slo) lo = mid;
        else hi = mid;
      }
      U[L::PHI] = m_clamp(ms / (double)((C)0.5 * (lo + hi)), P.phi_floor, 1.0);
    }
  }

  // wave-speed sum of a state without a source step (initial CFL)
  FV_HD static double cfl_sum(const Params& P, const Inst& I, const double* U) {
    double phi[NM], rho_l[NM], D[NS > 0 ? NS : 1];
    double rho = 0;
#pragma unroll
    for (int l = 0; l < NM; ++l) {
      phi[l] = U[L::PHI + l];
      const double ml = U[L::MASS + l] > 0.0 ? U[L::MASS + l] : 0.0;
      rho_l[l] = ml / phi[l];
      rho += ml;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double ms = U[L::MASS + s];
      D[s] = ms > 0.0 ? U[L::HIST + 2 * s + 1] / ms : 0.0;
    }
    double u[3] = {0, 0, 0}, ke = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) { u[k] = U[L::MOM + k] / rho; ke += u[k] * u[k]; }
    const double rho_e = U[L::ENE] - 0.5 * rho * ke;
    double V[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int q = 0; q < L::NV; ++q) V[vb_i<DIM>(q)][vb_j<DIM>(q)] = U[L::VB + q];
    double H[3][3];
    // 3D: the eigen-decomposition of V V^T is kept, so that the return (a
    // scaling of dev H) rebuilds the stretch from the same eigenvectors
    double Qe[3][3], he[3];
    if constexpr (DIM == 3) {
      double B[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          B[i][j] = V[i][0] * V[j][0] + V[i][1] * V[j][1] + V[i][2] * V[j][2];
      sym3_eig(B, Qe);
      half_log_eigs3<double>(V, B, he);
      const double mm = (he[0] + he[1] + he[2]) / 3.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) he[k] -= mm;
      sym3_compose(Qe, he, H);
    } else {
      hencky<DIM, double>(V, H);
    }
    const double J2 = J2_of<DIM, double>(H);
    Mix<NM, NS, double> mx;
    mix_terms<NM, NS, double, kExt>(P, phi, rho_l, D, J2, mx);
    const double p = mix_pressure<NM, NS, double>(P, phi, mx, rho_e);
    double Gmix;
    const double c = mix_sound<NM, NS, double>(P, phi, mx, p, rho, Gmix);
    double sum = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) sum += (fabs(u[k]) + c) / I.dx[k];
    return sum;
  }

  // RK combination + clamp (+ source and CFL in stage 3) for one cell.
  // Returns the CFL sum (stage 3) or 0, and sets *bad for a non-physical
  // state.
  FV_HD static double finish_cell(const Ctx& cx, int64_t g, const C* acc, bool* bad) {
    C us[S], ub[S];
    load_state(cx, cx.src, g, us);
    if (cx.stage != 1) load_state(cx, cx.base, g, ub);
    return finish_cell(cx, g, acc, us, ub, bad);
  }

  // us: the cell's stage input, ub: its U^n (stages 2 and 3)
  FV_HD static double finish_cell(const Ctx& cx, int64_t g, const C* acc, const C* us,
                                  const C* ub, bool* bad) {
    const Inst& I = *cx.I;
    // The third stage's weights 1/3 and 2/3 are applied in double: rounded
    // to float they would not sum to one (2/3 rounds up by 3e-8), and every
    // cell's mass, momentum and energy would grow by that fraction each step.
    double Un[S];
#pragma unroll
    for (int f = 0; f < S; ++f) {
      const C v = us[f] + cx.dt * acc[f];
      if (cx.stage == 1) Un[f] = (double)v;
      else if (cx.stage == 2) Un[f] = (double)((C)0.75 * ub[f] + (C)0.25 * v);
      else Un[f] = ((double)ub[f] + 2.0 * (double)v) / 3.0;
    }
#pragma unroll
    for (int l = 0; l < NM; ++l) Un[L::PHI + l] = m_clamp(Un[L::PHI + l], cx.P.phi_floor, 1.0);
    double cfl = 0;
    if (cx.stage == 3) cfl = source_and_cfl(cx.P, I, Un, (double)cx.dt, g, cx.tn);
    double rho = 0;
    bool nan = false;
#pragma unroll
    for (int f = 0; f < S; ++f) nan = nan || !(Un[f] == Un[f]) || Un[f] - Un[f] != 0.0;
#pragma unroll
    for (int l = 0; l < NM; ++l) rho += Un[L::MASS + l];
    *bad = nan || !(rho > 0.0);
#pragma unroll
    for (int f = 0; f < S; ++f) st(cx.out, f, I.ncell, g, (T)Un[f]);
    return cfl;
  }
};

// Per-cell primitive <-> conserved conversions (used by the load/diagnostic
// kernels).  Primitive layout: the state's field order with rho_l for the
// phasic mass, (eps_p, D) for the history densities, u for the momentum and
// p for the total energy; volume fractions are clamped to [phi_floor, 1].
template <int DIM, int NM, int NS>
struct Cell {
  using L = Lay<DIM, NM, NS>;
  FV_HD static void prim_to_cons(const Params& P, const double* W, double* U) {
    double phi[NM], rho_l[NM], D[NS > 0 ? NS : 1];
    for (int l = 0; l < NM; ++l) {
      phi[l] = m_clamp(W[L::PHI + l], P.phi_floor, 1.0);
      rho_l[l] = W[L::MASS + l];
    }
    for (int s = 0; s < NS; ++s) D[s] = W[L::HIST + 2 * s + 1];
    double V[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int q = 0; q < L::NV; ++q) V[vb_i<DIM>(q)][vb_j<DIM>(q)] = W[L::VB + q];
    double H[3][3];
    hencky<DIM, double>(V, H);
    const double J2 = J2_of<DIM, double>(H);
    Mix<NM, NS, double> mx;
    mix_terms<NM, NS, double>(P, phi, rho_l, D, J2, mx);
    const double p = W[L::ENE];
    const double rho_e = mix_energy<NM, NS, double>(P, phi, mx, p);
    double rho = 0;
    for (int l = 0; l < NM; ++l) rho += phi[l] * rho_l[l];
    double ke = 0;
    for (int k = 0; k < DIM; ++k) ke += W[L::MOM + k] * W[L::MOM + k];
    for (int l = 0; l < NM; ++l) { U[L::PHI + l] = phi[l]; U[L::MASS + l] = phi[l] * rho_l[l]; }
    for (int s = 0; s < NS; ++s) {
      U[L::HIST + 2 * s] = phi[s] * rho_l[s] * W[L::HIST + 2 * s];
      U[L::HIST + 2 * s + 1] = phi[s] * rho_l[s] * W[L::HIST + 2 * s + 1];
    }
    for (int k = 0; k < DIM; ++k) U[L::MOM + k] = rho * W[L::MOM + k];
    U[L::ENE] = rho_e + 0.5 * rho * ke;
    for (int q = 0; q < L::NV; ++q) U[L::VB + q] = W[L::VB + q];
    for (int k = 0; k < DIM; ++k) U[L::XC + k] = W[L::XC + k];
  }

  FV_HD static void cons_to_prim(const Params& P, const double* U, double* W) {
    double phi[NM], rho_l[NM], D[NS > 0 ? NS : 1], eps[NS > 0 ? NS : 1];
    double rho = 0;
    for (int l = 0; l < NM; ++l) {
      phi[l] = U[L::PHI + l];
      const double ml = m_max(U[L::MASS + l], 0.0);
      rho_l[l] = ml / phi[l];
      rho += ml;
    }
    for (int s = 0; s < NS; ++s) {
      const double ms = U[L::MASS + s];
      eps[s] = ms > 0.0 ? U[L::HIST + 2 * s] / ms : 0.0;
      D[s] = ms > 0.0 ? U[L::HIST + 2 * s + 1] / ms : 0.0;
    }
    double u[3] = {0, 0, 0}, ke = 0;
    for (int k = 0; k < DIM; ++k) { u[k] = U[L::MOM + k] / rho; ke += u[k] * u[k]; }
    const double rho_e = U[L::ENE] - 0.5 * rho * ke;
    double V[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int q = 0; q < L::NV; ++q) V[vb_i<DIM>(q)][vb_j<DIM>(q)] = U[L::VB + q];
    double H[3][3];
    // 3D: the eigen-decomposition of V V^T is kept, so that the return (a
    // scaling of dev H) rebuilds the stretch from the same eigenvectors
    double Qe[3][3], he[3];
    if constexpr (DIM == 3) {
      double B[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          B[i][j] = V[i][0] * V[j][0] + V[i][1] * V[j][1] + V[i][2] * V[j][2];
      sym3_eig(B, Qe);
      half_log_eigs3<double>(V, B, he);
      const double mm = (he[0] + he[1] + he[2]) / 3.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) he[k] -= mm;
      sym3_compose(Qe, he, H);
    } else {
      hencky<DIM, double>(V, H);
    }
    const double J2 = J2_of<DIM, double>(H);
    Mix<NM, NS, double> mx;
    mix_terms<NM, NS, double>(P, phi, rho_l, D, J2, mx);
    const double p = mix_pressure<NM, NS, double>(P, phi, mx, rho_e);
    for (int l = 0; l < NM; ++l) { W[L::PHI + l] = phi[l]; W[L::MASS + l] = rho_l[l]; }
    for (int s = 0; s < NS; ++s) { W[L::HIST + 2 * s] = eps[s]; W[L::HIST + 2 * s + 1] = D[s]; }
    for (int k = 0; k < DIM; ++k) W[L::MOM + k] = u[k];
    W[L::ENE] = p;
    for (int q = 0; q < L::NV; ++q) W[L::VB + q] = U[L::VB + q];
    for (int k = 0; k < DIM; ++k) W[L::XC + k] = U[L::XC + k];
  }
};

}  // namespace fv

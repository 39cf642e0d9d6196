// Device math of the fracture hot path: closures, mixture, kinematics,
// reconstruction, HLLC with the void-opening modifier, source step.
//
// Everything here is __host__ __device__ so that the per-thread phases of
// the stage kernel can also be stepped on the CPU for debugging; the
// library itself only ever runs them on the GPU.
//
// References are to arXiv 2210.04037 (Wallis, Barton, Nikiforakis):
// Section 2.1 evolution equations, Section 2.2 thermodynamics and damage,
// Section 2.3 closure models, Section 2.4 perturbation field, Section 3.1
// fracture, Section 3.2 Lagrangian coordinates.
#pragma once

#include <stdint.h>
#include <math.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define FV_HD __host__ __device__ __forceinline__
#else
#define FV_HD inline
#endif

namespace fv {

#if defined(__HIP_DEVICE_COMPILE__)
// A pointer that every lane of the wave holds alike, returned as a value the
// compiler keeps in scalar registers: address arithmetic on it then stays
// scalar instead of being folded into 64-bit per-lane addresses.
template <class E>
__device__ __forceinline__ E* wave_uniform(E* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (E*)(((uint64_t)hi << 32) | lo);
}
#endif

// ----------------------------------------------------------------------------
// scalar helpers (double and float overloads)
// ----------------------------------------------------------------------------
FV_HD double m_sqrt(double x) { return sqrt(x); }
FV_HD float m_sqrt(float x) { return sqrtf(x); }
FV_HD double m_log(double x) { return log(x); }
FV_HD float m_log(float x) { return logf(x); }
FV_HD double m_cbrt(double x) { return cbrt(x); }
FV_HD float m_cbrt(float x) { return cbrtf(x); }
FV_HD double m_exp(double x) { return exp(x); }
FV_HD float m_exp(float x) { return expf(x); }
FV_HD double m_pow(double x, double y) { return pow(x, y); }
FV_HD float m_pow(float x, float y) { return powf(x, y); }
FV_HD double m_abs(double x) { return fabs(x); }
FV_HD float m_abs(float x) { return fabsf(x); }
template <class C> FV_HD C m_min(C a, C b) { return a < b ? a : b; }
template <class C> FV_HD C m_max(C a, C b) { return a > b ? a : b; }
template <class C> FV_HD C m_clamp(C v, C lo, C hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// x^e with a fast path for small integer exponents (ei > 0).
template <class C> FV_HD C powi_or(C x, C e, int ei) {
  if (ei > 0) {
    C r = x;
    for (int k = 1; k < ei; ++k) r *= x;
    return r;
  }
  return m_pow(x, e);
}

// ----------------------------------------------------------------------------
// material and run parameters (passed by value to kernels)
// ----------------------------------------------------------------------------
struct MatP {
  int kind;       // 0 solid (Romenskii), 1 ideal gas
  int alpha_i;    // alpha as a small integer, else 0
  int beta1_i;    // beta + 1 as a small integer, else 0
  int jc;         // the yield depends on strain, rate or temperature
  double rho0, K0, alpha, G0, beta, Gamma0;
  double yield, Dcrit, D0, eps_th, eps_c, balpha, nhard, pgate;
  double jcB, jcC, jcm, Tmelt, CV;   // Johnson-Cook c2, c3, m, T_melt, C_V
  // Steinberg modulus G0 + Gp p_c eta^(-1/3) (stein), Burakovsky-Preston
  // Grueneisen Gamma0 + G1 eta^(-1/3) + G2 eta^(-gbp) (bp), simplified damage
  // law dD/deps = Ddot0 (1 - D) (Ddot0 > 0)
  double Gp, G1, G2, gbp, Ddot0;
  int stein, bp;
  // host-derived constants
  // Critical level of the Section 3.1 test D >= D_crit, which holds up to the
  // rounding of the advected ratio (phi rho D)/(phi rho) of a clamped cell:
  double Dcrit_eff;    // double storage: D_crit (1 - 1e-9)
  double Dcrit_bulk;   // float storage (FP32-bulk policy): D_crit (1 - 1e-6),
                       // about fifteen float ulps of D_crit
  // band of the stress sign tests (the tension of the void-opening modifier,
  // the pressure gate of the damage law): the same relative width of K0, so
  // that a cell at zero stress up to rounding counts as out of tension
  double sbnd;         // double storage: 1e-9 K0
  double sbnd_bulk;    // float storage: 1e-6 K0
  double invGamma;   // 1 / Gamma0
  double nu;         // Poisson ratio of the undamaged moduli
  double bonA;       // alpha_B (Dc - D0)^(1/alpha_B) / ln(eps_c / eps_th)
  double bonExp;     // (alpha_B - 1) / alpha_B
  // the closure constants rounded to float on the host, for the FP32-bulk
  // closures: the kernels read them as arguments in scalar registers instead
  // of converting the doubles per wave (the same rounding either way)
  float f_rho0, f_K0, f_alpha, f_G0, f_beta, f_Gamma0, f_invGamma, f_Dcrit_eff;
  float f_Gp, f_G1, f_G2, f_gbp;
};

struct Params {
  MatP mat[2];
  double cfl;
  double phi_floor;
  double weno_eps;
  double c_min2;
  double phi_fp64_cut;
  double seed_nu;      // void fraction above which X is reseeded (0: off)
  // THINC sharpening of the volume fractions: steepness (0: MUSCL), with
  // tanh(beta) and 1/cosh(beta) formed on the host
  double thinc_beta, thinc_tb, thinc_sech;
  // imposed-velocity driver of the ring (Section 4.3): inner radius, v0, v1,
  // t0, t1, r_max (r_max = 0: off)
  double drv[6];
  // tension band of the void-opening modifier: the largest of the solids'
  // stress bands (double storage, float storage)
  double tens_band, tens_band_bulk;
  float f_weno_eps, f_c_min2, f_phi_fp64_cut, f_pad;
  float f_thinc_beta, f_thinc_tb, f_thinc_sech, f_pad2;
};

// Host: the derived constants of a solid, from its own fields.
inline void set_solid_constants(MatP& q) {
  q.Dcrit_eff = q.Dcrit * (1.0 - 1.0e-9);
  q.Dcrit_bulk = q.Dcrit * (1.0 - 1.0e-6);
  q.sbnd = 1.0e-9 * q.K0;
  q.sbnd_bulk = 1.0e-6 * q.K0;
  q.nu = (3.0 * q.K0 - 2.0 * q.G0) / (2.0 * (3.0 * q.K0 + q.G0));
  q.bonA = q.balpha * pow(q.Dcrit - q.D0, 1.0 / q.balpha) / log(q.eps_c / q.eps_th);
  q.bonExp = (q.balpha - 1.0) / q.balpha;
}

// Host: fill the float copies once the double parameters are set.
inline void set_float_constants(Params& P) {
  P.tens_band = P.tens_band_bulk = 0.0;
  for (MatP& m : P.mat) {
    if (m.kind == 0) {
      P.tens_band = m.sbnd > P.tens_band ? m.sbnd : P.tens_band;
      P.tens_band_bulk = m.sbnd_bulk > P.tens_band_bulk ? m.sbnd_bulk : P.tens_band_bulk;
    }
    m.f_rho0 = (float)m.rho0; m.f_K0 = (float)m.K0; m.f_alpha = (float)m.alpha;
    m.f_G0 = (float)m.G0; m.f_beta = (float)m.beta; m.f_Gamma0 = (float)m.Gamma0;
    m.f_invGamma = (float)m.invGamma; m.f_Dcrit_eff = (float)m.Dcrit_bulk;
    m.f_Gp = (float)m.Gp; m.f_G1 = (float)m.G1; m.f_G2 = (float)m.G2; m.f_gbp = (float)m.gbp;
  }
  P.f_weno_eps = (float)P.weno_eps;
  P.f_c_min2 = (float)P.c_min2;
  P.f_phi_fp64_cut = (float)P.phi_fp64_cut;
  P.thinc_tb = P.thinc_beta > 0.0 ? tanh(P.thinc_beta) : 0.0;
  P.thinc_sech = P.thinc_beta > 0.0 ? 1.0 / cosh(P.thinc_beta) : 0.0;
  P.f_thinc_beta = (float)P.thinc_beta;
  P.f_thinc_tb = (float)P.thinc_tb;
  P.f_thinc_sech = (float)P.thinc_sech;
}

// A parameter in the closure precision C: the double itself, or its float
// copy.
template <class C> FV_HD C cst(double d, float f);
template <> FV_HD double cst<double>(double d, float) { return d; }
template <> FV_HD float cst<float>(double, float f) { return f; }

// ----------------------------------------------------------------------------
// field layout of the conserved state (Section 2.1 equation order)
// ----------------------------------------------------------------------------
template <int DIM, int NM, int NS>
struct Lay {
  static constexpr int NV = DIM == 1 ? 3 : (DIM == 2 ? 5 : 9);
  static constexpr int NH = DIM == 1 ? 3 : (DIM == 2 ? 4 : 6);
  // conserved state
  static constexpr int PHI = 0;
  static constexpr int MASS = NM;
  static constexpr int HIST = 2 * NM;
  static constexpr int MOM = 2 * NM + 2 * NS;
  static constexpr int ENE = MOM + DIM;
  static constexpr int VB = ENE + 1;
  static constexpr int XC = VB + NV;
  static constexpr int S = XC + DIM;
  // conserved-flux vector: masses, histories, momenta, energy
  static constexpr int NC = NM + 2 * NS + DIM + 1;
  static constexpr int C_MOM = NM + 2 * NS;
  static constexpr int C_ENE = C_MOM + DIM;
  // reconstructed primitives
  static constexpr int R_PHI = 0;
  static constexpr int R_RHO = NM;
  static constexpr int R_HIST = 2 * NM;
  static constexpr int R_U = 2 * NM + 2 * NS;
  static constexpr int R_P = R_U + DIM;
  static constexpr int R_H = R_P + 1;
  static constexpr int R_V = R_H + NH;
  static constexpr int NR = R_V + NV;
  // extra per-cell tile values
  static constexpr int W_X = NR;
  static constexpr int W_SIG = NR + DIM;   // sigma_aa per direction
  static constexpr int W_CRIT = NR + 2 * DIM;
  static constexpr int NW = W_CRIT + 1;
  // per-face data
  static constexpr int Q_F = 0;
  static constexpr int Q_UF = NC;
  static constexpr int Q_UT = NC + 1;          // DIM-1 tangential comps
  static constexpr int Q_PHI = Q_UT + (DIM - 1);
  static constexpr int Q_X = Q_PHI + NM;
  static constexpr int Q_V = Q_X + DIM;
  static constexpr int Q_OS = Q_V + NV;        // 0 normal, 1 closed
  static constexpr int Q_USL = Q_OS + 1;
  static constexpr int Q_USR = Q_OS + 2;
  static constexpr int NQ = Q_USR + 1;
};

// stored (i, j) components of the unimodular stretch
template <int DIM> FV_HD int vb_i(int q) {
  if (DIM == 1) return q;
  if (DIM == 2) { const int t[5] = {0, 0, 1, 1, 2}; return t[q]; }
  return q / 3;
}
template <int DIM> FV_HD int vb_j(int q) {
  if (DIM == 1) return q;
  if (DIM == 2) { const int t[5] = {0, 1, 0, 1, 2}; return t[q]; }
  return q % 3;
}
// independent components of the symmetric Hencky strain
template <int DIM> FV_HD int hk_i(int q) {
  if (DIM == 1) return q;
  if (DIM == 2) { const int t[4] = {0, 0, 1, 2}; return t[q]; }
  const int t[6] = {0, 0, 0, 1, 1, 2}; return t[q];
}
template <int DIM> FV_HD int hk_j(int q) {
  if (DIM == 1) return q;
  if (DIM == 2) { const int t[4] = {0, 1, 1, 2}; return t[q]; }
  const int t[6] = {0, 1, 2, 1, 2, 2}; return t[q];
}

// ----------------------------------------------------------------------------
// single-material closures (Sections 2.2, 2.3)
// ----------------------------------------------------------------------------
// Reference terms of one material in Mie-Grueneisen form, as products with
// the phasic density so that they stay finite for rho -> 0:
//   rho e_ref = (1-D)(rho e~_c + G~ J^2),  p_ref = (1-D)(p~_c + beta G~ J^2),
//   rho dp_ref/drho = (1-D)(rho dp~_c/drho + beta (beta+1) G~ J^2),
// with the Romenskii cold energy e~_c = K0/(2 rho0 a^2)(eta^a - 1)^2 (the
// denominator read as 2 rho0 a^2 so that a -> 0 is the log EOS) and shear
// modulus G~ = G0 eta^(beta+1).  Gas: all zero.  Solids come first in a
// material list (checked when a context is made), so material l is a solid
// exactly when l < NS and the kernels decide the kind at compile time.
// invG = 1/Gamma(rho) and g1 = Gamma + 1 + rho Gamma'/Gamma (the factor of
// the thermal pressure in rho c^2) carry the Grueneisen function per cell.
template <class C>
struct RefT { C rho_eref, pref, rho_dpref, G, invG, g1; };

// Shear modulus and its density derivatives rho G' and rho^2 G''.
// Romenskii: G0 eta^(beta+1), (beta+1) G, (beta+1) beta G.  Steinberg
// (Section 2.3): G0 + Gp p_c eta^(-1/3), from the cold pressure and its
// derivatives, rho G' = Gp eta^(-1/3)(rho p_c' - p_c/3) and
// rho^2 G'' = Gp eta^(-1/3)(rho^2 p_c'' - (2/3) rho p_c' + (4/9) p_c), with
// rho^2 p_c'' = (K0/a) eta^(a+1) ((2a+1) 2a eta^a - (a+1) a).
// EXT false: a build for materials without the Steinberg, Burakovsky-Preston,
// Johnson-Cook and simplified-damage rows (their branches compiled out).
template <class C, bool EXT = true>
FV_HD void shear_terms(const MatP& m, C eta, C ea, C ea1, C pc, C rho_dpc, C* G, C* rG1,
                       C* r2G2) {
  if (!EXT || !m.stein) {
    const C b = cst<C>(m.beta, m.f_beta);
    const C Gt = cst<C>(m.G0, m.f_G0) * powi_or(eta, b + (C)1, m.beta1_i);
    *G = Gt;
    *rG1 = (b + (C)1) * Gt;
    *r2G2 = (b + (C)1) * b * Gt;
    return;
  }
  const C a = cst<C>(m.alpha, m.f_alpha);
  const C K0 = cst<C>(m.K0, m.f_K0);
  const C r2 = K0 / a * ea1 * (((C)2 * a + (C)1) * (C)2 * a * ea - (a + (C)1) * a);
  const C e3 = (C)1 / m_cbrt(eta);
  const C Gp = cst<C>(m.Gp, m.f_Gp);
  *G = cst<C>(m.G0, m.f_G0) + Gp * pc * e3;
  *rG1 = Gp * e3 * (rho_dpc - pc / (C)3);
  *r2G2 = Gp * e3 * (r2 - (C)(2.0 / 3.0) * rho_dpc + (C)(4.0 / 9.0) * pc);
}

template <class C, bool EXT = true>
FV_HD RefT<C> solid_ref_terms(const MatP& m, C rho, C J2, C D) {
  RefT<C> r;
  const C a = cst<C>(m.alpha, m.f_alpha);
  const C rho0 = cst<C>(m.rho0, m.f_rho0);
  const C eta = rho / rho0;
  const C ea = powi_or(eta, a, m.alpha_i);
  const C ea1 = ea * eta;
  const C K0 = cst<C>(m.K0, m.f_K0);
  const C rho_ec = rho * K0 / ((C)2 * rho0 * a * a) * (ea - (C)1) * (ea - (C)1);
  const C pc = K0 / a * ea1 * (ea - (C)1);
  const C rho_dpc = K0 / a * ea1 * (((C)2 * a + (C)1) * ea - (a + (C)1));
  C Gt, rG1, r2G2;
  shear_terms<C, EXT>(m, eta, ea, ea1, pc, rho_dpc, &Gt, &rG1, &r2G2);
  const C w = (C)1 - D;
  r.rho_eref = w * (rho_ec + Gt * J2);
  r.pref = w * (pc + (rG1 - Gt) * J2);
  r.rho_dpref = w * (rho_dpc + r2G2 * J2);
  r.G = w * Gt;
  return r;
}

template <class C, bool EXT = true>
FV_HD C shear_modulus_undamaged(const MatP& m, C rho) {
  if (!EXT || !m.stein)
    return cst<C>(m.G0, m.f_G0) *
           powi_or(rho / cst<C>(m.rho0, m.f_rho0), cst<C>(m.beta, m.f_beta) + (C)1, m.beta1_i);
  const C a = cst<C>(m.alpha, m.f_alpha);
  const C eta = rho / cst<C>(m.rho0, m.f_rho0);
  const C ea = powi_or(eta, a, m.alpha_i);
  const C pc = cst<C>(m.K0, m.f_K0) / a * ea * eta * (ea - (C)1);
  return cst<C>(m.G0, m.f_G0) + cst<C>(m.Gp, m.f_Gp) * pc / m_cbrt(eta);
}

// Grueneisen share of a material at phasic density rho: sets invG and g1 of
// its reference terms (constants unless Burakovsky-Preston:
// Gamma = Gamma0 + G1 eta^(-1/3) + G2 eta^(-gbp),
// rho Gamma' = -G1 eta^(-1/3)/3 - gbp G2 eta^(-gbp)).
template <class C, bool EXT = true>
FV_HD void gamma_terms(const MatP& m, C rho, RefT<C>& t) {
  if (!EXT || !m.bp) {
    t.invG = cst<C>(m.invGamma, m.f_invGamma);
    t.g1 = cst<C>(m.Gamma0, m.f_Gamma0) + (C)1;
    return;
  }
  const C eta = rho / cst<C>(m.rho0, m.f_rho0);
  const C e3 = (C)1 / m_cbrt(eta);
  const C eg = m_pow(eta, -cst<C>(m.gbp, m.f_gbp));
  const C g1t = cst<C>(m.G1, m.f_G1) * e3, g2t = cst<C>(m.G2, m.f_G2) * eg;
  const C gam = cst<C>(m.Gamma0, m.f_Gamma0) + g1t + g2t;
  t.invG = (C)1 / gam;
  t.g1 = gam + (C)1 + (-g1t / (C)3 - cst<C>(m.gbp, m.f_gbp) * g2t) / gam;
}

// ----------------------------------------------------------------------------
// mixture (Allaire-type closure under mechanical and thermal equilibrium)
// ----------------------------------------------------------------------------
// p = [rho e - sum phi_l rho_l e_ref,l + sum phi_l p_ref,l / Gamma_l]
//     / sum phi_l / Gamma_l.
// The void carries no stress: sigma = -(1-nu) p I + 2 G_mix dev H with
// G_mix = sum phi_l G_l; c^2 = (1-nu) sum phi_l xi_l rho_l c_l^2 / (xi rho)
// + (4/3) G_mix / rho.
template <int NM, int NS, class C>
struct Mix {
  RefT<C> t[NM];
  C xi;
};

// A material below this volume fraction is a trace: its phasic density (the
// ratio of two trace quantities) is noise.  A trace takes the limit of its
// closures as the phasic density vanishes: the Romenskii cold energy and
// pressure, stiffness and shear modulus all go to zero there, so it carries
// no reference terms and no shear stiffness and enters the mixture only
// through its Grueneisen share.  The traces that matter sit in cells emptied
// to near vacuum, far below rho0, where this limit is continuous with the
// closures just above the threshold; evaluating them at rho0 instead would
// switch on the full modulus G0 with whatever distortion the cell carries.
constexpr double PHI_TRACE = 1.0e-6;

// halvings of the void relaxation's density bracket [rho0/2, 2 rho0]
constexpr int RELAX_ITERS = 64;

// the void relaxation runs (and then sets the CFL state after the seeding
// pass instead of the last stage): one solid and seeding on
FV_HD bool relax_on(const Params& P, int nm, int ns) {
  return nm == 1 && ns == 1 && P.seed_nu > 0.0;
}

// density for the closures that need one (the triaxiality's rho0/rho): the
// reference density for a trace
template <class C>
FV_HD C closure_density(const MatP& m, C phi_l, C rho_l) {
  return phi_l < (C)PHI_TRACE ? cst<C>(m.rho0, m.f_rho0) : rho_l;
}

template <int NM, int NS, class C, bool EXT = true>
FV_HD void mix_terms(const Params& P, const C* phi, const C* rho_l, const C* D,
                     C J2, Mix<NM, NS, C>& mx) {
  mx.xi = 0;
#pragma unroll
  for (int l = 0; l < NM; ++l) {
    const bool live = l < NS && phi[l] >= (C)PHI_TRACE;
    if (live) {
      mx.t[l] = solid_ref_terms<C, EXT>(P.mat[l], rho_l[l], J2, D[l < NS ? l : 0]);
    } else {
      mx.t[l].rho_eref = 0; mx.t[l].pref = 0; mx.t[l].rho_dpref = 0; mx.t[l].G = 0;
    }
    // a trace takes its Grueneisen function at the reference density
    gamma_terms<C, EXT>(P.mat[l], live ? rho_l[l] : cst<C>(P.mat[l].rho0, P.mat[l].f_rho0),
                        mx.t[l]);
    mx.xi += phi[l] * mx.t[l].invG;
  }
}

// Pressure inversion; the thermal energy density rho e - sum phi rho e_ref is
// taken non-negative (the cold curve is the zero-temperature bound).
template <int NM, int NS, class C>
FV_HD C mix_pressure(const Params& P, const C* phi, const Mix<NM, NS, C>& mx,
                     C rho_e) {
  C th = rho_e, cold = 0;
#pragma unroll
  for (int l = 0; l < NM; ++l) {
    th = th - phi[l] * mx.t[l].rho_eref;
    cold = cold + phi[l] * mx.t[l].pref * mx.t[l].invG;
  }
  return (m_max(th, (C)0) + cold) / mx.xi;
}

template <int NM, int NS, class C>
FV_HD C mix_energy(const Params& P, const C* phi, const Mix<NM, NS, C>& mx, C p) {
  C re = mx.xi * p;
#pragma unroll
  for (int l = 0; l < NM; ++l)
    re = re + phi[l] * mx.t[l].rho_eref -
         phi[l] * mx.t[l].pref * mx.t[l].invG;
  return re;
}

template <int NM, class C>
FV_HD C solid_frac(const C* phi) {
  C s = 0;
#pragma unroll
  for (int l = 0; l < NM; ++l) s += phi[l];
  return m_clamp(s, (C)0, (C)1);
}

// returns c, writes G_mix
template <int NM, int NS, class C>
FV_HD C mix_sound(const Params& P, const C* phi, const Mix<NM, NS, C>& mx, C p,
                  C rho, C& Gmix) {
  C acc = 0;
  Gmix = 0;
#pragma unroll
  for (int l = 0; l < NM; ++l) {
    // thermal term non-negative: a state below the cold curve (a gas
    // fraction pulled into tension) must not collapse the wave speed
    acc += phi[l] * mx.t[l].invG *
           (mx.t[l].rho_dpref + mx.t[l].g1 * m_max(p - mx.t[l].pref, (C)0));
    Gmix += phi[l] * mx.t[l].G;
  }
  const C cb2 = solid_frac<NM>(phi) * acc / (mx.xi * rho);
  const C c2 = m_max(cb2, (C)0) + (C)(4.0 / 3.0) * Gmix / rho;
  return m_sqrt(m_max(c2, cst<C>(P.c_min2, P.f_c_min2)));
}

// ----------------------------------------------------------------------------
// kinematics: deviatoric Hencky strain of Vbar (Section 2.2, dev H = ln Vbar)
// taken as 1/2 ln(Vbar Vbar^T) with the trace removed.
// ----------------------------------------------------------------------------
// log of a symmetric positive-definite 2x2 matrix M = [[b00, b01], [b01, b11]]
// given ld = ln(det M) / 2:
// log M = ld I + g (M - m I), m = tr/2, r = eigen half-gap,
// g = (ln l1 - ln l2)/(l1 - l2) = (ln l1 - ld)/r with l1 = m + r the larger
// eigenvalue (series in r/m for a small gap).  With M = V V^T the caller
// passes ld = ln|det V|: det M formed from M's entries cancels to nothing
// for a strongly sheared V (eigenvalue ratio near the rounding unit), and
// atanh(r/m) = g r would then see r/m round to 1.
template <class C>
FV_HD void sym2_log(C b00, C b01, C b11, C ld, C& l00, C& l01, C& l11) {
  const C m = (C)0.5 * (b00 + b11);
  const C d = (C)0.5 * (b00 - b11);
  const C r = m_sqrt(d * d + b01 * b01);
  const C x = r / m;
  const C xs = sizeof(C) == 8 ? (C)1e-3 : (C)5e-2;
  C g;
  if (x < xs) {
    const C x2 = x * x;
    g = ((C)1 + x2 * ((C)(1.0 / 3.0) + x2 * ((C)0.2 + x2 * (C)(1.0 / 7.0)))) / m;
  } else {
    g = (m_log(m + r) - ld) / r;
  }
  l00 = ld + g * d;
  l11 = ld - g * d;
  l01 = g * b01;
}

// exp of a symmetric 2x2 matrix [[a00, a01], [a01, a11]]:
// exp(A) = e^m [cosh(r) I + sinh(r)/r (A - m I)].
template <class C>
FV_HD void sym2_exp(C a00, C a01, C a11, C& e00, C& e01, C& e11) {
  const C m = (C)0.5 * (a00 + a11);
  const C d = (C)0.5 * (a00 - a11);
  const C r = m_sqrt(d * d + a01 * a01);
  const C em = m_exp(m);
  C ch, sh;
  const C rs = sizeof(C) == 8 ? (C)1e-3 : (C)5e-2;
  if (r < rs) {
    const C r2 = r * r;
    ch = (C)1 + r2 * ((C)0.5 + r2 * ((C)(1.0 / 24.0) + r2 * (C)(1.0 / 720.0)));
    sh = (C)1 + r2 * ((C)(1.0 / 6.0) + r2 * ((C)(1.0 / 120.0) + r2 * (C)(1.0 / 5040.0)));
  } else {
    const C ep = m_exp(r), en = m_exp(-r);
    ch = (C)0.5 * (ep + en);
    sh = (C)0.5 * (ep - en) / r;
  }
  e00 = em * (ch + sh * d);
  e11 = em * (ch - sh * d);
  e01 = em * sh * a01;
}

// Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations
// (each rotation zeroes one off-diagonal pair; sweeps repeat until the
// off-diagonal mass is below rounding).  Degenerate eigenvalues need no
// special case, which matters for the near-identity stretches of an elastic
// solid.  A is overwritten by its diagonal form, Q collects the rotations
// (columns are eigenvectors).
template <int P_, int Q_, int R_, class C>
FV_HD void jacobi_rotate(C A[3][3], C Q[3][3]) {
  const C apq = A[P_][Q_];
  // An off-diagonal entry below the rounding of the diagonal pair is already
  // zero.  The absolute floor keeps 1 / (2 apq) finite: with reciprocal
  // division a degenerate pair (equal diagonal) and a denormal apq would
  // otherwise give 0 * inf.
  const C rel = sizeof(C) == 8 ? (C)1e-18 : (C)1e-9;
  const C floor_abs = sizeof(C) == 8 ? (C)1e-280 : (C)1e-30;
  if (m_abs(apq) <= rel * (m_abs(A[P_][P_]) + m_abs(A[Q_][Q_])) || m_abs(apq) < floor_abs) {
    A[P_][Q_] = A[Q_][P_] = (C)0;
    return;
  }
  const C theta = (A[Q_][Q_] - A[P_][P_]) / ((C)2 * apq);
  const C at = m_abs(theta);
  // t = tan of the rotation angle, the smaller root of t^2 + 2 theta t - 1
  const C t0 = (C)1 / (at + m_sqrt(at * at + (C)1));
  const C t = theta < (C)0 ? -t0 : t0;
  const C cs = (C)1 / m_sqrt(t * t + (C)1);
  const C sn = t * cs;
  A[P_][P_] -= t * apq;
  A[Q_][Q_] += t * apq;
  A[P_][Q_] = A[Q_][P_] = (C)0;
  const C arp = A[R_][P_], arq = A[R_][Q_];
  A[R_][P_] = A[P_][R_] = cs * arp - sn * arq;
  A[R_][Q_] = A[Q_][R_] = sn * arp + cs * arq;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const C qp = Q[k][P_], qq = Q[k][Q_];
    Q[k][P_] = cs * qp - sn * qq;
    Q[k][Q_] = sn * qp + cs * qq;
  }
}

template <class C>
FV_HD void sym3_eig(C A[3][3], C Q[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Q[i][j] = i == j ? (C)1 : (C)0;
  const C eps = sizeof(C) == 8 ? (C)1e-32 : (C)1e-15;   // squared rounding
  const int max_sweeps = sizeof(C) == 8 ? 10 : 8;
  for (int s = 0; s < max_sweeps; ++s) {
    const C off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const C dg = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= eps * dg || off == (C)0) break;
    jacobi_rotate<0, 1, 2>(A, Q);
    jacobi_rotate<0, 2, 1>(A, Q);
    jacobi_rotate<1, 2, 0>(A, Q);
  }
}

// Q diag(f) Q^T
template <class C>
FV_HD void sym3_compose(const C Q[3][3], const C f[3], C M[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      M[i][j] = Q[i][0] * f[0] * Q[j][0] + Q[i][1] * f[1] * Q[j][1] + Q[i][2] * f[2] * Q[j][2];
}

// Half logs of the eigenvalues of B = V V^T from its diagonalised form
// (B[k][k] after sym3_eig): the two larger ones directly, the smallest from
// det B = det(V)^2, since an eigenvalue far below the rounding of the largest
// is lost in B itself (a strongly sheared V).
template <class C>
FV_HD void half_log_eigs3(const C V[3][3], const C B[3][3], C h[3]) {
  const C detv = V[0][0] * (V[1][1] * V[2][2] - V[1][2] * V[2][1]) -
                 V[0][1] * (V[1][0] * V[2][2] - V[1][2] * V[2][0]) +
                 V[0][2] * (V[1][0] * V[2][1] - V[1][1] * V[2][0]);
  const int k0 = B[0][0] <= B[1][1] ? (B[0][0] <= B[2][2] ? 0 : 2) : (B[1][1] <= B[2][2] ? 1 : 2);
  const int k1 = (k0 + 1) % 3, k2 = (k0 + 2) % 3;
  h[k1] = (C)0.5 * m_log(B[k1][k1]);
  h[k2] = (C)0.5 * m_log(B[k2][k2]);
  h[k0] = m_log(m_abs(detv)) - h[k1] - h[k2];
}

// dev H (full symmetric 3x3, zeros where the dimension keeps them zero)
template <int DIM, class C>
FV_HD void hencky(const C V[3][3], C H[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) H[i][j] = 0;
  if (DIM == 1) {
    const C h0 = m_log(m_abs(V[0][0])), h1 = m_log(m_abs(V[1][1])), h2 = m_log(m_abs(V[2][2]));
    const C mm = (h0 + h1 + h2) / (C)3;
    H[0][0] = h0 - mm; H[1][1] = h1 - mm; H[2][2] = h2 - mm;
  } else if (DIM == 3) {
    // B = V V^T, H = 1/2 ln B through its eigen-decomposition
    C B[3][3], Q[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        B[i][j] = V[i][0] * V[j][0] + V[i][1] * V[j][1] + V[i][2] * V[j][2];
    sym3_eig(B, Q);
    C h[3];
    half_log_eigs3(V, B, h);
    const C mm = (h[0] + h[1] + h[2]) / (C)3;
#pragma unroll
    for (int k = 0; k < 3; ++k) h[k] -= mm;
    sym3_compose(Q, h, H);
  } else {
    const C b00 = V[0][0] * V[0][0] + V[0][1] * V[0][1];
    const C b01 = V[0][0] * V[1][0] + V[0][1] * V[1][1];
    const C b11 = V[1][0] * V[1][0] + V[1][1] * V[1][1];
    C l00, l01, l11;
    const C ld = m_log(m_abs(V[0][0] * V[1][1] - V[0][1] * V[1][0]));
    sym2_log(b00, b01, b11, ld, l00, l01, l11);
    const C h00 = (C)0.5 * l00, h11 = (C)0.5 * l11, h01 = (C)0.5 * l01;
    const C h22 = m_log(m_abs(V[2][2]));
    const C mm = (h00 + h11 + h22) / (C)3;
    H[0][0] = h00 - mm; H[1][1] = h11 - mm; H[2][2] = h22 - mm;
    H[0][1] = h01; H[1][0] = h01;
  }
}

template <int DIM, class C>
FV_HD C J2_of(const C H[3][3]) {
  C s = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) s += H[i][j] * H[i][j];
  return s;
}

// symmetric unimodular stretch exp(H) for a trace-free symmetric H
template <int DIM, class C>
FV_HD void stretch_from_log(const C H[3][3], C V[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V[i][j] = 0;
  if (DIM == 1) {
    V[0][0] = m_exp(H[0][0]); V[1][1] = m_exp(H[1][1]); V[2][2] = m_exp(H[2][2]);
  } else if (DIM == 3) {
    C A[3][3], Q[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) A[i][j] = H[i][j];
    sym3_eig(A, Q);
    C e[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) e[k] = m_exp(A[k][k]);
    sym3_compose(Q, e, V);
  } else {
    C e00, e01, e11;
    sym2_exp(H[0][0], H[0][1], H[1][1], e00, e01, e11);
    V[0][0] = e00; V[0][1] = e01; V[1][0] = e01; V[1][1] = e11;
    V[2][2] = m_exp(H[2][2]);
  }
}

// ----------------------------------------------------------------------------
// limiter and WENO3 (reconstruction readings of Section 3 / Section 3.2.1)
// ----------------------------------------------------------------------------
template <class C> FV_HD C van_leer(C dm, C dp) {
  const C pr = dm * dp;
  return pr > (C)0 ? (C)2 * pr / (dm + dp) : (C)0;
}

// THINC (Xiao, Honma and Kono 2005): in a cell whose value q0 lies strictly
// between its neighbours qm and q1, the profile q_min + (dq/2)(1 + theta
// tanh(beta (x - x_c))) over the unit cell with the cell average q0.  With
// C = (q0 - q_min)/dq, B = exp(theta beta (2C - 1)) and
// A = (B sech(beta) - 1)/tanh(beta), the lower-face value is
// q_min + (dq/2)(1 + theta A) and the upper-face value
// q_min + (dq/2)(1 + theta (tanh(beta) + A)/(1 + A tanh(beta))).  Returns
// false where the profile is not used (not monotone, or C within 1e-6 of
// 0 or 1).
constexpr double THINC_EPS = 1.0e-6;

template <class C>
FV_HD bool thinc_cell(C qm, C q0, C q1, C beta, C tb, C sech, C* lower, C* upper) {
  if (!((q1 - q0) * (q0 - qm) > (C)0)) return false;
  const C qmin = m_min(qm, q1);
  const C dq = m_abs(q1 - qm);
  const C cn = (q0 - qmin) / dq;
  if (!(cn > (C)THINC_EPS && cn < (C)1 - (C)THINC_EPS)) return false;
  const C th = q1 >= qm ? (C)1 : (C)-1;
  const C B = m_exp(th * beta * ((C)2 * cn - (C)1));
  const C A = (B * sech - (C)1) / tb;
  if (lower) *lower = qmin + (C)0.5 * dq * ((C)1 + th * A);
  if (upper) *upper = qmin + (C)0.5 * dq * ((C)1 + th * (tb + A) / ((C)1 + A * tb));
  return true;
}

// face value from the left (upwind cell q0; stencil qm, q0, q1)
template <class C> FV_HD C weno3_left(C qm, C q0, C q1, C eps) {
  const C p0 = (C)-0.5 * qm + (C)1.5 * q0;
  const C p1 = (C)0.5 * q0 + (C)0.5 * q1;
  const C b0 = (q0 - qm) * (q0 - qm);
  const C b1 = (q1 - q0) * (q1 - q0);
  const C a0 = (C)(1.0 / 3.0) / ((eps + b0) * (eps + b0));
  const C a1 = (C)(2.0 / 3.0) / ((eps + b1) * (eps + b1));
  return (a0 * p0 + a1 * p1) / (a0 + a1);
}

// ----------------------------------------------------------------------------
// Imposed-velocity driver of the ring (Section 4.3): the radial speed
// v_r(t) = v0 t/t0 (t < t0), v0 + (v1 - v0)(t - t0)/(t1 - t0) (t0 < t < t1),
// v1 afterwards; the driver surface starts at the ring's inner radius and
// moves with v_r, R_d(t) = r_in + the integral of v_r, until it reaches
// r_max.  drv = {r_in, v0, v1, t0, t1, r_max}.
// ----------------------------------------------------------------------------
FV_HD double driver_speed(const double* d, double t) {
  if (t < d[3]) return d[1] * t / d[3];
  if (t < d[4]) return d[1] + (d[2] - d[1]) * (t - d[3]) / (d[4] - d[3]);
  return d[2];
}

FV_HD double driver_radius(const double* d, double t) {
  const double v0 = d[1], v1 = d[2], t0 = d[3], t1 = d[4];
  if (t < t0) return d[0] + 0.5 * v0 * t * t / t0;
  const double a = d[0] + 0.5 * v0 * t0;
  if (t < t1) {
    const double s = t - t0;
    return a + v0 * s + 0.5 * (v1 - v0) * s * s / (t1 - t0);
  }
  return a + 0.5 * (v0 + v1) * (t1 - t0) + v1 * (t - t1);
}

// ----------------------------------------------------------------------------
// Johnson-Cook plasticity: the law of Johnson and Cook (1983) with the
// constants of the paper's plasticity table (the paper names the law and
// tabulates c1..C_V without printing it).  Reference rate 1/s (slower rates
// keep the quasi-static yield) and reference temperature 300 K, of the law
// and of the thermal energy C_V (T - T_ref theta_D(rho)) of Section 2.2.
// ----------------------------------------------------------------------------
constexpr double JC_T_REF = 300.0;
constexpr double JC_RATE_REF = 1.0;

// Phase temperature: thermal energy per unit mass (p - p_ref)/(rho Gamma0)
// of the Mie-Grueneisen form, non-negative, over C_V, plus T_ref eta^Gamma0
// (the Romenskii Debye temperature).
FV_HD double jc_temperature(const MatP& m, double p, double pref, double rho) {
  if (!(m.CV > 0.0)) return JC_T_REF;
  const double eta = rho / m.rho0;
  double gam = m.Gamma0, th = pow(eta, m.Gamma0);
  if (m.bp) {
    // Burakovsky-Preston: Gamma(rho) and the Debye temperature
    // eta^Gamma0 exp[3 G1 (1 - eta^(-1/3)) + (G2/gbp)(1 - eta^(-gbp))]
    const double e3 = 1.0 / cbrt(eta), eg = pow(eta, -m.gbp);
    gam = m.Gamma0 + m.G1 * e3 + m.G2 * eg;
    th *= exp(3.0 * m.G1 * (1.0 - e3) + (m.G2 / m.gbp) * (1.0 - eg));
  }
  const double et = (p - pref > 0.0 ? p - pref : 0.0) / (rho * gam);
  return et / m.CV + JC_T_REF * th;
}

// Flow stress at plastic strain eps_n + dg, rate dg/dt and temperature T;
// *dY receives its derivative in dg (the rate term's where the rate
// exceeds the reference, the hardening term's where the strain is positive).
FV_HD double jc_yield(const MatP& m, double eps_n, double dg, double dt, double T, double* dY) {
  const double x = eps_n + dg > 0.0 ? eps_n + dg : 0.0;
  double hard = m.yield, dhard = 0.0;
  if (m.jcB != 0.0) {
    const double xn = pow(x, m.nhard);
    hard += m.jcB * xn;
    if (x > 0.0) dhard = m.jcB * m.nhard * xn / x;
  }
  double rf = 1.0, drf = 0.0;
  if (m.jcC != 0.0 && dt > 0.0) {
    const double r = dg / dt / JC_RATE_REF;
    if (r > 1.0) { rf = 1.0 + m.jcC * log(r); drf = m.jcC / dg; }
  }
  double tf = 1.0;
  if (m.Tmelt > 0.0) {
    double ts = (T - JC_T_REF) / (m.Tmelt - JC_T_REF);
    ts = ts < 0.0 ? 0.0 : (ts > 1.0 ? 1.0 : ts);
    tf = 1.0 - pow(ts, m.jcm);
  }
  if (dY) *dY = (dhard * rf + hard * drf) * tf;
  return hard * rf * tf;
}

// ----------------------------------------------------------------------------
// Bonora damage (Section 2.2)
// ----------------------------------------------------------------------------
FV_HD double triaxiality(const MatP& m, double p, double seq, double rho) {
  const double q = p / seq;
  return 3.0 * (1.0 - 2.0 * m.nu) * (m.rho0 / rho) * q * q + (2.0 / 3.0) * (1.0 + m.nu);
}

FV_HD double eps_threshold(const MatP& m, double R) {
  const double et = m.eps_th, ec = m.eps_c, n = m.nhard;
  const double num = pow(ec, 2.0 * n) - pow(et, 2.0 * n);
  const double den = pow(ec, 2.0 * n / R) - pow(et, 2.0 * n / R);
  return pow(et, 1.0 / R) / pow(R, 1.0 / n) * pow(num / den, 1.0 / (2.0 * n));
}

FV_HD double bonora_rate(const MatP& m, double D, double eps, double R) {
  if (D >= m.Dcrit) return 0.0;
  const double y = m.Dcrit - D;
  return m.bonA * R * pow(y, m.bonExp) / eps;
}

// classical RK4 in eps_p over [eps0, eps0 + h], every argument clamped
// dD/deps: the Bonora rate, or Ddot0 (1 - D) for the simplified law of the
// U-Nb ring (Section 4.3); zero once critical either way
template <bool EXT = true>
FV_HD double damage_rate(const MatP& m, double D, double eps, double R) {
  if (EXT && m.Ddot0 > 0.0) return D >= m.Dcrit ? 0.0 : m.Ddot0 * (1.0 - D);
  return bonora_rate(m, D, eps, R);
}

template <bool EXT = true>
FV_HD double damage_rk4(const MatP& m, double D, double eps0, double h, double R) {
  const double Dc = m.Dcrit;
  auto cl = [Dc](double v) { return v < 0.0 ? 0.0 : (v > Dc ? Dc : v); };
  const double k1 = damage_rate<EXT>(m, D, eps0, R);
  const double k2 = damage_rate<EXT>(m, cl(D + 0.5 * h * k1), eps0 + 0.5 * h, R);
  const double k3 = damage_rate<EXT>(m, cl(D + 0.5 * h * k2), eps0 + 0.5 * h, R);
  const double k4 = damage_rate<EXT>(m, cl(D + h * k3), eps0 + h, R);
  return cl(D + h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4));
}

}  // namespace fv

// Host stepping of the device kernels' phase functions, for running them under
// AddressSanitizer and UndefinedBehaviorSanitizer on the CPU (test support;
// built with g++, no GPU code).
//
// 1D and 2D follow the stage kernel's tiles: primitives of every tile cell
// with its halo, the faces of each direction into the face buffer, the gather
// per owned cell, then update, source and CFL.  3D follows the three passes:
// primitives of every cell, faces of each direction, then gather with update,
// source and CFL.  The shared-memory tile and the face buffers are exactly the
// sizes the kernels use and start as NaN, so a phase that reads a slot no
// earlier phase wrote poisons the result; every index the glue forms is
// asserted in range.
//
// Input (binary, native endian): fv_grid, int32 n_mat, n_mat fv_material,
// fv_options, int64 S, int64 ncell, int32 steps, int32 tile_x, then the
// primitive state (S x ncell doubles, field-major) and phi0 (ncell doubles).
// tile_x picks the 2D two-material tile: 32 (32 x 8), 16 (16 x 15 cells on
// 256 threads), 14 (16 x 14 cells on 256 threads), else 8 x 4.
// Output: time, device flag, then the conserved state (S x ncell doubles).
#include <algorithm>
#include <cassert>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/fv.h"
#include "../../paper_2210_04037_amd/csrc/fv_stage.hpp"

using namespace fv;

static void fill_params(const fv_material* mats, int n_mat, const fv_options* opt, Params& P) {
  std::memset(&P, 0, sizeof(P));
  for (int l = 0; l < n_mat; ++l) {
    const fv_material& m = mats[l];
    MatP& q = P.mat[l];
    q.kind = m.kind == FV_MAT_SOLID ? 0 : 1;
    q.rho0 = m.rho0; q.K0 = m.K0; q.alpha = m.alpha; q.G0 = m.G0; q.beta = m.beta;
    q.Gamma0 = m.Gamma0; q.yield = m.yield; q.Dcrit = m.D_crit; q.D0 = m.D0;
    q.eps_th = m.eps_th; q.eps_c = m.eps_c; q.balpha = m.bonora_alpha;
    q.nhard = m.n_hard; q.pgate = m.p_gate;
    q.jcB = m.jc_B; q.jcC = m.jc_C; q.jcm = m.jc_m; q.Tmelt = m.T_melt; q.CV = m.C_V;
    q.jc = q.kind == 0 && (m.jc_B != 0.0 || m.jc_C != 0.0 || m.T_melt > 0.0);
    q.Gp = m.G_p; q.G1 = m.Gamma1; q.G2 = m.Gamma2; q.gbp = m.gamma_bp; q.Ddot0 = m.Ddot0;
    q.stein = q.kind == 0 && m.G_p > 0.0;
    q.bp = q.kind == 0 && (m.Gamma1 != 0.0 || m.Gamma2 != 0.0);
    q.invGamma = 1.0 / m.Gamma0;
    auto small_int = [](double v) {
      const double r = std::round(v);
      return (r == v && r >= 1 && r <= 8) ? (int)r : 0;
    };
    if (q.kind == 0) {
      q.alpha_i = small_int(m.alpha);
      q.beta1_i = small_int(m.beta + 1.0);
      set_solid_constants(q);
    }
  }
  P.cfl = opt->cfl;
  P.phi_floor = opt->phi_floor;
  P.weno_eps = opt->weno_eps;
  P.c_min2 = 1.0e-6;
  P.phi_fp64_cut = opt->phi_fp64_cut;
  P.seed_nu = opt->seed_nu;
  P.thinc_beta = opt->thinc_beta;
  for (int k = 0; k < 6; ++k) P.drv[k] = opt->driver[k];
  set_float_constants(P);
}

struct Run {
  Params P;
  Inst I;
  int64_t nc = 0;
  std::vector<double> U, U1, U2, phi0, bacc, dts, Wb, Acc;
};

template <int DIM, int NM, int NS>
static void setup(Run& r, const fv_grid* g, const fv_material* mats, const fv_options* o,
                  const double* prim, const double* phi0) {
  using L = Lay<DIM, NM, NS>;
  using St = Stage<DIM, NM, NS, double, double, 1, 1>;
  fill_params(mats, NM, o, r.P);
  std::memset(&r.I, 0, sizeof(r.I));
  r.nc = (int64_t)g->n[0] * g->n[1] * g->n[2];
  r.U.assign(L::S * r.nc, 0.0);
  r.U1.assign(L::S * r.nc, NAN);
  r.U2.assign(L::S * r.nc, NAN);
  r.phi0.assign(phi0, phi0 + r.nc);
  for (int k = 0; k < 3; ++k) {
    r.I.n[k] = g->n[k];
    r.I.lo[k] = g->lo[k];
    r.I.dx[k] = (g->hi[k] - g->lo[k]) / g->n[k];
    r.I.bc[k][0] = g->bc[k][0];
    r.I.bc[k][1] = g->bc[k][1];
  }
  int off = 0;
  for (int a = 0; a < 3; ++a) {
    const int nt = a < DIM ? (int)(r.nc / g->n[a]) : 0;
    r.I.bacc_off[2 * a] = off;
    off += nt * L::NC;
    r.I.bacc_off[2 * a + 1] = off;
    off += nt * L::NC;
  }
  r.bacc.assign(off, 0.0);
  r.dts.assign(DTS_SIZE, 0.0);
  r.I.ncell = r.nc;
  r.I.U = r.U.data();
  r.I.U1 = r.U1.data();
  r.I.U2 = r.U2.data();
  r.I.phi0 = r.phi0.data();
  r.I.bacc = r.bacc.data();
  r.I.dts = r.dts.data();
  if (DIM == 3) {
    r.Wb.assign(L::NW * r.nc, NAN);
    r.Acc.assign(L::S * r.nc, NAN);
    r.I.Acc = r.Acc.data();
    r.I.Wb = r.Wb.data();
  }
  double m = 0.0;
  for (int64_t c = 0; c < r.nc; ++c) {
    double W[L::S], Uc[L::S];
    for (int f = 0; f < L::S; ++f) W[f] = prim[f * r.nc + c];
    Cell<DIM, NM, NS>::prim_to_cons(r.P, W, Uc);
    for (int f = 0; f < L::S; ++f) r.U[f * r.nc + c] = Uc[f];
    m = std::max(m, St::cfl_sum(r.P, r.I, Uc));
  }
  r.dts[DTS_TEND] = HUGE_VAL;
  dts_set_dtinv(r.dts.data(), 0, m);
}

// time step of a stage; the first stage advances the other parity's time slot
// and clears its CFL slot, as the device does
static double stage_dt(Run& r, int stage, int q) {
  const double t = r.dts[DTS_T + q];
  const double dt = std::min(r.P.cfl / dts_dtinv(r.dts.data(), q), r.dts[DTS_TEND] - t);
  if (stage == 1) {
    r.dts[DTS_T + 1 - q] = t + dt;
    dts_set_dtinv(r.dts.data(), 1 - q, 0.0);
  }
  return dt;
}

template <class Ctx>
static void init_ctx(Ctx& cx, Run& r, int stage, int q, double dt) {
  cx.I = &r.I;
  cx.P = r.P;
  cx.stage = stage;
  cx.dry = false;
  cx.parity = q;
  cx.bx = 0;
  cx.by = 0;
  cx.dt = dt;
  cx.tn = r.dts[DTS_T + q] + dt;
  cx.base = r.U.data();
  cx.src = stage == 1 ? r.U.data() : (stage == 2 ? r.U1.data() : r.U2.data());
  cx.out = stage == 1 ? r.U1.data() : (stage == 2 ? r.U2.data() : r.U.data());
}

// Lagrangian seeding after a step, as the device's two passes: every cell's
// new coordinates from the state before seeding, then copied back.
template <int DIM, int NM, int NS>
static void seed_all(Run& r, int nq) {
  using St = Stage<DIM, NM, NS, double, double, 1, 1>;
  using L = Lay<DIM, NM, NS>;
  if (!(r.P.seed_nu > 0)) return;
  std::vector<double> X((size_t)DIM * r.nc, NAN);
  for (int64_t g = 0; g < r.nc; ++g) {
    double Xn[DIM];
    St::seed_cell(r.P, r.I, r.U.data(), g, Xn);
    for (int k = 0; k < DIM; ++k) X[(size_t)k * r.nc + g] = Xn[k];
  }
  for (int k = 0; k < DIM; ++k)
    for (int64_t g = 0; g < r.nc; ++g) r.U[(size_t)(L::XC + k) * r.nc + g] = X[(size_t)k * r.nc + g];
  // one solid: the void relaxation, and the next step's CFL value from the
  // relaxed state (the device's copy-back pass)
  if (!relax_on(r.P, NM, NS)) return;
  double m = 0.0;
  for (int64_t g = 0; g < r.nc; ++g) {
    double Uc[L::S];
    for (int f = 0; f < L::S; ++f) Uc[f] = r.U[(size_t)f * r.nc + g];
    St::relax_void_cell(r.P, Uc);
    r.U[(size_t)L::PHI * r.nc + g] = Uc[L::PHI];
    const double v = St::cfl_sum(r.P, r.I, Uc);
    if (!(v == v)) r.dts[DTS_FLAG] = 1.0;
    else m = std::max(m, v);
  }
  r.dts[dts_slot(nq, 0)] = m;
}

template <int DIM, int NM, int NS, int TX, int TY, int NTH = TX * TY>
static void step_tiles(Run& r, int nsteps) {
  using St = Stage<DIM, NM, NS, double, double, TX, TY, NTH>;
  using TL = typename St::TL;
  std::vector<double> sm(St::smem_elems());
  r.I.tiles[0] = (r.I.n[0] + TX - 1) / TX;
  r.I.tiles[1] = DIM >= 2 ? (r.I.n[1] + TY - 1) / TY : 1;
  r.I.tiles[2] = 1;
  std::vector<double> acc((size_t)TL::NT * St::S);
  for (int s = 0; s < nsteps; ++s) {
    const int q = s & 1;
    for (int stage = 1; stage <= 3; ++stage) {
      const double dt = stage_dt(r, stage, q);
      double bmax = 0.0;
      for (int by = 0; by < r.I.tiles[1]; ++by)
        for (int bx = 0; bx < r.I.tiles[0]; ++bx) {
          typename St::Ctx cx;
          init_ctx(cx, r, stage, q, dt);
          cx.bx = bx;
          cx.by = by;
          std::fill(sm.begin(), sm.end(), NAN);
          double* W = sm.data();
          double* fb = W + (size_t)St::NW * TL::NCELL;
          for (int tc = 0; tc < TL::NCELL; ++tc) St::load_cell(cx, W, tc);
          std::fill(acc.begin(), acc.end(), 0.0);
          for (int a = 0; a < DIM; ++a) {
            for (int it = 0; it < St::face_items(a); ++it) {
              int cm, c0, c1, c2, gf, fs, bs;
              if (!St::face_item(cx, a, it, cm, c0, c1, c2, gf, fs, bs)) continue;
              assert(cm >= 0 && cm < TL::NCELL && c0 >= 0 && c0 < TL::NCELL);
              assert(c1 >= 0 && c1 < TL::NCELL && c2 >= 0 && c2 < TL::NCELL);
              assert(fs >= 0 && fs < TL::NFACE);
              St::template compute_face<int>(cx, W, TL::NCELL, a, cm, c0, c1, c2, gf, fs,
                                             TL::NFACE, bs, fb);
            }
            for (int tid = 0; tid < TL::NT; ++tid) {
              int tx, ty;
              int64_t g;
              if (St::own_cell(cx, tid, tx, ty, g))
                St::gather(cx, W, fb, a, tx, ty, &acc[(size_t)tid * St::S]);
            }
          }
          for (int tid = 0; tid < TL::NT; ++tid) {
            int tx, ty;
            int64_t g;
            if (!St::own_cell(cx, tid, tx, ty, g)) continue;
            assert(g >= 0 && g < r.nc);
            bool bad = false;
            bmax = std::max(bmax, St::finish_cell(cx, g, &acc[(size_t)tid * St::S], &bad));
            if (bad) r.dts[DTS_FLAG] = 1.0;
          }
        }
      if (stage == 3) r.dts[dts_slot(1 - q, 0)] = bmax;
    }
    seed_all<DIM, NM, NS>(r, 1 - q);
  }
}

// The 3D stage as the device runs it: primitives of every cell, the x-face
// runs through a block-sized buffer (the kernel's LDS), the y and z marches
// over the bricks of their launches, then the per-cell update from the sums.
template <int NM, int NS>
static void step_3d(Run& r, int nsteps) {
  using St = Stage<3, NM, NS, double, double, 1, 1>;
  using L = Lay<3, NM, NS>;
  const int64_t nc = r.nc;
  const int nx = r.I.n[0], ny = r.I.n[1], nz = r.I.n[2];
  double* Wb = r.Wb.data();
  double* Ab = r.Acc.data();
  std::vector<double> fb((size_t)L::NQ * (St::XRUN + 1));
  for (int s = 0; s < nsteps; ++s) {
    const int q = s & 1;
    for (int stage = 1; stage <= 3; ++stage) {
      const double dt = stage_dt(r, stage, q);
      typename St::Ctx cx;
      init_ctx(cx, r, stage, q, dt);
      for (int64_t g = 0; g < nc; ++g) St::template cell_prims<int64_t, true>(cx, g, Wb, nc, g);
      std::fill(r.Acc.begin(), r.Acc.end(), NAN);
      const int64_t nb = St::xrun_count(r.I);
      for (int64_t b = 0; b < nb; ++b) {
        std::fill(fb.begin(), fb.end(), NAN);
        for (int t = 0; t < St::XRUN + 1; ++t) St::xrun_face(cx, Wb, b, t, fb.data());
        for (int t = 0; t < St::XRUN + 1; ++t) St::xrun_cell(cx, Wb, b, t, fb.data(), Ab);
      }
      // the x pass starts every cell's sum
      for (size_t k = 0; k < r.Acc.size(); ++k) assert(!std::isnan(Ab[k]));
      for (int a = 1; a <= 2; ++a) {
        const int nu = a == 1 ? nz : ny, ns = St::march_runs(r.I, a);
        const int64_t nbb = brick_blocks(nx, nu, ns);
        for (int64_t b = 0; b < nbb; ++b)
          for (int tid = 0; tid < 256; ++tid) {
            int x, u, sr;
            if (!brick_pos(b, tid, nx, nu, ns, x, u, sr)) continue;
            assert(x >= 0 && x < nx && u >= 0 && u < nu && sr >= 0 && sr < ns);
            St::march_cells(cx, Wb, a, x, u, sr, Ab);
          }
      }
      double bmax = 0.0;
      for (int64_t g = 0; g < nc; ++g) {
        double acc[L::S];
        for (int f = 0; f < L::S; ++f) acc[f] = Ab[(size_t)f * nc + g];
        bool bad = false;
        bmax = std::max(bmax, St::finish_cell(cx, g, acc, &bad));
        if (bad) r.dts[DTS_FLAG] = 1.0;
      }
      if (stage == 3) r.dts[dts_slot(1 - q, 0)] = bmax;
    }
    seed_all<3, NM, NS>(r, 1 - q);
  }
}

template <class T>
static bool get(FILE* f, T* p, size_t n) {
  return std::fread(p, sizeof(T), n, f) == n;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: phase_step in.bin out.bin\n");
    return 2;
  }
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  fv_grid g;
  int32_t nm = 0, nsteps = 0, tx = 0;
  fv_material m[2];
  fv_options o;
  int64_t S = 0, nc = 0;
  bool ok = get(f, &g, 1) && get(f, &nm, 1) && nm >= 1 && nm <= 2 && get(f, m, nm) &&
            get(f, &o, 1) && get(f, &S, 1) && get(f, &nc, 1) && get(f, &nsteps, 1) &&
            get(f, &tx, 1) && S > 0 && nc > 0 && nc == (int64_t)g.n[0] * g.n[1] * g.n[2];
  std::vector<double> prim, phi0;
  if (ok) {
    prim.resize(S * nc);
    phi0.resize(nc);
    ok = get(f, prim.data(), prim.size()) && get(f, phi0.data(), phi0.size());
  }
  std::fclose(f);
  int ns = 0;
  for (int l = 0; ok && l < nm; ++l) ns += m[l].kind == FV_MAT_SOLID;
  if (!ok || ns < 1 || ns > 2 || (ns == 2 && (nm != 2 || g.dim == 3))) {
    std::fprintf(stderr, "phase_step: bad input\n");
    return 2;
  }
  Run r;
  const double* P = prim.data();
  const double* Z = phi0.data();
  if (ns == 2 && g.dim == 1) {
    setup<1, 2, 2>(r, &g, m, &o, P, Z);
    step_tiles<1, 2, 2, 16, 1>(r, nsteps);
  } else if (ns == 2 && tx == 16) {
    // the FP64 default shape: 16 x 15 cells on 256 threads
    setup<2, 2, 2>(r, &g, m, &o, P, Z);
    step_tiles<2, 2, 2, 16, 15, 256>(r, nsteps);
  } else if (ns == 2) {
    setup<2, 2, 2>(r, &g, m, &o, P, Z);
    step_tiles<2, 2, 2, 8, 4>(r, nsteps);
  } else if (g.dim == 1 && nm == 1) {
    setup<1, 1, 1>(r, &g, m, &o, P, Z);
    step_tiles<1, 1, 1, 16, 1>(r, nsteps);
  } else if (g.dim == 1) {
    setup<1, 2, 1>(r, &g, m, &o, P, Z);
    step_tiles<1, 2, 1, 16, 1>(r, nsteps);
  } else if (g.dim == 2 && nm == 1) {
    setup<2, 1, 1>(r, &g, m, &o, P, Z);
    step_tiles<2, 1, 1, 8, 4>(r, nsteps);
  } else if (g.dim == 2 && tx == 32) {
    setup<2, 2, 1>(r, &g, m, &o, P, Z);
    step_tiles<2, 2, 1, 32, 8>(r, nsteps);
  } else if (g.dim == 2 && tx == 16) {
    // more threads than interior cells: 16 x 15 cells, 256 threads
    setup<2, 2, 1>(r, &g, m, &o, P, Z);
    step_tiles<2, 2, 1, 16, 15, 256>(r, nsteps);
  } else if (g.dim == 2 && tx == 14) {
    setup<2, 2, 1>(r, &g, m, &o, P, Z);
    step_tiles<2, 2, 1, 16, 14, 256>(r, nsteps);
  } else if (g.dim == 2) {
    setup<2, 2, 1>(r, &g, m, &o, P, Z);
    step_tiles<2, 2, 1, 8, 4>(r, nsteps);
  } else if (g.dim == 3 && nm == 1) {
    setup<3, 1, 1>(r, &g, m, &o, P, Z);
    step_3d<1, 1>(r, nsteps);
  } else if (g.dim == 3) {
    setup<3, 2, 1>(r, &g, m, &o, P, Z);
    step_3d<2, 1>(r, nsteps);
  } else {
    std::fprintf(stderr, "phase_step: unsupported dimension\n");
    return 2;
  }
  if ((int64_t)r.U.size() != S * nc) return 2;
  FILE* out = std::fopen(argv[2], "wb");
  if (!out) return 2;
  const double head[2] = {r.dts[DTS_T + (nsteps & 1)], r.dts[DTS_FLAG]};
  ok = std::fwrite(head, 8, 2, out) == 2 && std::fwrite(r.U.data(), 8, r.U.size(), out) == r.U.size();
  return std::fclose(out) == 0 && ok ? 0 : 2;
}

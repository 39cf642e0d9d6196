// 3D stage on column tiles marching in z.
//
// A 3D cell with its two-cell halo in every direction does not fit in LDS at
// the 30-32 primitive words a 3D cell carries, so the stage runs in two
// passes.  The first (prim3_kernel) converts every cell of the stage input to
// primitives once, into a full-grid buffer in HBM.  The second is this one: a
// block owns a TX x TY column of cells and walks up a run of NZC planes.  For
// each plane it
//   1 loads the plane's primitives over the tile and its x and y halo (a
//     cross: the tile's corners are never read) into LDS;
//   2 computes every x-face of the tile once into an LDS face buffer, and
//     each thread adds its own cell's two x-faces to its update accumulator;
//   3 the same for the y-faces;
//   4 computes the z-face above its own cell from the primitives of its own
//     column (four planes, read from HBM through the caches); the face below
//     is the one it computed on the previous plane, kept in registers;
//   5 forms the RK combination and, in stage 3, the source step and the CFL
//     wave-speed sum of its cell.
// Every face is computed once per block (faces on a tile edge or chunk edge
// by the two blocks that share them), so no face data goes through HBM.
// The phases are per-thread functions so that the CPU can step them.
#pragma once

#include "fv_stage.hpp"

namespace fv {

template <int NM, int NS, class T, class C, int TX, int TY, int NTH = TX * TY>
struct Zm {
  using St = Stage<3, NM, NS, T, C, 1, 1>;
  using L = Lay<3, NM, NS>;
  static constexpr int S = L::S;
  static constexpr int NW = L::NW;
  static constexpr int NQ = L::NQ;
  static constexpr int NOWN = TX * TY;
  static_assert(NTH >= NOWN, "a tile needs a thread per column");
  // the cross of a plane: the TX x TY cells, then the x halo (columns -2,
  // -1, TX, TX+1 of every tile row), then the y halo (rows -2, -1, TY, TY+1
  // of every tile column)
  static constexpr int NXH = 4 * TY;
  static constexpr int NYH = 4 * TX;
  static constexpr int NCC = NOWN + NXH + NYH;
  static constexpr int NFX = (TX + 1) * TY;
  static constexpr int NFY = TX * (TY + 1);
  static constexpr int NFACE = NFX > NFY ? (NFX > NOWN ? NFX : NOWN) : (NFY > NOWN ? NFY : NOWN);
  static constexpr int NT = NTH;

  // LDS: W[NW][NCC] then FB[NQ][NFACE] (both of type C)
  static constexpr size_t smem_elems() { return (size_t)NW * NCC + (size_t)NQ * NFACE; }
  static constexpr size_t smem_bytes() { return smem_elems() * sizeof(C); }

  struct Ctx {
    typename St::Ctx s;   // instance, parameters, stage buffers, dt
    int bx, by;           // tile
    int z0, z1;           // planes of this block: [z0, z1)
  };

  // cross index of tile cell (hx, hy), hx in [0, TX + 4), hy in [0, TY + 4),
  // not a corner (both coordinates in the halo)
  FV_HD static int cc(int hx, int hy) {
    const int ix = hx - 2, iy = hy - 2;
    if (ix >= 0 && ix < TX && iy >= 0 && iy < TY) return iy * TX + ix;
    if (iy >= 0 && iy < TY) return NOWN + iy * 4 + (ix < 0 ? ix + 2 : ix - TX + 2);
    return NOWN + NXH + (iy < 0 ? iy + 2 : iy - TY + 2) * TX + ix;
  }
  // tile cell of cross index c
  FV_HD static void cross_pos(int c, int& hx, int& hy) {
    if (c < NOWN) {
      hx = c % TX + 2;
      hy = c / TX + 2;
      return;
    }
    c -= NOWN;
    if (c < NXH) {
      const int k = c % 4;
      hy = c / 4 + 2;
      hx = k < 2 ? k : TX + k;
      return;
    }
    c -= NXH;
    const int k = c / TX;
    hx = c % TX + 2;
    hy = k < 2 ? k : TY + k;
  }

  FV_HD static int64_t cell_index(const Inst& I, int x, int y, int z) {
    return ((int64_t)z * I.n[1] + y) * I.n[0] + x;
  }

  // ---------------------------------------------------------------- phase 1
  // primitives of cross cell c of plane z from the full-grid buffer
  FV_HD static void load_cross(const Ctx& cx, int z, int c, C* W) {
    const Inst& I = *cx.s.I;
    int hx, hy;
    cross_pos(c, hx, hy);
    const int gx = St::map_index(cx.bx * TX + hx - 2, I.n[0], I.bc[0][0], I.bc[0][1]);
    const int gy = St::map_index(cx.by * TY + hy - 2, I.n[1], I.bc[1][0], I.bc[1][1]);
    const int64_t g = cell_index(I, gx, gy, z);
    const C* Wb = (const C*)I.Wb;
#pragma unroll
    for (int v = 0; v < NW; ++v) W[v * NCC + c] = Wb[(int64_t)v * I.ncell + g];
  }

  // ---------------------------------------------------------------- phase 2
  // x-face item (a = 0) or y-face item (a = 1) of plane z -> stencil in the
  // cross, face slot, and boundary slot; false outside the domain
  FV_HD static bool face_item(const Ctx& cx, int a, int z, int item, int& cm, int& c0, int& c1,
                              int& c2, int& gface, int& fslot, int64_t& bslot) {
    const Inst& I = *cx.s.I;
    if (a == 0) {
      const int fx = item % (TX + 1), ty = item / (TX + 1);
      if (ty >= TY) return false;
      gface = cx.bx * TX + fx;
      const int gy = cx.by * TY + ty;
      if (gface > I.n[0] || gy >= I.n[1]) return false;
      const int hy = ty + 2;
      cm = cc(fx, hy); c0 = cc(fx + 1, hy); c1 = cc(fx + 2, hy); c2 = cc(fx + 3, hy);
      fslot = ty * (TX + 1) + fx;
      bslot = (int64_t)z * I.n[1] + gy;
      return true;
    }
    const int tx = item % TX, fy = item / TX;
    if (fy > TY) return false;
    gface = cx.by * TY + fy;
    const int gx = cx.bx * TX + tx;
    if (gface > I.n[1] || gx >= I.n[0]) return false;
    const int hx = tx + 2;
    cm = cc(hx, fy); c0 = cc(hx, fy + 1); c1 = cc(hx, fy + 2); c2 = cc(hx, fy + 3);
    fslot = fy * TX + tx;
    bslot = (int64_t)z * I.n[0] + gx;
    return true;
  }

  FV_HD static int face_items(int a) { return a == 0 ? NFX : NFY; }

  // own column of thread tid; false for a spare thread or outside the domain
  FV_HD static bool own_column(const Ctx& cx, int tid, int& tx, int& ty) {
    const Inst& I = *cx.s.I;
    if (NTH > NOWN && tid >= NOWN) return false;
    tx = tid % TX;
    ty = tid / TX;
    return cx.bx * TX + tx < I.n[0] && cx.by * TY + ty < I.n[1];
  }

  // centre values of the own cell (tx, ty) of the plane in the cross
  FV_HD static void centre(const C* W, int tx, int ty, C* Xc, C* uc, C* phic, C Vc[3][3]) {
    const int c = ty * TX + tx;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Xc[k] = W[(L::W_X + k) * NCC + c];
      uc[k] = W[(L::R_U + k) * NCC + c];
    }
#pragma unroll
    for (int l = 0; l < NM; ++l) phic[l] = W[(L::R_PHI + l) * NCC + c];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Vc[i][j] = 0;
#pragma unroll
    for (int q = 0; q < L::NV; ++q) Vc[vb_i<3>(q)][vb_j<3>(q)] = W[(L::R_V + q) * NCC + c];
  }

  // ---------------------------------------------------------------- phase 3
  // the two faces of direction a (0: x, 1: y) of the own cell into acc
  FV_HD static void gather_xy(const Ctx& cx, const C* W, const C* fb, int a, int tx, int ty,
                              C* acc) {
    C Xc[3], uc[3], phic[NM], Vc[3][3];
    centre(W, tx, ty, Xc, uc, phic, Vc);
    int fm, fp;
    if (a == 0) { fm = ty * (TX + 1) + tx; fp = fm + 1; }
    else { fm = ty * TX + tx; fp = fm + TX; }
    typename St::FaceC m, p;
    St::template face_contrib<int>(fb, fm, NFACE, a, 1, Xc, Vc, uc, m);
    St::template face_contrib<int>(fb, fp, NFACE, a, 0, Xc, Vc, uc, p);
    St::gather_dir(cx.s, a, m, p, Xc, uc, phic, Vc, acc);
  }

  // ---------------------------------------------------------------- phase 4
  // z-face f (between planes f - 1 and f) of the own column from the
  // full-grid primitives, into fb[q * fstride + fslot]
  FV_HD static void zface(const Ctx& cx, int tx, int ty, int f, C* fb, int fslot, int fstride) {
    const Inst& I = *cx.s.I;
    const int gx = cx.bx * TX + tx, gy = cx.by * TY + ty;
    int64_t st[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      st[k] = cell_index(I, gx, gy, St::map_index(f - 2 + k, I.n[2], I.bc[2][0], I.bc[2][1]));
    St::template compute_face<int64_t>(cx.s, (const C*)I.Wb, I.ncell, 2, st[0], st[1], st[2],
                                       st[3], f, fslot, fstride,
                                       (int64_t)gy * I.n[0] + gx, fb);
  }

  // the z-faces below (zm: the previous plane's, a record of NQ values) and
  // above (the face buffer's slot) of the own cell into acc
  FV_HD static void gather_z(const Ctx& cx, const C* W, const C* zm, const C* fb, int fslot,
                             int tx, int ty, C* acc) {
    C Xc[3], uc[3], phic[NM], Vc[3][3];
    centre(W, tx, ty, Xc, uc, phic, Vc);
    typename St::FaceC m, p;
    St::template face_contrib<int>(zm, 0, 1, 2, 1, Xc, Vc, uc, m);
    St::template face_contrib<int>(fb, fslot, NFACE, 2, 0, Xc, Vc, uc, p);
    St::gather_dir(cx.s, 2, m, p, Xc, uc, phic, Vc, acc);
  }
};

}  // namespace fv

// Device kernels of libfv: the stage kernel (1D, 2D), the three 3D passes,
// state conversions, the CFL reduction and the exact sums.  Their launchers
// and the host context are in fv_launch.hpp.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fv_stage.hpp"
#include "../../include/fv.h"

namespace fvk {

using namespace fv;

constexpr int NBINS = 70;  // 32-bit bins covering every finite double

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block maximum of a non-negative value, then an integer atomicMax on its
// bit pattern (order-preserving for non-negative doubles), so the result is
// independent of the order in which blocks finish.
template <int NT>
__device__ void block_max_to(double v, double* scratch, double* target) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  constexpr int NWV = (NT + 63) / 64;
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = scratch[0];
    for (int w = 1; w < NWV; ++w) m = fmax(m, scratch[w]);
    if (m > 0.0)
      atomicMax(reinterpret_cast<unsigned long long*>(target),
                (unsigned long long)__double_as_longlong(m));
  }
}

// Exact sum into 32-bit bins of the integer value * 2^1074.
__device__ __forceinline__ void bin_add(unsigned long long* bins, double v) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  const int ex = (int)((bits >> 52) & 0x7FF);
  if (ex == 0x7FF) return;              // non-finite values are flagged elsewhere
  unsigned long long m = bits & ((1ull << 52) - 1);
  int shift;
  if (ex == 0) {
    shift = 0;                          // subnormal: m * 2^-1074
  } else {
    m |= 1ull << 52;
    shift = ex - 1;                     // m * 2^(ex - 1075) = m * 2^(shift - 1074)
  }
  if (m == 0) return;
  const int k0 = shift >> 5, off = shift & 31;
  const unsigned long long mlo = m & 0xFFFFFFFFull, mhi = m >> 32;
  const unsigned long long t0 = mlo << off, t1 = mhi << off;
  const unsigned long long c0 = t0 & 0xFFFFFFFFull;
  const unsigned long long c1 = (t0 >> 32) + (t1 & 0xFFFFFFFFull);
  const unsigned long long c2 = t1 >> 32;
  const bool neg = (bits >> 63) != 0;
  // two's complement wrap-around makes unsigned adds of negated chunks exact
  atomicAdd(&bins[k0], neg ? (0ull - c0) : c0);
  atomicAdd(&bins[k0 + 1], neg ? (0ull - c1) : c1);
  if (c2) atomicAdd(&bins[k0 + 2], neg ? (0ull - c2) : c2);
}

template <class T>
__global__ void __launch_bounds__(256) exact_sum_kernel(const T* data, int64_t n,
                                                        int64_t stride,
                                                        unsigned long long* out) {
  __shared__ unsigned long long bins[NBINS];
  for (int k = threadIdx.x; k < NBINS; k += blockDim.x) bins[k] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bin_add(bins, (double)data[i * stride]);
  __syncthreads();
  for (int k = threadIdx.x; k < NBINS; k += blockDim.x)
    if (bins[k]) atomicAdd(&out[k], bins[k]);
}

// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2:
// this renumbering gives every XCD one contiguous run of block numbers, so
// neighbouring work (tiles sharing halos, bricks sharing stencil planes)
// meets in one L2.
__device__ __forceinline__ int64_t xcd_block() {
  const int64_t nb = gridDim.x;
  const int64_t xcd = blockIdx.x & 7, qb = nb >> 3, rb = nb & 7;
  return xcd * qb + (xcd < rb ? xcd : rb) + (blockIdx.x >> 3);
}

// ---------------------------------------------------------------------------
// stage kernel
// ---------------------------------------------------------------------------
// Three 256-thread FP32-bulk 2D blocks share a CU (160 KiB of LDS) when the
// tile's LDS fits a third of it (16 x 14: 52 KiB), and then each lane may
// hold at most 168 registers: the bound makes the compiler keep to that
// rather than lose the third block.  Larger tiles keep the default.
template <class St, int DIM, class C, int NTH>
constexpr int stage_waves_per_eu() {
  return (DIM == 2 && sizeof(C) == 4 && NTH == 256 && 3 * St::smem_bytes() <= 160 * 1024) ? 3
                                                                                          : 1;
}

template <int DIM, int NM, int NS, class T, class C, int TX, int TY, int NTH, int EXT>
__global__ void __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(
    stage_waves_per_eu<Stage<DIM, NM, NS, T, C, TX, TY, NTH>, DIM, C, NTH>())))
stage_kernel(const Inst* __restrict__ insts, const int2* __restrict__ block_tab, Params P,
             int stage, int parity) {
  using St = Stage<DIM, NM, NS, T, C, TX, TY, NTH, EXT>;
  using TL = typename St::TL;
  constexpr int NT = NTH;
  extern __shared__ double smem_d[];
  C* sm = reinterpret_cast<C*>(smem_d);
  C* fb = sm + (size_t)St::NW * TL::NCELL;
  const int b = (int)xcd_block();
  // (instance, tile of that instance); a single instance passes no table
  // and its blocks are its tiles in order
  const int2 e = block_tab ? block_tab[b] : make_int2(0, b);
  const int ii = e.x;
  const Inst& I = insts[ii];
  const int lb = e.y;
  const int tid = threadIdx.x;
  // stage 0: a timing run of stage 1 that leaves the time, the dt state and
  // the boundary accumulators alone (its output goes to the stage-1 buffer)
  const bool dry = stage == 0;
  if (dry) stage = 1;
  typename St::Ctx cx;
  cx.I = &I;
  cx.P = P;
  cx.stage = stage;
  cx.dry = dry;
  cx.parity = parity & 1;
  cx.bx = lb % I.tiles[0];
  cx.by = lb / I.tiles[0];
  const T* U = (const T*)I.U;
  cx.base = U;
  cx.src = stage == 1 ? U : (stage == 2 ? (const T*)I.U1 : (const T*)I.U2);
  cx.out = stage == 1 ? (T*)I.U1 : (stage == 2 ? (T*)I.U2 : (T*)I.U);

  // Every global load of the thread goes out at once, ahead of the time-step
  // test so that the two do not wait one after the other: its own cell's
  // stage input (kept for the update), the cell's U^n (stages 2 and 3) and
  // its first halo cell (in bounds whatever the step).  The primitives are
  // formed after they arrive.
  constexpr int S = St::S;
  const bool has_a = NT == TL::NOWN || tid < TL::NOWN;
  const int tcA = has_a ? TL::own(tid) : 0;
  C UA[S], UN[S], UH[S];
  if (has_a) St::load_state(cx, cx.src, St::tile_global(cx, tcA), UA);
  int tx, ty;
  int64_t g = 0;
  const bool own = St::own_cell(cx, tid, tx, ty, g);
  if (stage != 1 && own) St::load_state(cx, cx.base, g, UN);
  const bool has_h = tid < TL::NHALO;
  const int tcH = has_h ? TL::halo_cell(tid) : 0;
  if (has_h) St::load_state(cx, cx.src, St::tile_global(cx, tcH), UH);

  double* dts = I.dts;
  const int q = parity & 1;
  double t, dtinv, dtfix, tend;
  read_dt_state(dts, q, t, dtinv, dtfix, tend);
  double dt = dtfix > 0.0 ? dtfix : P.cfl / dtinv;
  dt = fmin(dt, tend - t);
  // an instance at its end time takes no step
  if (!(dt > 0.0)) {
    if (stage == 1 && !dry && lb == 0 && tid == 0) {
      dts[DTS_T + 1 - q] = t;
      dts_set_dtinv(dts, 1 - q, dtinv);
    }
    return;
  }
  if (stage == 1 && !dry && lb == 0 && tid == 0) {
    dts[DTS_T + 1 - q] = t + dt;
    dts_set_dtinv(dts, 1 - q, 0.0);
  }
  cx.dt = (C)dt;
  cx.tn = t + dt;
  if (has_a) St::template prims_of<int>(cx, UA, sm, TL::NCELL, tcA);
  if (has_h) St::template prims_of<int>(cx, UH, sm, TL::NCELL, tcH);
  for (int h = tid + NT; h < TL::NHALO; h += NT) St::load_cell(cx, sm, TL::halo_cell(h));
  __syncthreads();

  C acc[S];
#pragma unroll
  for (int f = 0; f < S; ++f) acc[f] = 0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const int nit = St::face_items(a);
    for (int it = tid; it < nit; it += NT) {
      int cm, c0, c1, c2, gf, fs, bs;
      if (St::face_item(cx, a, it, cm, c0, c1, c2, gf, fs, bs))
        St::template compute_face<int>(cx, sm, TL::NCELL, a, cm, c0, c1, c2, gf, fs, TL::NFACE, bs, fb);
    }
    __syncthreads();
    if (own) St::gather(cx, sm, fb, a, tx, ty, acc);
    __syncthreads();
  }
  double cflv = 0.0;
  if (own) {
    bool bad = false;
    cflv = St::finish_cell(cx, g, acc, UA, UN, &bad);
    if (bad) atomicOr(reinterpret_cast<unsigned int*>(&dts[DTS_FLAG]), (unsigned)FLAG_NONPHYS);
  }
  // blocks are dispatched round-robin over the XCDs: blockIdx.x & 7 is the
  // block's XCD and picks its CFL slot
  if (stage == 3 && !relax_on(P, NM, NS))
    block_max_to<NT>(cflv, reinterpret_cast<double*>(smem_d),
                     &dts[dts_slot(1 - q, blockIdx.x & (DTS_NSLOT - 1))]);
}

// ---------------------------------------------------------------------------
// primitive <-> conserved, CFL
// ---------------------------------------------------------------------------
template <int DIM, int NM, int NS, class T>
__global__ void __launch_bounds__(256) prim_to_cons_kernel(const Inst* insts, int ii, Params P,
                                                           const double* prim) {
  using L = Lay<DIM, NM, NS>;
  const Inst& I = insts[ii];
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= I.ncell) return;
  double W[L::S], U[L::S];
#pragma unroll
  for (int f = 0; f < L::S; ++f) W[f] = prim[(int64_t)f * I.ncell + g];
  Cell<DIM, NM, NS>::prim_to_cons(P, W, U);
  T* Us = (T*)I.U;
#pragma unroll
  for (int f = 0; f < L::S; ++f) Us[(int64_t)f * I.ncell + g] = (T)U[f];
}

template <int DIM, int NM, int NS, class T>
__global__ void __launch_bounds__(256) cons_to_prim_kernel(const Inst* insts, int ii, Params P,
                                                           double* prim) {
  using L = Lay<DIM, NM, NS>;
  const Inst& I = insts[ii];
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= I.ncell) return;
  const T* Us = (const T*)I.U;
  double U[L::S], W[L::S];
#pragma unroll
  for (int f = 0; f < L::S; ++f) U[f] = (double)Us[(int64_t)f * I.ncell + g];
  Cell<DIM, NM, NS>::cons_to_prim(P, U, W);
#pragma unroll
  for (int f = 0; f < L::S; ++f) prim[(int64_t)f * I.ncell + g] = W[f];
}

// Lagrangian seeding after the step of parity `parity` (Section 3.2.1): the
// coordinates every cell takes (reseeded or kept) go to the X rows of the
// stage-1 buffer, free until the next step, and a second pass copies them
// back, so that every cell is seeded from the coordinates before seeding.
// An instance that did not step (at its end time) is left alone.
__device__ __forceinline__ bool stepped(const Inst& I, int parity) {
  const int q = parity & 1;
  return I.dts[DTS_T + 1 - q] != I.dts[DTS_T + q];
}

template <int DIM, int NM, int NS, class T>
__global__ void __launch_bounds__(256) seed_kernel(const Inst* insts, int ii, Params P,
                                                   int parity) {
  using L = Lay<DIM, NM, NS>;
  using St = Stage<DIM, NM, NS, T, T, 1, 1>;
  const Inst& I = insts[ii];
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= I.ncell || !stepped(I, parity)) return;
  double Xn[DIM];
  St::seed_cell(P, I, (const T*)I.U, g, Xn);
  T* out = (T*)I.U1;
#pragma unroll
  for (int k = 0; k < DIM; ++k) out[(int64_t)(L::XC + k) * I.ncell + g] = (T)Xn[k];
}

// The seeded coordinates back into the state; with one solid, then the void
// relaxation of the cell and the CFL reduction for the next step (which the
// last stage leaves to this pass).
template <int DIM, int NM, int NS, class T>
__global__ void __launch_bounds__(256) seed_copy_kernel(const Inst* insts, int ii, Params P,
                                                        int parity) {
  using L = Lay<DIM, NM, NS>;
  using St = Stage<DIM, NM, NS, T, T, 1, 1>;
  __shared__ double scratch[4];
  const Inst& I = insts[ii];
  if (!stepped(I, parity)) return;     // uniform over the launch
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool relax = relax_on(P, NM, NS);
  double v = 0.0;
  if (g < I.ncell) {
    const T* src = (const T*)I.U1;
    T* U = (T*)I.U;
#pragma unroll
    for (int k = 0; k < DIM; ++k)
      U[(int64_t)(L::XC + k) * I.ncell + g] = src[(int64_t)(L::XC + k) * I.ncell + g];
    if (relax) {
      double Ud[L::S];
#pragma unroll
      for (int f = 0; f < L::S; ++f) Ud[f] = (double)U[(int64_t)f * I.ncell + g];
      St::relax_void_cell(P, Ud);
      U[(int64_t)L::PHI * I.ncell + g] = (T)Ud[L::PHI];
      Ud[L::PHI] = (double)U[(int64_t)L::PHI * I.ncell + g];
      v = St::cfl_sum(P, I, Ud);
      if (!(v == v)) {
        atomicOr(reinterpret_cast<unsigned int*>(&I.dts[DTS_FLAG]), (unsigned)FLAG_NONPHYS);
        v = 0.0;
      }
    }
  }
  if (relax) block_max_to<256>(v, scratch, &I.dts[dts_slot(1 - (parity & 1), blockIdx.x & (DTS_NSLOT - 1))]);
}

template <int DIM, int NM, int NS, class T, class C, int TX, int TY>
__global__ void __launch_bounds__(256) cfl_kernel(const Inst* insts, int ii, Params P, int parity) {
  using St = Stage<DIM, NM, NS, T, C, TX, TY>;
  using L = Lay<DIM, NM, NS>;
  __shared__ double scratch[4];
  const Inst& I = insts[ii];
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (g < I.ncell) {
    const T* Us = (const T*)I.U;
    double U[L::S];
#pragma unroll
    for (int f = 0; f < L::S; ++f) U[f] = (double)Us[(int64_t)f * I.ncell + g];
    v = St::cfl_sum(P, I, U);
    if (!(v == v)) {
      atomicOr(reinterpret_cast<unsigned int*>(&I.dts[DTS_FLAG]), (unsigned)FLAG_NONPHYS);
      v = 0.0;
    }
  }
  block_max_to<256>(v, scratch, &I.dts[dts_slot(parity & 1, blockIdx.x & (DTS_NSLOT - 1))]);
}


// ---------------------------------------------------------------------------
// 3D stage: three passes over full-grid buffers in HBM.  A tile with a
// two-cell halo in three directions does not fit in LDS at the number of
// primitive fields a 3D cell carries, so the primitives go to HBM once, every
// face of a direction is computed once from them, and a per-cell pass
// gathers the six faces, applies the RK combination and (third stage) the
// source step and CFL reduction.
// ---------------------------------------------------------------------------
// time step of the stage from the device dt state; fills the context.
// stage 0 is the timing run of stage 1 (see stage_kernel).
template <class St, class T, class C>
__device__ __forceinline__ bool setup3(const Inst& I, const Params& P, int stage, int parity,
                                       typename St::Ctx& cx, double& t, double& dtinv,
                                       double& dt) {
  const int q = parity & 1;
  double dtfix, tend;
  read_dt_state(I.dts, q, t, dtinv, dtfix, tend);
  dt = dtfix > 0.0 ? dtfix : P.cfl / dtinv;
  dt = fmin(dt, tend - t);
  const bool dry = stage == 0;
  if (dry) stage = 1;
  cx.I = &I;
  cx.P = P;
  cx.stage = stage;
  cx.dry = dry;
  cx.parity = q;
  cx.bx = 0;
  cx.by = 0;
  cx.dt = (C)dt;
  cx.tn = t + dt;
  const T* U = (const T*)I.U;
  cx.base = U;
  cx.src = stage == 1 ? U : (stage == 2 ? (const T*)I.U1 : (const T*)I.U2);
  cx.out = stage == 1 ? (T*)I.U1 : (stage == 2 ? (T*)I.U2 : (T*)I.U);
  return dt > 0.0;
}

__device__ __forceinline__ int64_t nfaces3(const Inst& I, int a) {
  return I.ncell / I.n[a] * (I.n[a] + 1);
}

template <int NM, int NS, class T, class C>
__global__ void __launch_bounds__(256) prim3_kernel(const Inst* insts, int ii, Params P,
                                                    int stage, int parity) {
  using St = Stage<3, NM, NS, T, C, 1, 1>;
  const Inst& I = insts[ii];
  typename St::Ctx cx;
  double t, dtinv, dt;
  if (!setup3<St, T, C>(I, P, stage, parity, cx, t, dtinv, dt)) return;
  const int64_t g = xcd_block() * blockDim.x + threadIdx.x;
  if (g >= I.ncell) return;
  St::template cell_prims<int64_t, true>(cx, g, (C*)I.Wb, I.ncell, g);
}

// x-faces in runs of XRUN + 1 faces overlapping by one (a block per run):
// each thread computes one face into LDS, then the cell between its face and
// the next one starts its divergence sum
// (one material in FP32: bounded to five waves per SIMD, which costs the
// compiler one register and no spill)
template <int NM, int NS, class T, class C>
__global__ void __launch_bounds__(256, (sizeof(C) == 4 && NM == 1) ? 5 : 1)
    xface3_kernel(const Inst* insts, int ii, Params P, int stage, int parity) {
  using St = Stage<3, NM, NS, T, C, 1, 1>;
  using L = Lay<3, NM, NS>;
  static_assert(St::XRUN + 1 == 256, "one face per thread");
  __shared__ C fb[L::NQ * (St::XRUN + 1)];
  const Inst& I = insts[ii];
  typename St::Ctx cx;
  double t, dtinv, dt;
  if (!setup3<St, T, C>(I, P, stage, parity, cx, t, dtinv, dt)) return;
  const int64_t b = xcd_block();
  St::xrun_face(cx, (const C*)I.Wb, b, (int)threadIdx.x, fb);
  __syncthreads();
  St::xrun_cell(cx, (const C*)I.Wb, b, (int)threadIdx.x, fb, (C*)I.Acc);
}

// y- and z-faces: a thread walks a run of MARCH cells along A (the direction
// is a template argument: every per-direction index in the face computation
// is then a constant; a runtime direction would put those arrays in scratch
// memory)
template <int NM, int NS, class T, class C, int A>
__global__ void __launch_bounds__(256) march3_kernel(const Inst* insts, int ii, Params P,
                                                     int stage, int parity) {
  using St = Stage<3, NM, NS, T, C, 1, 1>;
  const Inst& I = insts[ii];
  typename St::Ctx cx;
  double t, dtinv, dt;
  if (!setup3<St, T, C>(I, P, stage, parity, cx, t, dtinv, dt)) return;
  int x, u, s;
  if (!brick_pos(xcd_block(), (int)threadIdx.x, I.n[0], A == 1 ? I.n[2] : I.n[1],
                 St::march_runs(I, A), x, u, s))
    return;
  St::march_cells(cx, (const C*)I.Wb, A, x, u, s, (C*)I.Acc);
}

template <int NM, int NS, class T, class C>
__global__ void __launch_bounds__(256) finish3_kernel(const Inst* insts, int ii, Params P,
                                                      int stage, int parity) {
  using St = Stage<3, NM, NS, T, C, 1, 1>;
  __shared__ double scratch[4];
  const Inst& I = insts[ii];
  typename St::Ctx cx;
  double t, dtinv, dt;
  const bool dry = stage == 0;
  const bool go = setup3<St, T, C>(I, P, stage, parity, cx, t, dtinv, dt);
  const int q = parity & 1;
  // time of the next step and a cleared CFL slot for the third stage's
  // reduction (a finished instance carries its time and CFL value over)
  if (cx.stage == 1 && !dry && blockIdx.x == 0 && threadIdx.x == 0) {
    I.dts[DTS_T + 1 - q] = go ? t + dt : t;
    dts_set_dtinv(I.dts, 1 - q, go ? 0.0 : dtinv);
  }
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double cflv = 0.0;
  if (go && g < I.ncell) {
    const C* accb = (const C*)I.Acc;
    const int64_t nc = I.ncell;
    C acc[St::S];
#pragma unroll
    for (int f = 0; f < St::S; ++f) acc[f] = accb[f * nc + g];
    bool bad = false;
    cflv = St::finish_cell(cx, g, acc, &bad);
    if (bad) atomicOr(reinterpret_cast<unsigned int*>(&I.dts[DTS_FLAG]), (unsigned)FLAG_NONPHYS);
  }
  if (cx.stage == 3 && go && !relax_on(P, NM, NS))
    block_max_to<256>(cflv, scratch, &I.dts[dts_slot(1 - q, blockIdx.x & (DTS_NSLOT - 1))]);
}

}  // namespace fvk

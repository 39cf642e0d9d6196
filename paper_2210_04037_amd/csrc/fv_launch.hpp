// Host side of libfv shared by the translation units: the context behind
// the C ABI's opaque handle, the per-tile-shape launchers of the kernels in
// fv_kernels.hpp and the kernel-set tables of each precision.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "fv_kernels.hpp"

namespace fvk {

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct Ops {
  int S = 0, NC = 0, NTOT = 0, TX = 0, TY = 0, NT = 0, NW = 0, NQ = 0;
  size_t smem = 0;
  void (*stage)(fv_ctx*, int, int, hipStream_t) = nullptr;
  void (*p2c)(fv_ctx*, int, const double*) = nullptr;
  void (*c2p)(fv_ctx*, int, double*) = nullptr;
  void (*cfl)(fv_ctx*, int, int) = nullptr;
  void (*seed)(fv_ctx*, int, hipStream_t) = nullptr;
  size_t elem = 8;
};

}  // namespace fvk

// Context behind the opaque fv_ctx handle of the C ABI.
struct fv_ctx {
  int n_inst = 0, dim = 0, nm = 0, ns = 0, precision = 0;
  int device = 0;                     // HIP device current at fv_init
  fv::Params P{};
  hipStream_t stream = nullptr;
  std::vector<fv::Inst> insts;
  fv::Inst* insts_d = nullptr;
  int2* block_tab_d = nullptr;       // (instance, tile) of every stage block
  unsigned long long* bins_d = nullptr;
  int total_blocks = 0;
  long long step = 0;
  fvk::Ops ops;                       // the selected tile shape
  std::vector<fvk::Ops> vars;         // every compiled tile shape
  int var = 0;
  int max_blocks = 0;                 // capacity of the block table
  std::vector<int2> h_block_tab;
  int sched = 0;                      // block order (FV_SCHED_*)
  // captured multi-step graphs, keyed by (step count, starting parity)
  static constexpr int NGRAPH = 4;
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec[NGRAPH] = {};
  int gkey[NGRAPH] = {};              // 2 * n_steps + parity, 0 = empty
  int gnext = 0;                      // slot replaced next
  std::vector<double> h_dt, h_tend;   // staging for async copies
  bool dtfix_set = false;             // a fixed dt may be set on the device
  std::vector<char> loaded;           // state written (load_primitive / reset)
  std::vector<double> h_ck;           // checkpoint header staging
  std::string err;
};

namespace fvk {

// launchers shared by every tile shape: state conversions and the CFL
// reduction of a state without a source step
template <int DIM, int NM, int NS, class T, class C>
void common_ops(Ops& o) {
  using L = Lay<DIM, NM, NS>;
  o.S = L::S;
  o.NC = L::NC;
  o.NW = L::NW;
  o.NQ = L::NQ;
  o.NTOT = NM + DIM + 1;
  o.elem = sizeof(T);
  o.p2c = [](fv_ctx* c, int ii, const double* prim) {
    const int64_t n = c->insts[ii].ncell;
    hipLaunchKernelGGL((prim_to_cons_kernel<DIM, NM, NS, T>), dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, c->stream, c->insts_d, ii, c->P, prim);
  };
  o.c2p = [](fv_ctx* c, int ii, double* prim) {
    const int64_t n = c->insts[ii].ncell;
    hipLaunchKernelGGL((cons_to_prim_kernel<DIM, NM, NS, T>), dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, c->stream, c->insts_d, ii, c->P, prim);
  };
  o.seed = [](fv_ctx* c, int parity, hipStream_t s) {
    for (int ii = 0; ii < c->n_inst; ++ii) {
      const int64_t n = c->insts[ii].ncell;
      const dim3 grid((unsigned)((n + 255) / 256)), blk(256);
      hipLaunchKernelGGL((seed_kernel<DIM, NM, NS, T>), grid, blk, 0, s, c->insts_d, ii, c->P,
                         parity);
      hipLaunchKernelGGL((seed_copy_kernel<DIM, NM, NS, T>), grid, blk, 0, s, c->insts_d, ii,
                         c->P, parity);
    }
  };
  o.cfl = [](fv_ctx* c, int ii, int parity) {
    const int64_t n = c->insts[ii].ncell;
    hipLaunchKernelGGL((cfl_kernel<DIM, NM, NS, T, C, 1, 1>), dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, c->stream, c->insts_d, ii, c->P, parity);
  };
}

template <int DIM, int NM, int NS, class T, class C, int TX, int TY, int NTH, int EXT>
Ops make_ops() {
  using St = Stage<DIM, NM, NS, T, C, TX, TY, NTH, EXT>;
  Ops o;
  common_ops<DIM, NM, NS, T, C>(o);
  o.TX = TX;
  o.TY = TY;
  o.NT = NTH;
  o.smem = St::smem_bytes();
  o.stage = [](fv_ctx* c, int stage, int parity, hipStream_t s) {
    hipLaunchKernelGGL((stage_kernel<DIM, NM, NS, T, C, TX, TY, NTH, EXT>), dim3(c->total_blocks),
                       dim3(NTH), St::smem_bytes(), s, c->insts_d,
                       c->n_inst == 1 ? (const int2*)nullptr : c->block_tab_d, c->P, stage,
                       parity);
  };
  return o;
}

// 3D kernel set: the three passes per stage, launched instance by instance
// (block size 256; TX reports it, TY = 1)
template <int NM, int NS, class T, class C>
Ops make_ops3() {
  Ops o;
  common_ops<3, NM, NS, T, C>(o);
  o.TX = 256;
  o.TY = 1;
  o.NT = 256;
  o.smem = 0;
  o.stage = [](fv_ctx* c, int stage, int parity, hipStream_t s) {
    for (int ii = 0; ii < c->n_inst; ++ii) {
      const Inst& I = c->insts[ii];
      const unsigned nbc = (unsigned)((I.ncell + 255) / 256);
      hipLaunchKernelGGL((prim3_kernel<NM, NS, T, C>), dim3(nbc), dim3(256), 0, s, c->insts_d, ii,
                         c->P, stage, parity);
      using St = Stage<3, NM, NS, T, C, 1, 1>;
      const int nx = I.n[0], ny = I.n[1], nz = I.n[2];
      hipLaunchKernelGGL((xface3_kernel<NM, NS, T, C>), dim3((unsigned)St::xrun_count(I)),
                         dim3(256), 0, s, c->insts_d, ii, c->P, stage, parity);
      hipLaunchKernelGGL((march3_kernel<NM, NS, T, C, 1>),
                         dim3((unsigned)brick_blocks(nx, nz, St::march_runs(I, 1))), dim3(256),
                         0, s, c->insts_d, ii, c->P, stage, parity);
      hipLaunchKernelGGL((march3_kernel<NM, NS, T, C, 2>),
                         dim3((unsigned)brick_blocks(nx, ny, St::march_runs(I, 2))), dim3(256),
                         0, s, c->insts_d, ii, c->P, stage, parity);
      hipLaunchKernelGGL((finish3_kernel<NM, NS, T, C>), dim3(nbc), dim3(256), 0, s, c->insts_d,
                         ii, c->P, stage, parity);
    }
  };
  return o;
}

template <int DIM, int NM, int NS, class T, class C, int TX, int TY, int NTH, int EXT>
hipError_t set_smem_attr() {
  using St = Stage<DIM, NM, NS, T, C, TX, TY, NTH, EXT>;
  return hipFuncSetAttribute((const void*)&stage_kernel<DIM, NM, NS, T, C, TX, TY, NTH, EXT>,
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)St::smem_bytes());
}

// one compiled tile shape of a kernel set (the first one listed is the
// default), in the build with the extended closures (ext) or the one
// without; set_attr also raises the kernel's dynamic LDS limit, a runtime
// call that size-only queries skip
#define FV_VARN(D, M, S_, TT, CC, X, Y, N)                                          \
  {                                                                                 \
    if (ext) {                                                                      \
      vars.push_back(make_ops<D, M, S_, TT, CC, X, Y, N, 1>());                     \
      if (set_attr && herr == hipSuccess) herr = set_smem_attr<D, M, S_, TT, CC, X, Y, N, 1>(); \
    } else {                                                                        \
      vars.push_back(make_ops<D, M, S_, TT, CC, X, Y, N, 0>());                     \
      if (set_attr && herr == hipSuccess) herr = set_smem_attr<D, M, S_, TT, CC, X, Y, N, 0>(); \
    }                                                                               \
  }
// a tile shape with one thread per interior cell
#define FV_VAR(D, M, S_, TT, CC, X, Y) FV_VARN(D, M, S_, TT, CC, X, Y, (X) * (Y))

#define FV_VAR3(M, S_, TT, CC)                                              \
  { vars.push_back(make_ops3<M, S_, TT, CC>()); }

// kernel sets of each translation unit: every tile shape compiled for a
// (dimension, materials, solids) combination
// (ext: the run uses an extended closure, THINC or the driver; 1D and 2D
// only, the 3D passes are built with them)
bool select_ops_fp64(int dim, int nm, int ns, bool ext, std::vector<Ops>& vars,
                     hipError_t& herr, bool set_attr);
bool select_ops_fp32(int dim, int nm, int ns, bool ext, std::vector<Ops>& vars,
                     hipError_t& herr, bool set_attr);

}  // namespace fvk

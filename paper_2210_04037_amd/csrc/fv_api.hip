// libfv host API: the C ABI declared in include/fv.h (argument checks,
// workspace plan, context set-up, stepping and step graphs, autotuner,
// totals, fragments, checkpoints).  The kernel sets of the two precision
// forms are compiled in fv_fp64.hip and fv_fp32.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fv_launch.hpp"
#include "fv_ccl.hpp"

using namespace fv;
using namespace fvk;


namespace {
// Correctly rounded (ties to even) value of sum_k bins[k] 2^(32k) 2^-1074.
double bins_to_double(const unsigned long long* ub) {
  long long bins[NBINS];
  for (int k = 0; k < NBINS; ++k) bins[k] = (long long)ub[k];
  uint32_t limb[NBINS + 2];
  long long carry = 0;
  for (int k = 0; k < NBINS; ++k) {
    // exact: |bins[k]| < 2^62 and |carry| < 2^31
    const __int128 v = (__int128)bins[k] + carry;
    limb[k] = (uint32_t)(v & 0xFFFFFFFF);
    carry = (long long)(v >> 32);
  }
  limb[NBINS] = (uint32_t)(carry & 0xFFFFFFFF);
  limb[NBINS + 1] = (uint32_t)((carry >> 32) & 0xFFFFFFFF);
  const int NL = NBINS + 2;
  bool neg = (limb[NL - 1] >> 31) != 0;
  if (neg) {  // magnitude of the two's complement number
    unsigned long long c = 1;
    for (int k = 0; k < NL; ++k) {
      const unsigned long long v = (unsigned long long)(uint32_t)~limb[k] + c;
      limb[k] = (uint32_t)v;
      c = v >> 32;
    }
  }
  int top = -1;
  for (int k = NL - 1; k >= 0 && top < 0; --k)
    if (limb[k]) top = k * 32 + (31 - __builtin_clz(limb[k]));
  if (top < 0) return 0.0;
  auto bit = [&](int i) -> int { return i < 0 ? 0 : (limb[i >> 5] >> (i & 31)) & 1; };
  // 53 significant bits [top-52, top]
  const int lo = top - 52;
  unsigned long long mant = 0;
  for (int i = top; i >= std::max(lo, 0); --i) mant = (mant << 1) | bit(i);
  int e2 = 0;  // value = mant * 2^(e2 - 1074)
  if (lo > 0) {
    e2 = lo;
    const int rb = bit(lo - 1);
    bool sticky = false;
    for (int i = lo - 2; i >= 0 && !sticky; --i) sticky = bit(i) != 0;
    if (rb && (sticky || (mant & 1))) {
      mant += 1;
      if (mant >> 53) { mant >>= 1; e2 += 1; }
    }
  } else {
    mant = 0;
    for (int i = top; i >= 0; --i) mant = (mant << 1) | bit(i);
  }
  const double r = std::ldexp((double)mant, e2 - 1074);
  return neg ? -r : r;
}

}  // namespace

static std::string g_init_error;

static int fail(fv_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg; else g_init_error = msg;
  return code;
}

static int hip_check(fv_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return FV_OK;
  return fail(c, FV_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}


// Every compiled tile shape of the kernel set for this combination, the
// default first.  set_attr: also raise each kernel's dynamic LDS limit (a HIP
// runtime call; size-only queries skip it so that they run without a device)
static bool select_ops(int dim, int nm, int ns, bool ext, int prec, std::vector<Ops>& vars,
                       hipError_t& herr, bool set_attr = true) {
  if (prec == FV_FP32_BULK) return select_ops_fp32(dim, nm, ns, ext, vars, herr, set_attr);
  return select_ops_fp64(dim, nm, ns, ext, vars, herr, set_attr);
}

// Does the run need the kernels with the extended closures (a Johnson-Cook,
// Steinberg, Burakovsky-Preston or simplified-damage row, THINC or the
// driver)?  Runs without them take the build whose branches are compiled
// out (the same results).
static bool needs_ext(int n_mat, const fv_material* mats, const fv_options* opt) {
  bool e = opt->thinc_beta > 0.0 || opt->driver[5] > 0.0;
  for (int l = 0; l < n_mat; ++l) {
    const fv_material& m = mats[l];
    if (m.kind != FV_MAT_SOLID) continue;
    e = e || m.jc_B != 0.0 || m.jc_C != 0.0 || m.T_melt > 0.0 || m.G_p > 0.0 ||
        m.Gamma1 != 0.0 || m.Gamma2 != 0.0 || m.Ddot0 > 0.0;
  }
  return e;
}

// index of the tile shape asked for in the options (0, 0: the default)
static int pick_variant(const std::vector<Ops>& vars, const fv_options* opt) {
  if (opt->tile[0] == 0 && opt->tile[1] == 0) return 0;
  for (size_t v = 0; v < vars.size(); ++v)
    if (vars[v].TX == opt->tile[0] && vars[v].TY == opt->tile[1]) return (int)v;
  return -1;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int validate(int32_t n_inst, const fv_grid* grids, int32_t n_mat,
                    const fv_material* mats, const fv_options* opt, int& ns,
                    std::string& msg) {
  if (n_inst < 1 || !grids || !mats || !opt) { msg = "null argument or n_inst < 1"; return FV_EINVAL; }
  if (n_mat < 1 || n_mat > 2) { msg = "n_mat must be 1 or 2"; return FV_EINVAL; }
  ns = 0;
  for (int l = 0; l < n_mat; ++l) {
    if (mats[l].kind != FV_MAT_SOLID && mats[l].kind != FV_MAT_GAS) { msg = "bad material kind"; return FV_EINVAL; }
    if (mats[l].kind == FV_MAT_SOLID) {
      if (l != ns) { msg = "solids must precede gases"; return FV_EINVAL; }
      ++ns;
      const fv_material& m = mats[l];
      if (!(m.rho0 > 0 && m.K0 > 0 && m.alpha > 0 && m.G0 >= 0 && m.Gamma0 > 0 &&
            m.D_crit > m.D0 && m.D_crit < 1 && m.eps_c > m.eps_th && m.eps_th > 0 &&
            m.bonora_alpha > 0 && m.n_hard > 0 && m.yield >= 0 && m.jc_B >= 0 &&
            m.jc_C >= 0 && m.T_melt >= 0 &&
            (m.T_melt == 0 || (m.T_melt > 300.0 && m.jc_m > 0 && m.C_V > 0)) &&
            m.G_p >= 0 && m.Ddot0 >= 0 &&
            ((m.Gamma1 == 0 && m.Gamma2 == 0) || m.gamma_bp > 0))) {
        msg = "invalid solid constants"; return FV_EINVAL;
      }
    } else if (!(mats[l].Gamma0 > 0)) { msg = "gas needs Gamma0 > 0"; return FV_EINVAL; }
  }
  if (ns == 2 && grids[0].dim != 1) { msg = "two solids are compiled for 1D only"; return FV_EINVAL; }
  if (opt->precision != FV_FP64 && opt->precision != FV_FP32_BULK) { msg = "bad precision"; return FV_EINVAL; }
  if (!(opt->cfl > 0 && opt->cfl <= 1)) { msg = "cfl must be in (0, 1]"; return FV_EINVAL; }
  if (!(opt->phi_floor > 0 && opt->phi_floor < 0.5)) { msg = "phi_floor must be in (0, 0.5)"; return FV_EINVAL; }
  if (!(opt->weno_eps > 0)) { msg = "weno_eps must be > 0"; return FV_EINVAL; }
  if (!(opt->seed_nu >= 0 && opt->seed_nu < 1)) { msg = "seed_nu must be in [0, 1)"; return FV_EINVAL; }
  if (!(opt->thinc_beta >= 0 && opt->thinc_beta <= 10)) { msg = "thinc_beta must be in [0, 10]"; return FV_EINVAL; }
  {
    const double* d = opt->driver;
    if (d[5] != 0.0 && !(grids[0].dim >= 2 && d[0] >= 0 && d[5] > d[0] && d[3] > 0 &&
                         d[4] > d[3] && d[1] == d[1] && d[2] == d[2])) {
      msg = "driver needs dim >= 2, 0 <= r_in < r_max, 0 < t0 < t1";
      return FV_EINVAL;
    }
  }
  if (opt->tile[2] < FV_SCHED_BY_INSTANCE || opt->tile[2] > FV_SCHED_INTERLEAVED) {
    msg = "tile[2] must be a block schedule (0, 1 or 2)"; return FV_EINVAL;
  }
  const int dim = grids[0].dim;
  for (int i = 0; i < n_inst; ++i) {
    const fv_grid& g = grids[i];
    if (g.dim != dim) { msg = "all instances must share the dimension"; return FV_EINVAL; }
    if (g.dim < 1 || g.dim > 3) { msg = "dim must be 1, 2 or 3"; return FV_EINVAL; }
    for (int k = 0; k < 3; ++k) {
      if (g.n[k] < 1 || (k >= g.dim && g.n[k] != 1)) { msg = "bad cell counts"; return FV_EINVAL; }
      if (!(g.hi[k] > g.lo[k])) { msg = "hi must exceed lo"; return FV_EINVAL; }
      if (k < g.dim) {
        for (int s = 0; s < 2; ++s)
          if (g.bc[k][s] < FV_BC_TRANSMISSIVE || g.bc[k][s] > FV_BC_PERIODIC) { msg = "bad boundary kind"; return FV_EINVAL; }
        if ((g.bc[k][0] == FV_BC_PERIODIC) != (g.bc[k][1] == FV_BC_PERIODIC)) { msg = "periodic sides must be paired"; return FV_EINVAL; }
        // a one-cell periodic direction would be its own neighbour
        if (g.bc[k][0] == FV_BC_PERIODIC && g.n[k] < 2) { msg = "a periodic direction needs at least 2 cells"; return FV_EINVAL; }
      }
    }
    const int64_t nc = (int64_t)g.n[0] * g.n[1] * g.n[2];
    if (nc > ((int64_t)1 << 31)) { msg = "too many cells"; return FV_EINVAL; }
    // 1D and 2D stage kernels address a cell within a field by a 32-bit byte offset
    const int64_t elem = opt->precision == FV_FP64 ? 8 : 4;
    if (g.dim <= 2 && nc * elem > ((int64_t)1 << 32)) {
      msg = "1D/2D instance too large: one state field must fit in 4 GiB"; return FV_EINVAL;
    }
  }
  return FV_OK;
}

struct WsPlan {
  std::vector<size_t> u1, u2, bacc, dts, wb, acc;
  size_t insts = 0, block_tab = 0, bins = 0, total = 0;
  int max_blocks = 0;
};

static int tiles_of(const fv_grid& g, const Ops& o, int& tx, int& ty) {
  tx = (g.n[0] + o.TX - 1) / o.TX;
  ty = g.dim >= 2 ? (g.n[1] + o.TY - 1) / o.TY : 1;
  return tx * ty;
}

// Workspace layout; the block table holds the block count of the tile shape
// with the most blocks, so that any compiled shape can be selected later.
static void plan_ws(int32_t n_inst, const fv_grid* grids, const std::vector<Ops>& vars,
                    WsPlan& W) {
  const Ops& o = vars[0];
  size_t off = 0;
  for (const Ops& v : vars) {
    int nb = 0, tx, ty;
    for (int i = 0; i < n_inst; ++i) nb += tiles_of(grids[i], v, tx, ty);
    W.max_blocks = std::max(W.max_blocks, nb);
  }
  for (int i = 0; i < n_inst; ++i) {
    const fv_grid& g = grids[i];
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const size_t sb = align256((size_t)o.S * ncell * o.elem);
    W.u1.push_back(off); off += sb;
    W.u2.push_back(off); off += sb;
    size_t nb = 0;
    for (int a = 0; a < 3; ++a) {
      const int nt = a < g.dim ? (int)(((int64_t)g.n[0] * g.n[1] * g.n[2]) / g.n[a]) : 0;
      nb += 2 * (size_t)nt * o.NC;
    }
    W.bacc.push_back(off); off += align256(nb * sizeof(double));
    W.dts.push_back(off); off += align256(DTS_SIZE * sizeof(double));
    // 3D passes: primitives of every cell and each cell's divergence sum
    W.wb.push_back(off);
    if (g.dim == 3) off += align256((size_t)o.NW * ncell * o.elem);
    W.acc.push_back(off);
    if (g.dim == 3) off += sb;
  }
  W.insts = off; off += align256(sizeof(Inst) * n_inst);
  W.block_tab = off; off += align256(sizeof(int2) * W.max_blocks);
  // totals bins: per instance and total, the interior sum and one per
  // boundary side (2 per direction)
  W.bins = off;
  off += align256(sizeof(unsigned long long) * NBINS * (size_t)n_inst * o.NTOT *
                  (1 + 2 * (size_t)grids[0].dim));
  W.total = off;
}

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

// Select tile shape v: per-instance tile counts, the block -> instance table,
// and their device copies (synchronises the stream).  Captured step graphs
// hold the old launch shape and are dropped.
static void drop_graphs(fv_ctx* c) {
  for (int k = 0; k < fv_ctx::NGRAPH; ++k) {
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    c->gexec[k] = nullptr;
    c->gkey[k] = 0;
  }
  c->gnext = 0;
}

// Tile shape v and block schedule sched: the block table lists (instance,
// tile) for every block of a stage launch, in the order the schedule gives
// (blocks start roughly in table order, so it decides which instances share
// the device at a time and which tiles meet in an XCD's L2).
static int set_tiles(fv_ctx* c, int v, int sched) {
  const Ops& o = c->vars[v];
  int total = 0;
  for (int i = 0; i < c->n_inst; ++i) {
    Inst& I = c->insts[i];
    fv_grid g{};
    g.dim = c->dim;
    for (int k = 0; k < 3; ++k) g.n[k] = I.n[k];
    int tx, ty;
    tiles_of(g, o, tx, ty);
    I.tiles[0] = tx; I.tiles[1] = ty; I.tiles[2] = 1;
    I.nblocks = tx * ty;
    total += I.nblocks;
  }
  if (total > c->max_blocks) return fail(c, FV_EINVAL, "block table overflow");
  std::vector<int> order(c->n_inst);
  for (int i = 0; i < c->n_inst; ++i) order[i] = i;
  if (sched == FV_SCHED_LARGEST_FIRST)
    std::stable_sort(order.begin(), order.end(), [c](int a, int b) {
      return c->insts[a].nblocks > c->insts[b].nblocks;
    });
  c->h_block_tab.clear();
  if (sched == FV_SCHED_INTERLEAVED) {
    int most = 0;
    for (int i = 0; i < c->n_inst; ++i) most = std::max(most, c->insts[i].nblocks);
    for (int t = 0; t < most; ++t)
      for (int i = 0; i < c->n_inst; ++i)
        if (t < c->insts[i].nblocks) c->h_block_tab.push_back(make_int2(i, t));
  } else {
    for (int i : order)
      for (int t = 0; t < c->insts[i].nblocks; ++t) c->h_block_tab.push_back(make_int2(i, t));
  }
  drop_graphs(c);
  c->var = v;
  c->sched = sched;
  c->ops = o;
  c->total_blocks = total;
  int rc = hip_check(c, hipMemcpyAsync(c->insts_d, c->insts.data(), sizeof(Inst) * c->n_inst,
                                       hipMemcpyHostToDevice, c->stream), "copy instance table");
  if (rc == FV_OK)
    rc = hip_check(c, hipMemcpyAsync(c->block_tab_d, c->h_block_tab.data(), sizeof(int2) * total,
                                     hipMemcpyHostToDevice, c->stream), "copy block table");
  if (rc == FV_OK) rc = hip_check(c, hipStreamSynchronize(c->stream), "tile table sync");
  return rc;
}

// Static fragment scratch of fv_fragments_noalloc: one array per GPU, held
// from the library's load to the end of the process.  Host code never uses
// its name as an address (that is a host-side stand-in): fv_init looks up
// each device's address once with hipGetSymbolAddress, with that device
// current, and the entry point passes that address to the kernels.
static __device__ __align__(256) unsigned char frag_scratch[FV_FRAGMENT_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;   // per device id

// Address of the scratch array on the current device (looked up once).
int scratch_setup(fv_ctx* c) {
  int dev = 0;
  int rc = hip_check(c, hipGetDevice(&dev), "current device");
  if (rc != FV_OK) return rc;
  c->device = dev;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_addr.size() <= dev) g_scratch_addr.resize(dev + 1, nullptr);
  if (g_scratch_addr[dev]) return FV_OK;
  void* p = nullptr;
  rc = hip_check(c, hipGetSymbolAddress(&p, HIP_SYMBOL(frag_scratch)), "fragment scratch address");
  if (rc != FV_OK) return rc;
  g_scratch_addr[dev] = p;
  return FV_OK;
}

void* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return dev >= 0 && dev < (int)g_scratch_addr.size() ? g_scratch_addr[dev] : nullptr;
}
}  // namespace

__global__ void __launch_bounds__(256) zero_words_kernel(unsigned int* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

extern "C" {

int32_t fv_state_fields(int32_t dim, int32_t n_mat, const fv_material* mats) {
  if (dim < 1 || dim > 3 || n_mat < 1 || n_mat > 2 || !mats) return 0;
  int ns = 0;
  for (int l = 0; l < n_mat; ++l) ns += mats[l].kind == FV_MAT_SOLID;
  const int nv = dim == 1 ? 3 : (dim == 2 ? 5 : 9);
  return 2 * n_mat + 2 * ns + dim + 1 + nv + dim;
}

size_t fv_workspace_bytes(int32_t n_inst, const fv_grid* grids, int32_t n_mat,
                          const fv_material* mats, const fv_options* opt) {
  int ns = 0;
  std::string msg;
  if (validate(n_inst, grids, n_mat, mats, opt, ns, msg) != FV_OK) return 0;
  std::vector<Ops> vars;
  hipError_t he;
  if (!select_ops(grids[0].dim, n_mat, ns, needs_ext(n_mat, mats, opt), opt->precision, vars,
                  he, false))
    return 0;
  if (pick_variant(vars, opt) < 0) return 0;
  WsPlan W;
  plan_ws(n_inst, grids, vars, W);
  return W.total;
}

static int reset_inst(fv_ctx* c, int i, bool cfl);

int32_t fv_init(fv_ctx** out, int32_t n_inst, const fv_grid* grids, int32_t n_mat,
                const fv_material* mats, const fv_options* opt, void* const* state,
                const void* const* phi0, void* workspace, size_t workspace_bytes,
                void* stream) {
  if (!out) return fail(nullptr, FV_EINVAL, "out is NULL");
  *out = nullptr;
  int ns = 0;
  std::string msg;
  int rc = validate(n_inst, grids, n_mat, mats, opt, ns, msg);
  if (rc != FV_OK) return fail(nullptr, rc, msg);
  if (!state || !phi0 || !workspace) return fail(nullptr, FV_EINVAL, "null device pointer");
  for (int i = 0; i < n_inst; ++i)
    if (!state[i] || !phi0[i]) return fail(nullptr, FV_EINVAL, "null state or phi0 pointer");
  fv_ctx* c = new fv_ctx();
  c->n_inst = n_inst;
  c->dim = grids[0].dim;
  c->nm = n_mat;
  c->ns = ns;
  c->precision = opt->precision;
  c->stream = (hipStream_t)stream;
  hipError_t he;
  if (!select_ops(c->dim, n_mat, ns, needs_ext(n_mat, mats, opt), opt->precision, c->vars,
                  he)) {
    delete c;
    return fail(nullptr, FV_EINVAL, "unsupported dimension/material/precision combination");
  }
  c->var = pick_variant(c->vars, opt);
  if (c->var < 0) {
    delete c;
    return fail(nullptr, FV_EINVAL, "tile shape " + std::to_string(opt->tile[0]) + "x" +
                                         std::to_string(opt->tile[1]) + " is not compiled");
  }
  c->ops = c->vars[c->var];
  c->use_graph = opt->use_graph != 0;
  if (he != hipSuccess) {
    std::string m = std::string("hipFuncSetAttribute: ") + hipGetErrorString(he);
    delete c;
    return fail(nullptr, FV_EDEVICE, m);
  }
  fill_params(mats, n_mat, opt, c->P);
  rc = scratch_setup(c);
  if (rc != FV_OK) {
    g_init_error = c->err;
    delete c;
    return rc;
  }
  WsPlan W;
  plan_ws(n_inst, grids, c->vars, W);
  if (workspace_bytes < W.total) {
    delete c;
    return fail(nullptr, FV_ENOMEM, "workspace too small: need " + std::to_string(W.total) + " bytes");
  }
  char* ws = (char*)workspace;
  c->insts.resize(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    const fv_grid& g = grids[i];
    Inst& I = c->insts[i];
    std::memset(&I, 0, sizeof(Inst));
    I.U = state[i];
    I.U1 = ws + W.u1[i];
    I.U2 = ws + W.u2[i];
    I.phi0 = phi0[i];
    I.bacc = (double*)(ws + W.bacc[i]);
    I.Wb = g.dim == 3 ? (void*)(ws + W.wb[i]) : nullptr;
    I.Acc = g.dim == 3 ? (void*)(ws + W.acc[i]) : nullptr;
    I.dts = (double*)(ws + W.dts[i]);
    for (int k = 0; k < 3; ++k) {
      I.n[k] = g.n[k];
      I.lo[k] = g.lo[k];
      I.dx[k] = (g.hi[k] - g.lo[k]) / g.n[k];
      I.bc[k][0] = g.bc[k][0];
      I.bc[k][1] = g.bc[k][1];
    }
    I.ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    int off = 0;
    for (int a = 0; a < 3; ++a) {
      const int nt = a < g.dim ? (int)(((int64_t)g.n[0] * g.n[1] * g.n[2]) / g.n[a]) : 0;
      I.bacc_off[2 * a] = off; off += nt * c->ops.NC;
      I.bacc_off[2 * a + 1] = off; off += nt * c->ops.NC;
    }
  }
  c->insts_d = (Inst*)(ws + W.insts);
  c->block_tab_d = (int2*)(ws + W.block_tab);
  c->bins_d = (unsigned long long*)(ws + W.bins);
  c->max_blocks = W.max_blocks;
  rc = set_tiles(c, c->var, opt->tile[2]);
  if (rc != FV_OK) {
    g_init_error = c->err;
    delete c;
    return rc;
  }
  c->h_dt.assign(n_inst * DTS_SIZE, 0.0);
  c->loaded.assign(n_inst, 0);
  for (int i = 0; i < n_inst && rc == FV_OK; ++i) rc = reset_inst(c, i, false);
  if (rc == FV_OK) rc = hip_check(c, hipStreamSynchronize(c->stream), "init sync");
  if (rc != FV_OK) {
    g_init_error = c->err;
    delete c;
    return rc;
  }
  *out = c;
  return FV_OK;
}

// zero accumulators and flag, time 0; with cfl, also the first CFL step of
// the current state (a state that has not been written is never read)
static int reset_inst(fv_ctx* c, int i, bool cfl) {
  const Inst& I = c->insts[i];
  const int q = (int)(c->step & 1);
  size_t nb = 0;
  for (int a = 0; a < c->dim; ++a) {
    const int nt = (int)(I.ncell / I.n[a]);
    nb += 2 * (size_t)nt * c->ops.NC;
  }
  int rc = hip_check(c, hipMemsetAsync(I.bacc, 0, nb * sizeof(double), c->stream), "zero accumulators");
  if (rc != FV_OK) return rc;
  double* h = &c->h_dt[(size_t)i * DTS_SIZE];
  for (int k = 0; k < DTS_SIZE; ++k) h[k] = 0.0;
  h[DTS_TEND] = HUGE_VAL;
  rc = hip_check(c, hipMemcpyAsync(I.dts, h, DTS_SIZE * sizeof(double), hipMemcpyHostToDevice, c->stream),
                 "reset dt state");
  if (rc != FV_OK || !cfl) return rc;
  c->ops.cfl(c, i, q);
  return hip_check(c, hipGetLastError(), "cfl kernel");
}

// every instance holds a written state
static int check_loaded(fv_ctx* c) {
  for (int i = 0; i < c->n_inst; ++i)
    if (!c->loaded[i])
      return fail(c, FV_ESTATE, "instance " + std::to_string(i) +
                                    " has no state: call fv_load_primitive or fv_reset first");
  return FV_OK;
}

int32_t fv_reset(fv_ctx* c) {
  if (!c) return FV_EINVAL;
  for (int i = 0; i < c->n_inst; ++i) {
    const int rc = reset_inst(c, i, true);
    if (rc != FV_OK) return rc;
    c->loaded[i] = 1;
  }
  return hip_check(c, hipStreamSynchronize(c->stream), "reset sync");
}

int32_t fv_load_primitive(fv_ctx* c, int32_t inst, const void* prim) {
  if (!c) return FV_EINVAL;
  if (inst < 0 || inst >= c->n_inst || !prim) return fail(c, FV_EINVAL, "bad instance or prim pointer");
  c->ops.p2c(c, inst, (const double*)prim);
  int rc = hip_check(c, hipGetLastError(), "prim_to_cons kernel");
  if (rc != FV_OK) return rc;
  rc = reset_inst(c, inst, true);
  if (rc != FV_OK) return rc;
  c->loaded[inst] = 1;
  return hip_check(c, hipStreamSynchronize(c->stream), "load sync");
}

int32_t fv_primitive(fv_ctx* c, int32_t inst, void* prim) {
  if (!c) return FV_EINVAL;
  if (inst < 0 || inst >= c->n_inst || !prim) return fail(c, FV_EINVAL, "bad instance or prim pointer");
  c->ops.c2p(c, inst, (double*)prim);
  return hip_check(c, hipGetLastError(), "cons_to_prim kernel");
}

static int read_dts(fv_ctx* c, std::vector<double>& h) {
  h.assign((size_t)c->n_inst * DTS_SIZE, 0.0);
  for (int i = 0; i < c->n_inst; ++i) {
    const int rc = hip_check(c, hipMemcpyAsync(&h[(size_t)i * DTS_SIZE], c->insts[i].dts,
                                                DTS_SIZE * sizeof(double), hipMemcpyDeviceToHost,
                                                c->stream), "read dt state");
    if (rc != FV_OK) return rc;
  }
  int rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
  if (rc != FV_OK) return rc;
  for (int i = 0; i < c->n_inst; ++i) {
    unsigned flag;
    std::memcpy(&flag, &h[(size_t)i * DTS_SIZE + DTS_FLAG], sizeof(unsigned));
    if (flag & FLAG_NONPHYS)
      return fail(c, FV_ENONPHYS, "non-physical state (NaN/Inf or non-positive density) in instance " +
                                      std::to_string(i));
  }
  return FV_OK;
}

int32_t fv_cfl_dt(fv_ctx* c, double* dt_host) {
  if (!c || !dt_host) return FV_EINVAL;
  if (check_loaded(c) != FV_OK) return FV_ESTATE;
  std::vector<double> h;
  const int rc = read_dts(c, h);
  if (rc != FV_OK) return rc;
  const int q = (int)(c->step & 1);
  for (int i = 0; i < c->n_inst; ++i) {
    const double* d = &h[(size_t)i * DTS_SIZE];
    double dt = d[DTS_DTFIX] > 0 ? d[DTS_DTFIX] : c->P.cfl / dts_dtinv(d, q);
    dt_host[i] = std::fmin(dt, d[DTS_TEND] - d[DTS_T + q]);
  }
  return FV_OK;
}

int32_t fv_time(fv_ctx* c, double* t_host) {
  if (!c || !t_host) return FV_EINVAL;
  std::vector<double> h;
  const int rc = read_dts(c, h);
  if (rc != FV_OK) return rc;
  const int q = (int)(c->step & 1);
  for (int i = 0; i < c->n_inst; ++i) t_host[i] = h[(size_t)i * DTS_SIZE + DTS_T + q];
  return FV_OK;
}

// ---------------------------------------------------------------------------
// checkpoint / restore of the context's own state
// ---------------------------------------------------------------------------
namespace {
constexpr double CK_MAGIC = 4.7e15;  // tag of a checkpoint blob (this dt-state layout)

size_t bacc_doubles(const fv_ctx* c, int i) {
  const Inst& I = c->insts[i];
  size_t nb = 0;
  for (int a = 0; a < c->dim; ++a) nb += 2 * (size_t)(I.ncell / I.n[a]) * c->ops.NC;
  return nb;
}

// header: magic, n_inst, step count, 0, then ncell of every instance;
// then per instance its dt state and boundary accumulators
size_t ck_doubles(const fv_ctx* c) {
  size_t n = 4 + (size_t)c->n_inst;
  for (int i = 0; i < c->n_inst; ++i) n += DTS_SIZE + bacc_doubles(c, i);
  return n;
}
}  // namespace

size_t fv_checkpoint_bytes(const fv_ctx* c) { return c ? ck_doubles(c) * sizeof(double) : 0; }

int32_t fv_checkpoint(fv_ctx* c, void* dst) {
  if (!c) return FV_EINVAL;
  if (!dst) return fail(c, FV_EINVAL, "null checkpoint buffer");
  if (check_loaded(c) != FV_OK) return FV_ESTATE;
  c->h_ck.assign(4 + c->n_inst, 0.0);
  c->h_ck[0] = CK_MAGIC;
  c->h_ck[1] = c->n_inst;
  c->h_ck[2] = (double)c->step;
  for (int i = 0; i < c->n_inst; ++i) c->h_ck[4 + i] = (double)c->insts[i].ncell;
  double* d = static_cast<double*>(dst);
  int rc = hip_check(c, hipMemcpyAsync(d, c->h_ck.data(), sizeof(double) * c->h_ck.size(),
                                       hipMemcpyHostToDevice, c->stream), "write checkpoint header");
  size_t off = c->h_ck.size();
  for (int i = 0; i < c->n_inst && rc == FV_OK; ++i) {
    const Inst& I = c->insts[i];
    rc = hip_check(c, hipMemcpyAsync(d + off, I.dts, sizeof(double) * DTS_SIZE,
                                     hipMemcpyDeviceToDevice, c->stream), "save dt state");
    off += DTS_SIZE;
    const size_t nb = bacc_doubles(c, i);
    if (rc == FV_OK && nb)
      rc = hip_check(c, hipMemcpyAsync(d + off, I.bacc, sizeof(double) * nb, hipMemcpyDeviceToDevice,
                                       c->stream), "save boundary accumulators");
    off += nb;
  }
  // the header staging buffer must outlive the copy
  if (rc == FV_OK) rc = hip_check(c, hipStreamSynchronize(c->stream), "checkpoint sync");
  return rc;
}

int32_t fv_restore(fv_ctx* c, const void* src) {
  if (!c) return FV_EINVAL;
  if (!src) return fail(c, FV_EINVAL, "null checkpoint buffer");
  const double* s = static_cast<const double*>(src);
  std::vector<double> hdr(4 + c->n_inst);
  int rc = hip_check(c, hipMemcpyAsync(hdr.data(), s, sizeof(double) * hdr.size(),
                                       hipMemcpyDeviceToHost, c->stream), "read checkpoint header");
  if (rc == FV_OK) rc = hip_check(c, hipStreamSynchronize(c->stream), "restore sync");
  if (rc != FV_OK) return rc;
  if (hdr[0] != CK_MAGIC || hdr[1] != c->n_inst)
    return fail(c, FV_EINVAL, "not a checkpoint of a context with these instances");
  for (int i = 0; i < c->n_inst; ++i)
    if (hdr[4 + i] != (double)c->insts[i].ncell)
      return fail(c, FV_EINVAL, "checkpoint grid of instance " + std::to_string(i) + " differs");
  size_t off = hdr.size();
  for (int i = 0; i < c->n_inst && rc == FV_OK; ++i) {
    const Inst& I = c->insts[i];
    rc = hip_check(c, hipMemcpyAsync(I.dts, s + off, sizeof(double) * DTS_SIZE,
                                     hipMemcpyDeviceToDevice, c->stream), "restore dt state");
    off += DTS_SIZE;
    const size_t nb = bacc_doubles(c, i);
    if (rc == FV_OK && nb)
      rc = hip_check(c, hipMemcpyAsync(I.bacc, s + off, sizeof(double) * nb, hipMemcpyDeviceToDevice,
                                       c->stream), "restore boundary accumulators");
    off += nb;
  }
  if (rc == FV_OK) rc = hip_check(c, hipStreamSynchronize(c->stream), "restore sync");
  if (rc != FV_OK) return rc;
  c->step = (long long)hdr[2];
  for (int i = 0; i < c->n_inst; ++i) c->loaded[i] = 1;
  // the restored dt state may hold a fixed step
  c->dtfix_set = true;
  return FV_OK;
}

int32_t fv_step(fv_ctx* c, const double* dt_host, int32_t n_steps, const double* t_end) {
  if (!c) return FV_EINVAL;
  if (n_steps < 0) return fail(c, FV_EINVAL, "n_steps < 0");
  if (check_loaded(c) != FV_OK) return FV_ESTATE;
  // A NULL dt_host asks for the CFL step: a fixed step set by an earlier call
  // (or restored from a checkpoint) is cleared first.
  if (dt_host || t_end || c->dtfix_set) {
    // fixed step and end time of every instance (DTS_DTFIX, DTS_TEND)
    int rc = hip_check(c, hipStreamSynchronize(c->stream), "sync before parameter write");
    if (rc != FV_OK) return rc;
    for (int i = 0; i < c->n_inst; ++i) {
      if (dt_host && !(dt_host[i] >= 0)) return fail(c, FV_EINVAL, "dt must be >= 0");
      double* h = &c->h_dt[(size_t)i * DTS_SIZE];
      h[0] = t_end ? t_end[i] : 0.0;
      h[1] = dt_host ? dt_host[i] : 0.0;
      if (t_end) {
        rc = hip_check(c, hipMemcpyAsync(c->insts[i].dts + DTS_TEND, &h[0], sizeof(double),
                                         hipMemcpyHostToDevice, c->stream), "write t_end");
        if (rc != FV_OK) return rc;
      }
      rc = hip_check(c, hipMemcpyAsync(c->insts[i].dts + DTS_DTFIX, &h[1], sizeof(double),
                                       hipMemcpyHostToDevice, c->stream), "write dt");
      if (rc != FV_OK) return rc;
    }
    rc = hip_check(c, hipStreamSynchronize(c->stream), "sync after parameter write");
    if (rc != FV_OK) return rc;
    c->dtfix_set = false;
    for (int i = 0; dt_host && i < c->n_inst; ++i) c->dtfix_set = c->dtfix_set || dt_host[i] > 0;
  }
  if (n_steps == 0) return FV_OK;
  const int p0 = (int)(c->step & 1);
  if (!c->use_graph) {
    for (int s = 0; s < n_steps; ++s) {
      const int parity = (p0 + s) & 1;
      for (int st = 1; st <= 3; ++st) c->ops.stage(c, st, parity, c->stream);
      if (c->P.seed_nu > 0) c->ops.seed(c, parity, c->stream);
    }
    c->step += n_steps;
    return hip_check(c, hipGetLastError(), "stage kernel launch");
  }
  // n_steps steps as one graph, captured on a private stream at the first
  // call with this step count and starting parity, then replayed on the
  // context's stream (launch arguments are fixed; dt, time and the CFL state
  // live on the device).  A few graphs are kept, the oldest replaced first.
  const int key = 2 * n_steps + p0;
  int slot = -1;
  for (int k = 0; k < fv_ctx::NGRAPH; ++k)
    if (c->gkey[k] == key) slot = k;
  if (slot < 0) {
    slot = c->gnext;
    c->gnext = (c->gnext + 1) % fv_ctx::NGRAPH;
    if (c->gexec[slot]) (void)hipGraphExecDestroy(c->gexec[slot]);
    c->gexec[slot] = nullptr;
    c->gkey[slot] = 0;
    int rc = FV_OK;
    if (!c->cap_stream)
      rc = hip_check(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking),
                     "capture stream");
    if (rc != FV_OK) return rc;
    rc = hip_check(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed),
                   "begin capture");
    if (rc != FV_OK) return rc;
    for (int s = 0; s < n_steps; ++s) {
      const int parity = (p0 + s) & 1;
      for (int st = 1; st <= 3; ++st) c->ops.stage(c, st, parity, c->cap_stream);
      if (c->P.seed_nu > 0) c->ops.seed(c, parity, c->cap_stream);
    }
    hipGraph_t graph = nullptr;
    const hipError_t le = hipGetLastError();
    const hipError_t ee = hipStreamEndCapture(c->cap_stream, &graph);
    rc = hip_check(c, le != hipSuccess ? le : ee, "capture step graph");
    if (rc == FV_OK)
      rc = hip_check(c, hipGraphInstantiate(&c->gexec[slot], graph, nullptr, nullptr, 0),
                     "instantiate step graph");
    if (graph) (void)hipGraphDestroy(graph);
    if (rc != FV_OK) {
      c->gexec[slot] = nullptr;
      return rc;
    }
    c->gkey[slot] = key;
  }
  c->step += n_steps;
  return hip_check(c, hipGraphLaunch(c->gexec[slot], c->stream), "step graph launch");
}

int32_t fv_autotune(fv_ctx* c, int32_t reps, int32_t max_report, int32_t* tiles, float* ms,
                    int32_t* n_variants, int32_t* chosen) {
  if (!c) return FV_EINVAL;
  if (reps < 1 || max_report < 0 || (max_report > 0 && (!tiles || !ms)))
    return fail(c, FV_EINVAL, "reps < 1 or null report arrays");
  if (check_loaded(c) != FV_OK) return FV_ESTATE;
  // configurations: every compiled tile shape under every block schedule
  // (one schedule for a single instance, where they coincide)
  const int nsched = c->n_inst > 1 ? FV_SCHED_INTERLEAVED + 1 : 1;
  const int nv = (int)c->vars.size() * nsched;
  if (n_variants) *n_variants = nv;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = hip_check(c, hipEventCreate(&e0), "event");
  if (rc == FV_OK) rc = hip_check(c, hipEventCreate(&e1), "event");
  const int orig = c->var, orig_sched = c->sched;
  int best = 0;
  float best_ms = 0.0f;
  const int parity = (int)(c->step & 1);
  for (int k = 0; k < nv && rc == FV_OK; ++k) {
    const int v = k / nsched, sc = k % nsched;
    rc = set_tiles(c, v, sc);
    if (rc != FV_OK) break;
    c->ops.stage(c, 0, parity, c->stream);  // warm-up (code object load)
    rc = hip_check(c, hipEventRecord(e0, c->stream), "event record");
    for (int r = 0; r < reps && rc == FV_OK; ++r) c->ops.stage(c, 0, parity, c->stream);
    if (rc == FV_OK) rc = hip_check(c, hipGetLastError(), "timing launch");
    if (rc == FV_OK) rc = hip_check(c, hipEventRecord(e1, c->stream), "event record");
    if (rc == FV_OK) rc = hip_check(c, hipEventSynchronize(e1), "event sync");
    float t = 0.0f;
    if (rc == FV_OK) rc = hip_check(c, hipEventElapsedTime(&t, e0, e1), "event time");
    if (rc != FV_OK) break;
    t /= (float)reps;
    if (k < max_report) {
      tiles[3 * k] = c->vars[v].TX;
      tiles[3 * k + 1] = c->vars[v].TY;
      tiles[3 * k + 2] = sc;
      ms[k] = t;
    }
    // a configuration displaces the best one listed before it only when it
    // is at least 2 % faster, so that timing noise between configurations of
    // equal speed does not change the choice from run to run
    if (k == 0 || t < 0.98f * best_ms) {
      best_ms = t;
      best = k;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  const int rc2 = rc == FV_OK ? set_tiles(c, best / nsched, best % nsched)
                              : set_tiles(c, orig, orig_sched);
  if (rc != FV_OK) return rc;
  if (chosen) *chosen = best;
  return rc2;
}

int32_t fv_totals(fv_ctx* c, double* out) {
  if (!c || !out) return FV_EINVAL;
  std::vector<double> h;
  int rc = read_dts(c, h);
  if (rc != FV_OK) return rc;
  const int NT = c->ops.NTOT, NC = c->ops.NC;
  const int nsum = c->n_inst * NT * (1 + 2 * c->dim);
  rc = hip_check(c, hipMemsetAsync(c->bins_d, 0, sizeof(unsigned long long) * NBINS * nsum, c->stream),
                 "zero bins");
  if (rc != FV_OK) return rc;
  // interior fields: masses, momenta, energy; boundary sides: same rows of
  // the conserved-flux vector (histories skipped)
  const int nm = c->nm, ns = c->ns, dim = c->dim;
  auto field_of = [&](int k) { return k < nm ? nm + k : (k < nm + dim ? 2 * nm + 2 * ns + (k - nm) : 2 * nm + 2 * ns + dim); };
  auto flux_of = [&](int k) { return k < nm ? k : (k < nm + dim ? nm + 2 * ns + (k - nm) : nm + 2 * ns + dim); };
  int slot = 0;
  for (int i = 0; i < c->n_inst; ++i) {
    const Inst& I = c->insts[i];
    for (int k = 0; k < NT; ++k, ++slot) {
      const int f = field_of(k);
      const int nblk = (int)std::min<int64_t>((I.ncell + 255) / 256, 1024);
      if (c->ops.elem == 8)
        hipLaunchKernelGGL(exact_sum_kernel<double>, dim3(nblk), dim3(256), 0, c->stream,
                           (const double*)I.U + (int64_t)f * I.ncell, I.ncell, (int64_t)1,
                           c->bins_d + (size_t)slot * NBINS);
      else
        hipLaunchKernelGGL(exact_sum_kernel<float>, dim3(nblk), dim3(256), 0, c->stream,
                           (const float*)I.U + (int64_t)f * I.ncell, I.ncell, (int64_t)1,
                           c->bins_d + (size_t)slot * NBINS);
    }
    for (int a = 0; a < dim; ++a) {
      const int nt = (int)(I.ncell / I.n[a]);
      for (int side = 0; side < 2; ++side) {
        for (int k = 0; k < NT; ++k, ++slot) {
          if (I.bc[a][side] == FV_BC_PERIODIC) continue;
          const double* base = I.bacc + I.bacc_off[2 * a + side] + flux_of(k);
          hipLaunchKernelGGL(exact_sum_kernel<double>, dim3(std::max(1, std::min(64, (nt + 255) / 256))),
                             dim3(256), 0, c->stream, base, (int64_t)nt, (int64_t)NC,
                             c->bins_d + (size_t)slot * NBINS);
        }
      }
    }
  }
  rc = hip_check(c, hipGetLastError(), "exact sum kernels");
  if (rc != FV_OK) return rc;
  std::vector<unsigned long long> bins((size_t)NBINS * nsum);
  rc = hip_check(c, hipMemcpyAsync(bins.data(), c->bins_d, bins.size() * sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, c->stream), "read bins");
  if (rc != FV_OK) return rc;
  rc = hip_check(c, hipStreamSynchronize(c->stream), "totals sync");
  if (rc != FV_OK) return rc;
  slot = 0;
  for (int i = 0; i < c->n_inst; ++i) {
    const Inst& I = c->insts[i];
    const double vol = I.dx[0] * I.dx[1] * I.dx[2];
    double* o = out + (size_t)i * 2 * NT;
    for (int k = 0; k < NT; ++k, ++slot) o[k] = bins_to_double(&bins[(size_t)slot * NBINS]) * vol;
    // boundary: per side exact sum times face area, then an exact sum of the
    // per-side values
    std::vector<std::vector<double>> per(NT);
    for (int a = 0; a < dim; ++a) {
      const double area = a == 0 ? I.dx[1] * I.dx[2] : (a == 1 ? I.dx[0] * I.dx[2] : I.dx[0] * I.dx[1]);
      for (int side = 0; side < 2; ++side)
        for (int k = 0; k < NT; ++k, ++slot)
          per[k].push_back(bins_to_double(&bins[(size_t)slot * NBINS]) * area);
    }
    for (int k = 0; k < NT; ++k) {
      unsigned long long hb[NBINS] = {0};
      for (double v : per[k]) {
        // host copy of bin_add
        uint64_t bits;
        std::memcpy(&bits, &v, 8);
        const int ex = (int)((bits >> 52) & 0x7FF);
        uint64_t m = bits & ((1ull << 52) - 1);
        if (ex == 0x7FF) continue;
        int shift = 0;
        if (ex != 0) { m |= 1ull << 52; shift = ex - 1; }
        if (!m) continue;
        const int k0 = shift >> 5, off = shift & 31;
        const uint64_t t0 = (m & 0xFFFFFFFFull) << off, t1 = (m >> 32) << off;
        const uint64_t c0 = t0 & 0xFFFFFFFFull, c1 = (t0 >> 32) + (t1 & 0xFFFFFFFFull), c2 = t1 >> 32;
        const bool neg = bits >> 63;
        hb[k0] += neg ? 0ull - c0 : c0;
        hb[k0 + 1] += neg ? 0ull - c1 : c1;
        hb[k0 + 2] += neg ? 0ull - c2 : c2;
      }
      o[NT + k] = bins_to_double(hb);
    }
  }
  return FV_OK;
}

// ---------------------------------------------------------------------------
// fragments
// ---------------------------------------------------------------------------
namespace {
struct FragPlan {
  size_t fid, bcount, n_root, flabel, fcount, fflag, fbins, total;
  int nblk;
};

FragPlan plan_frag(int64_t ncell, int64_t cap) {
  FragPlan F{};
  F.nblk = (int)((ncell + 255) / 256);
  size_t o = 0;
  F.fid = o;     o = align256(o + sizeof(int) * (size_t)ncell);
  F.bcount = o;  o = align256(o + sizeof(int) * (size_t)F.nblk);
  F.n_root = o;  o = align256(o + sizeof(long long));
  F.flabel = o;  o = align256(o + sizeof(int) * (size_t)cap);
  F.fcount = o;  o = align256(o + sizeof(unsigned long long) * (size_t)cap);
  F.fflag = o;   o = align256(o + sizeof(unsigned int) * (size_t)cap);
  F.fbins = o;   o = align256(o + sizeof(unsigned long long) * NBINS * (size_t)cap);
  F.total = o;
  return F;
}
}  // namespace

size_t fv_fragment_workspace_bytes(const fv_ctx* c, int32_t inst, int64_t cap) {
  if (!c || inst < 0 || inst >= c->n_inst || cap < 0) return 0;
  return plan_frag(c->insts[inst].ncell, cap).total;
}

int32_t fv_fragment_histogram(const fv_fragment* frags, int64_t n, const double* edges,
                              int32_t n_edges, int64_t* counts) {
  if (n < 0 || n_edges < 0 || (n > 0 && !frags) || (n_edges > 0 && (!edges || !counts)))
    return FV_EINVAL;
  std::vector<double> m((size_t)n);
  for (int64_t i = 0; i < n; ++i) m[(size_t)i] = frags[i].mass;
  std::sort(m.begin(), m.end());
  // fragments at or above an edge: those past the first mass not below it
  for (int32_t k = 0; k < n_edges; ++k)
    counts[k] = (int64_t)(m.end() - std::lower_bound(m.begin(), m.end(), edges[k]));
  return FV_OK;
}

}  // extern "C"

// fv_fragments and fv_fragments_noalloc: frag_ws is the fragment workspace
// (the caller's buffer, or this library's static scratch array); what the
// kernels need zeroed is cleared here with a fill kernel.
static int32_t fragments_impl(fv_ctx* c, int32_t inst, double cut, int32_t* labels,
                              void* frag_ws, size_t frag_ws_bytes, int64_t cap, int64_t* n_frag,
                              fv_fragment* out) {
  if (inst < 0 || inst >= c->n_inst) return fail(c, FV_EINVAL, "bad instance");
  if (!labels || !frag_ws || !n_frag) return fail(c, FV_EINVAL, "null labels, workspace or n_frag");
  if (cap < 0 || (cap > 0 && !out)) return fail(c, FV_EINVAL, "bad cap or null output array");
  if (!(cut == cut) || cut - cut != 0.0) return fail(c, FV_EINVAL, "cut must be finite");
  if (c->ns < 1) return fail(c, FV_EINVAL, "no solid material");
  const Inst& I = c->insts[inst];
  if (I.ncell > 0x7FFFFFFF) return fail(c, FV_EINVAL, "more than 2^31 - 1 cells");
  const FragPlan F = plan_frag(I.ncell, cap);
  if (frag_ws_bytes < F.total)
    return fail(c, FV_ENOMEM, "fragment workspace too small: need " + std::to_string(F.total) + " bytes");
  *n_frag = 0;
  char* ws = static_cast<char*>(frag_ws);
  int* fid = reinterpret_cast<int*>(ws + F.fid);
  int* bcount = reinterpret_cast<int*>(ws + F.bcount);
  long long* n_root = reinterpret_cast<long long*>(ws + F.n_root);
  int* flabel = reinterpret_cast<int*>(ws + F.flabel);
  unsigned long long* fcount = reinterpret_cast<unsigned long long*>(ws + F.fcount);
  unsigned int* fflag = reinterpret_cast<unsigned int*>(ws + F.fflag);
  unsigned long long* fbins = reinterpret_cast<unsigned long long*>(ws + F.fbins);
  const CclGrid g{I.n[0], I.n[1], I.n[2], I.ncell};
  const dim3 grid((unsigned)F.nblk), blk(256);
  hipStream_t s = c->stream;
  // the solid is material 0: its volume fraction is field 0, its phasic
  // mass field nm
  if (c->ops.elem == 8)
    hipLaunchKernelGGL(ccl_init_kernel<double>, grid, blk, 0, s, (const double*)I.U, cut, g, labels);
  else
    hipLaunchKernelGGL(ccl_init_kernel<float>, grid, blk, 0, s, (const float*)I.U, cut, g, labels);
  hipLaunchKernelGGL(ccl_merge_kernel, grid, blk, 0, s, g, labels);
  hipLaunchKernelGGL(ccl_compress_kernel, grid, blk, 0, s, g, labels);
  hipLaunchKernelGGL(ccl_count_kernel, grid, blk, 0, s, g, (const int*)labels, bcount);
  hipLaunchKernelGGL(ccl_scan_kernel, dim3(1), dim3(1024), 0, s, F.nblk, bcount, n_root);
  int rc = hip_check(c, hipGetLastError(), "labelling kernels");
  if (rc != FV_OK) return rc;
  long long nr = 0;
  rc = hip_check(c, hipMemcpyAsync(&nr, n_root, sizeof(nr), hipMemcpyDeviceToHost, s), "read count");
  if (rc == FV_OK) rc = hip_check(c, hipStreamSynchronize(s), "labelling sync");
  if (rc != FV_OK) return rc;
  *n_frag = nr;
  if (nr > cap)
    return fail(c, FV_ENOMEM, std::to_string(nr) + " fragments exceed cap " + std::to_string(cap));
  if (nr == 0) return FV_OK;
  hipLaunchKernelGGL(ccl_assign_kernel, grid, blk, 0, s, g, (const int*)labels, (const int*)bcount,
                     fid, flabel);
  // per-fragment counters start at zero (a fill kernel: the scratch array
  // keeps the previous call's contents)
  auto zero = [&](void* p, int64_t words) {
    hipLaunchKernelGGL(zero_words_kernel,
                       dim3((unsigned)std::min<int64_t>((words + 255) / 256, 4096)), dim3(256), 0,
                       s, reinterpret_cast<unsigned int*>(p), words);
  };
  zero(fcount, 2 * nr);
  zero(fflag, nr);
  zero(fbins, 2 * (int64_t)NBINS * nr);
  rc = hip_check(c, hipGetLastError(), "zero fragment counters");
  if (rc != FV_OK) return rc;
  if (c->ops.elem == 8)
    hipLaunchKernelGGL(ccl_stats_kernel<double>, grid, blk, 0, s, g, (const int*)labels, (const int*)fid,
                       (const double*)I.U + (int64_t)c->nm * I.ncell, fbins, fcount, fflag);
  else
    hipLaunchKernelGGL(ccl_stats_kernel<float>, grid, blk, 0, s, g, (const int*)labels, (const int*)fid,
                       (const float*)I.U + (int64_t)c->nm * I.ncell, fbins, fcount, fflag);
  rc = hip_check(c, hipGetLastError(), "fragment statistics kernel");
  if (rc != FV_OK) return rc;
  std::vector<int> hl((size_t)nr);
  std::vector<unsigned long long> hc((size_t)nr), hb((size_t)nr * NBINS);
  std::vector<unsigned int> hf((size_t)nr);
  rc = hip_check(c, hipMemcpyAsync(hl.data(), flabel, sizeof(int) * nr, hipMemcpyDeviceToHost, s), "read labels");
  if (rc == FV_OK)
    rc = hip_check(c, hipMemcpyAsync(hc.data(), fcount, sizeof(unsigned long long) * nr, hipMemcpyDeviceToHost, s),
                   "read counts");
  if (rc == FV_OK)
    rc = hip_check(c, hipMemcpyAsync(hf.data(), fflag, sizeof(unsigned int) * nr, hipMemcpyDeviceToHost, s),
                   "read flags");
  if (rc == FV_OK)
    rc = hip_check(c, hipMemcpyAsync(hb.data(), fbins, sizeof(unsigned long long) * NBINS * nr,
                                     hipMemcpyDeviceToHost, s), "read bins");
  if (rc == FV_OK) rc = hip_check(c, hipStreamSynchronize(s), "fragment sync");
  if (rc != FV_OK) return rc;
  const double vol = I.dx[0] * I.dx[1] * I.dx[2];
  for (long long f = 0; f < nr; ++f) {
    out[f].label = hl[f];
    out[f].n_cells = (int64_t)hc[f];
    out[f].mass = bins_to_double(&hb[(size_t)f * NBINS]) * vol;
    out[f].touches_boundary = hf[f] ? 1 : 0;
    out[f].reserved = 0;
  }
  return FV_OK;
}

extern "C" {

int32_t fv_fragments(fv_ctx* c, int32_t inst, double cut, int32_t* labels, void* frag_ws,
                     size_t frag_ws_bytes, int64_t cap, int64_t* n_frag, fv_fragment* out) {
  if (!c) return FV_EINVAL;
  return fragments_impl(c, inst, cut, labels, frag_ws, frag_ws_bytes, cap, n_frag, out);
}

int32_t fv_fragments_noalloc(fv_ctx* c, int32_t inst, double cut, int32_t* labels, int64_t cap,
                             int64_t* n_frag, fv_fragment* out) {
  if (!c) return FV_EINVAL;
  if (inst < 0 || inst >= c->n_inst) return fail(c, FV_EINVAL, "bad instance");
  if (cap < 0) return fail(c, FV_EINVAL, "bad cap or null output array");
  void* ws = scratch_ptr(c->device);
  if (!ws) return fail(c, FV_EDEVICE, "fragment scratch address of device " +
                                          std::to_string(c->device) + " unknown");
  const size_t need = plan_frag(c->insts[inst].ncell, cap).total;
  if (need > (size_t)FV_FRAGMENT_SCRATCH_BYTES)
    return fail(c, FV_ENOMEM, "instance and cap need " + std::to_string(need) +
                                  " bytes of fragment scratch, above the static " +
                                  std::to_string((size_t)FV_FRAGMENT_SCRATCH_BYTES) +
                                  " (use fv_fragments with a workspace)");
  return fragments_impl(c, inst, cut, labels, ws, (size_t)FV_FRAGMENT_SCRATCH_BYTES, cap, n_frag,
                        out);
}

const char* fv_last_error(const fv_ctx* c) {
  return c ? c->err.c_str() : g_init_error.c_str();
}

void fv_destroy(fv_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

}  // extern "C"

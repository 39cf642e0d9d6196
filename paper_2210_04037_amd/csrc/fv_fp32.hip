// The FP32-bulk form of the stage kernels: FP32 state and fluxes, with the
// double-precision islands of fv_stage.hpp (trace-fraction pressure
// inversion, plastic return, totals).  This translation unit is compiled
// with fast reciprocals and approximate transcendental functions; the FP64
// form (fv_api.hip) keeps IEEE division and library functions.
#include "fv_kernels.hpp"

namespace fvk {

bool select_ops_fp32(int dim, int nm, int ns, Ops& o, hipError_t& herr, bool set_attr) {
  herr = hipSuccess;
  FV_SEL(1, 1, 1, float, float, 256, 1)
  FV_SEL(1, 2, 1, float, float, 256, 1)
  FV_SEL(2, 1, 1, float, float, 32, 16)
  FV_SEL(2, 2, 1, float, float, 32, 16)
  return false;
}

}  // namespace fvk

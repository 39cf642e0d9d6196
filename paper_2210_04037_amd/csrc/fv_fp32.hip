// The FP32-bulk form of the stage kernels: FP32 state and fluxes, with the
// double-precision islands of fv_stage.hpp (trace-fraction pressure
// inversion, plastic return, totals).  This translation unit is compiled
// with fast reciprocals and approximate transcendental functions; the FP64
// form (fv_fp64.hip) keeps IEEE division and library functions.
#include "fv_launch.hpp"

namespace fvk {

bool select_ops_fp32(int dim, int nm, int ns, bool ext, std::vector<Ops>& vars,
                     hipError_t& herr,
                     bool set_attr) {
  herr = hipSuccess;
  vars.clear();
  if (dim == 1 && nm == 1 && ns == 1) {
    FV_VAR(1, 1, 1, float, float, 256, 1)
    FV_VARN(1, 1, 1, float, float, 255, 1, 256)
    FV_VAR(1, 1, 1, float, float, 128, 1)
    FV_VARN(1, 1, 1, float, float, 127, 1, 128)
    FV_VAR(1, 1, 1, float, float, 64, 1)
    return true;
  }
  if (dim == 1 && nm == 2 && ns == 1) {
    FV_VAR(1, 2, 1, float, float, 256, 1)
    FV_VARN(1, 2, 1, float, float, 255, 1, 256)
    FV_VAR(1, 2, 1, float, float, 128, 1)
    FV_VARN(1, 2, 1, float, float, 127, 1, 128)
    FV_VAR(1, 2, 1, float, float, 64, 1)
    return true;
  }
  // two solids (Section 4.1: an aluminium flyer on a copper target), 1D
  if (dim == 1 && nm == 2 && ns == 2) {
    FV_VAR(1, 2, 2, float, float, 256, 1)
    FV_VAR(1, 2, 2, float, float, 128, 1)
    return true;
  }
  if (dim == 2 && nm == 1 && ns == 1) {
    FV_VARN(2, 1, 1, float, float, 16, 14, 256)
    FV_VARN(2, 1, 1, float, float, 16, 15, 256)
    FV_VARN(2, 1, 1, float, float, 32, 7, 256)
    FV_VARN(2, 1, 1, float, float, 15, 16, 256)
    FV_VARN(2, 1, 1, float, float, 32, 15, 512)
    FV_VAR(2, 1, 1, float, float, 64, 8)
    FV_VAR(2, 1, 1, float, float, 32, 8)
    return true;
  }
  if (dim == 2 && nm == 2 && ns == 1) {
    FV_VARN(2, 2, 1, float, float, 16, 14, 256)
    FV_VARN(2, 2, 1, float, float, 16, 15, 256)
    FV_VARN(2, 2, 1, float, float, 32, 7, 256)
    FV_VARN(2, 2, 1, float, float, 15, 16, 256)
    FV_VARN(2, 2, 1, float, float, 32, 15, 512)
    FV_VAR(2, 2, 1, float, float, 64, 8)
    FV_VAR(2, 2, 1, float, float, 32, 8)
    return true;
  }
  if (dim == 3 && nm == 1 && ns == 1) {
    FV_VAR3(1, 1, float, float)
    return true;
  }
  if (dim == 3 && nm == 2 && ns == 1) {
    FV_VAR3(2, 1, float, float)
    return true;
  }
  return false;
}

}  // namespace fvk

// The plain FP64 form of the stage kernels (state and arithmetic in double,
// IEEE division and library functions): the reference form the oracle
// checks and the FP32-bulk form is measured against.
#include "fv_launch.hpp"

namespace fvk {

bool select_ops_fp64(int dim, int nm, int ns, bool ext, std::vector<Ops>& vars,
                     hipError_t& herr,
                     bool set_attr) {
  herr = hipSuccess;
  vars.clear();
  if (dim == 1 && nm == 1 && ns == 1) {
    FV_VAR(1, 1, 1, double, double, 256, 1)
    FV_VARN(1, 1, 1, double, double, 255, 1, 256)
    FV_VAR(1, 1, 1, double, double, 128, 1)
    FV_VARN(1, 1, 1, double, double, 127, 1, 128)
    FV_VAR(1, 1, 1, double, double, 64, 1)
    return true;
  }
  if (dim == 1 && nm == 2 && ns == 1) {
    FV_VAR(1, 2, 1, double, double, 256, 1)
    FV_VARN(1, 2, 1, double, double, 255, 1, 256)
    FV_VAR(1, 2, 1, double, double, 128, 1)
    FV_VARN(1, 2, 1, double, double, 127, 1, 128)
    FV_VAR(1, 2, 1, double, double, 64, 1)
    return true;
  }
  // two solids (Section 4.1: an aluminium flyer on a copper target), 1D
  if (dim == 1 && nm == 2 && ns == 2) {
    FV_VAR(1, 2, 2, double, double, 256, 1)
    FV_VAR(1, 2, 2, double, double, 128, 1)
    return true;
  }
  if (dim == 2 && nm == 1 && ns == 1) {
    FV_VARN(2, 1, 1, double, double, 16, 15, 256)
    FV_VARN(2, 1, 1, double, double, 32, 7, 256)
    FV_VARN(2, 1, 1, double, double, 16, 7, 128)
    FV_VAR(2, 1, 1, double, double, 16, 8)
    FV_VAR(2, 1, 1, double, double, 32, 8)
    return true;
  }
  if (dim == 2 && nm == 2 && ns == 1) {
    FV_VARN(2, 2, 1, double, double, 16, 15, 256)
    FV_VARN(2, 2, 1, double, double, 32, 7, 256)
    FV_VARN(2, 2, 1, double, double, 16, 7, 128)
    FV_VAR(2, 2, 1, double, double, 16, 8)
    // no 32 x 8 tile: that build of this kernel (256 VGPRs and 12 spilled to
    // accumulation registers, the most of any shape) drifts from the oracle
    // (4.7e-8 after 20 steps of the ring) while every other shape, from the
    // same source, agrees with it to 1e-12 and bitwise with each other
    return true;
  }
  if (dim == 3 && nm == 1 && ns == 1) {
    FV_VAR3(1, 1, double, double)
    return true;
  }
  if (dim == 3 && nm == 2 && ns == 1) {
    FV_VAR3(2, 1, double, double)
    return true;
  }
  return false;
}

}  // namespace fvk

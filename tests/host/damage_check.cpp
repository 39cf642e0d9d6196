// Host evaluation of the kernels' damage closures (fv_core.hpp) for the
// threshold-strain and damage-rate test.  stdin: a solid's eps_th, eps_c,
// n_hard, bonora_alpha, D_crit, D0, K0, G0 on the first line, then one
// "R D eps" triple per line; prints the threshold strain at R and the damage
// rate dD/d(eps_p) at (D, eps, R) per line.
#include <cstdio>
#include <cstring>

#include "../../paper_2210_04037_amd/csrc/fv_core.hpp"

int main() {
  fv::MatP m;
  std::memset(&m, 0, sizeof(m));
  if (std::scanf("%lf %lf %lf %lf %lf %lf %lf %lf", &m.eps_th, &m.eps_c, &m.nhard, &m.balpha,
                 &m.Dcrit, &m.D0, &m.K0, &m.G0) != 8)
    return 2;
  fv::set_solid_constants(m);
  double R, D, eps;
  while (std::scanf("%lf %lf %lf", &R, &D, &eps) == 3)
    std::printf("%.17g %.17g\n", fv::eps_threshold(m, R), fv::bonora_rate(m, D, eps, R));
  return 0;
}

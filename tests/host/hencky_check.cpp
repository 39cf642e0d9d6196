// Host evaluation of the kernels' Hencky strain (fv_core.hpp) for the
// conditioning test: reads a dimension, then the 9 entries of V row by row,
// one stretch per line on stdin; prints the 9 entries of dev H per line.
#include <cstdio>

#include "../../paper_2210_04037_amd/csrc/fv_core.hpp"

int main() {
  int dim = 0;
  if (std::scanf("%d", &dim) != 1 || dim < 2 || dim > 3) return 2;
  double v[9];
  while (true) {
    for (int k = 0; k < 9; ++k)
      if (std::scanf("%lf", &v[k]) != 1) return 0;
    double V[3][3], H[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) V[i][j] = v[3 * i + j];
    if (dim == 2)
      fv::hencky<2, double>(V, H);
    else
      fv::hencky<3, double>(V, H);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) std::printf("%.17g ", H[i][j]);
    std::printf("\n");
  }
}

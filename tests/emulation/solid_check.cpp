// TEST INFRASTRUCTURE: the solid ratio of solid.h (the kernels' code) compiled for the host
// against the emulated HIP headers.  Reads lines "r dx dy" from stdin and prints the single-
// and double-precision ratios of each cell, for comparison with the oracle's exact area.
#include "hip/hip_runtime.h"

#include <cstdio>

#include "solid.h"

int main() {
  double r, dx, dy;
  while (std::scanf("%lf %lf %lf", &r, &dx, &dy) == 3) {
    const float f = imb::cell_solid_ratio<float>((float)r, (float)dx, (float)dy, 0);
    const double d = imb::cell_solid_ratio<double>(r, dx, dy, 0);
    std::printf("%.9e %.17e\n", (double)f, d);
  }
  return 0;
}

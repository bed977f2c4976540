// Separating-axis test of a triangle against an axis-aligned box in FP64
// (the 13 axes: the 9 products of box axes and triangle edges, the 3 box
// normals, the triangle normal), closed: touching counts. Sums of products
// are taken left to right and the files that include this are compiled
// without contraction, so the test is the plain definition evaluated in a
// fixed order. Shared by the generation front end and the facet registration.
#pragma once

#include <hip/hip_runtime.h>

namespace fppg {

struct Tri {
  double a[3], b[3], c[3];
};

__device__ __forceinline__ bool separated(double p0, double p1, double p2, double r) {
  return fmin(fmin(p0, p1), p2) > r || fmax(fmax(p0, p1), p2) < -r;
}

// Separating-axis test of triangle T against the box of centre c, half-width h.
__device__ inline bool tri_box(const Tri& T, const double c[3], double h) {
  double v0[3], v1[3], v2[3];
  for (int q = 0; q < 3; ++q) {
    v0[q] = T.a[q] - c[q];
    v1[q] = T.b[q] - c[q];
    v2[q] = T.c[q] - c[q];
  }
  double e[3][3];
  for (int q = 0; q < 3; ++q) {
    e[0][q] = v1[q] - v0[q];
    e[1][q] = v2[q] - v1[q];
    e[2][q] = v0[q] - v2[q];
  }
  // axes e_k x f: (0, -f2, f1), (f2, 0, -f0), (-f1, f0, 0)
  for (int m = 0; m < 3; ++m) {
    const double f0 = e[m][0], f1 = e[m][1], f2 = e[m][2];
    {
      const double r = h * fabs(f2) + h * fabs(f1);
      if (separated(v0[1] * -f2 + v0[2] * f1, v1[1] * -f2 + v1[2] * f1, v2[1] * -f2 + v2[2] * f1, r)) return false;
    }
    {
      const double r = h * fabs(f2) + h * fabs(f0);
      if (separated(v0[0] * f2 + v0[2] * -f0, v1[0] * f2 + v1[2] * -f0, v2[0] * f2 + v2[2] * -f0, r)) return false;
    }
    {
      const double r = h * fabs(f1) + h * fabs(f0);
      if (separated(v0[0] * -f1 + v0[1] * f0, v1[0] * -f1 + v1[1] * f0, v2[0] * -f1 + v2[1] * f0, r)) return false;
    }
  }
  for (int q = 0; q < 3; ++q)
    if (fmin(fmin(v0[q], v1[q]), v2[q]) > h || fmax(fmax(v0[q], v1[q]), v2[q]) < -h) return false;
  const double nx = e[0][1] * e[1][2] - e[0][2] * e[1][1];
  const double ny = e[0][2] * e[1][0] - e[0][0] * e[1][2];
  const double nz = e[0][0] * e[1][1] - e[0][1] * e[1][0];
  const double d = (nx * v0[0] + ny * v0[1]) + nz * v0[2];
  const double r = (h * fabs(nx) + h * fabs(ny)) + h * fabs(nz);
  return !(fabs(d) > r);
}

}  // namespace fppg

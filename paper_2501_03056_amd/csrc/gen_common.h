// Helpers of the particle generation front end (sections 3.1.1, 3.1.2,
// 3.2.1), shared by the dense classification (generate.hip) and the sparse
// path through the Morton/hash storage (gen_sparse.hip). FP64 throughout,
// sums of three products left to right, no contraction.
#pragma once

#include "internal.h"
#include "sat.h"

namespace fppg {
// Stable LSD radix sort of (keys, vals) by val bits [0, val_bits), then key
// bits [0, key_bits), 4-bit digits (register.hip); the four pointers are
// swapped so that keys/vals hold the result. Synchronous on s.
fppg_status radix_sort_pairs(fppg_ctx* ctx, uint64_t*& keys, uint32_t*& vals, uint64_t*& ktmp, uint32_t*& vtmp,
                             int n, int val_bits, int key_bits, hipStream_t s);

namespace gen {

using fppg::Tri;
using fppg::tri_box;

constexpr uint8_t kExternal = 0, kInternal = 1, kSurface = 2;
constexpr int kWave = 64;

struct Grid {
  double o[3];
  double dx;
  int n[3];
};

__device__ __forceinline__ double centre(const Grid& g, int a, int i) { return g.o[a] + (double(i) + 0.5) * g.dx; }

__device__ __forceinline__ int64_t cell_index(const Grid& g, int i, int j, int k) {
  return (int64_t(k) * g.n[1] + j) * g.n[0] + i;
}

// Cell range of [lo, hi] along axis a, widened by one cell, clamped.
__device__ __forceinline__ void cell_range(const Grid& g, int a, double lo, double hi, int& i0, int& i1) {
  i0 = min(max(int(floor((lo - g.o[a]) / g.dx)) - 1, 0), g.n[a] - 1);
  i1 = min(max(int(floor((hi - g.o[a]) / g.dx)) + 1, 0), g.n[a] - 1);
}

__device__ __forceinline__ Tri load_tri(const double* __restrict__ vert, const int* __restrict__ tri, int t) {
  Tri T;
  const int ia = tri[3 * t], ib = tri[3 * t + 1], ic = tri[3 * t + 2];
  for (int q = 0; q < 3; ++q) {
    T.a[q] = vert[3 * ia + q];
    T.b[q] = vert[3 * ib + q];
    T.c[q] = vert[3 * ic + q];
  }
  return T;
}

// Projection of c along the unit normal of T: plane distance d, foot p, and
// whether the foot lies in T (all barycentric coordinates >= 0).
__device__ inline bool project_inside(const Tri& T, const double c[3], double& d, double p[3]) {
  double e0[3], e1[3];
  for (int q = 0; q < 3; ++q) {
    e0[q] = T.b[q] - T.a[q];
    e1[q] = T.c[q] - T.a[q];
  }
  double n[3] = {e0[1] * e1[2] - e0[2] * e1[1], e0[2] * e1[0] - e0[0] * e1[2], e0[0] * e1[1] - e0[1] * e1[0]};
  const double len = sqrt((n[0] * n[0] + n[1] * n[1]) + n[2] * n[2]);
  for (int q = 0; q < 3; ++q) n[q] = n[q] / len;
  d = ((c[0] - T.a[0]) * n[0] + (c[1] - T.a[1]) * n[1]) + (c[2] - T.a[2]) * n[2];
  double v[3];
  for (int q = 0; q < 3; ++q) {
    p[q] = c[q] - d * n[q];
    v[q] = p[q] - T.a[q];
  }
  const double d00 = (e0[0] * e0[0] + e0[1] * e0[1]) + e0[2] * e0[2];
  const double d01 = (e0[0] * e1[0] + e0[1] * e1[1]) + e0[2] * e1[2];
  const double d11 = (e1[0] * e1[0] + e1[1] * e1[1]) + e1[2] * e1[2];
  const double d20 = (v[0] * e0[0] + v[1] * e0[1]) + v[2] * e0[2];
  const double d21 = (v[0] * e1[0] + v[1] * e1[1]) + v[2] * e1[2];
  const double den = d00 * d11 - d01 * d01;
  const double lb = (d11 * d20 - d01 * d21) / den;
  const double lc = (d00 * d21 - d01 * d20) / den;
  return fmin(fmin(1.0 - lb - lc, lb), lc) >= 0.0;
}

// Edge function of the directed edge (ax, ay) -> (bx, by) at (px, py), with
// the endpoints taken in lexicographic order and the sign restored.
__device__ __forceinline__ double edge_fn(double ax, double ay, double bx, double by, double px, double py) {
  const bool swap = ax > bx || (ax == bx && ay > by);
  const double ux = swap ? bx : ax, uy = swap ? by : ay, wx = swap ? ax : bx, wy = swap ? ay : by;
  const double e = (wx - ux) * (py - uy) - (wy - uy) * (px - ux);
  return swap ? -e : e;
}

__device__ __forceinline__ bool edge_in(double ax, double ay, double bx, double by, double px, double py) {
  const double e = edge_fn(ax, ay, bx, by, px, py);
  const double dxe = bx - ax, dye = by - ay;
  return e > 0.0 || (e == 0.0 && (dye < 0.0 || (dye == 0.0 && dxe < 0.0)));
}

// The vertical crossings of one facet (section 3.1.2 ray casting, reading
// R20): the columns under its xy box whose centre lies in its xy projection
// (fill rule by the edge functions above) and, for each, the first cell whose
// centre lies strictly above the crossing (g.n[2]: none). Vertical facets
// (zero projected area) are not crossed.
struct Crossing {
  bool valid;
  double p0x, p0y, p1x, p1y, p2x, p2y, q1x, q1y, q2x, q2y, area;
  double az, bz, cz;
  int r0[2], sx, sy;
};

__device__ __forceinline__ Crossing crossing_of(const Tri& T, const Grid& g) {
  Crossing X;
  X.p0x = T.a[0]; X.p0y = T.a[1]; X.p1x = T.b[0]; X.p1y = T.b[1]; X.p2x = T.c[0]; X.p2y = T.c[1];
  X.az = T.a[2]; X.bz = T.b[2]; X.cz = T.c[2];
  X.area = (X.p1x - X.p0x) * (X.p2y - X.p0y) - (X.p1y - X.p0y) * (X.p2x - X.p0x);
  X.valid = X.area != 0.0;
  const bool cw = X.area < 0.0;
  X.q1x = cw ? X.p2x : X.p1x; X.q1y = cw ? X.p2y : X.p1y; X.q2x = cw ? X.p1x : X.p2x; X.q2y = cw ? X.p1y : X.p2y;
  int r1[2];
  for (int a = 0; a < 2; ++a) {
    const double lo = fmin(fmin(T.a[a], T.b[a]), T.c[a]), hi = fmax(fmax(T.a[a], T.b[a]), T.c[a]);
    cell_range(g, a, lo, hi, X.r0[a], r1[a]);
  }
  X.sx = r1[0] - X.r0[0] + 1;
  X.sy = r1[1] - X.r0[1] + 1;
  return X;
}

// The cell toggled in column (i, j), or -1 if the column is not crossed.
__device__ __forceinline__ int crossing_cell(const Crossing& X, const Grid& g, int i, int j) {
  const double px = centre(g, 0, i), py = centre(g, 1, j);
  if (!(edge_in(X.p0x, X.p0y, X.q1x, X.q1y, px, py) && edge_in(X.q1x, X.q1y, X.q2x, X.q2y, px, py) &&
        edge_in(X.q2x, X.q2y, X.p0x, X.p0y, px, py)))
    return -1;
  const double l1 = ((px - X.p0x) * (X.p2y - X.p0y) - (py - X.p0y) * (X.p2x - X.p0x)) / X.area;
  const double l2 = ((X.p1x - X.p0x) * (py - X.p0y) - (X.p1y - X.p0y) * (px - X.p0x)) / X.area;
  const double z = X.az + l1 * (X.bz - X.az) + l2 * (X.cz - X.az);
  // first cell whose centre lies strictly above z
  double fk = floor((z - g.o[2]) / g.dx - 0.5) + 1.0;
  int k = int(fmin(fmax(fk, 0.0), double(g.n[2])));
  while (k > 0 && centre(g, 2, k - 1) > z) --k;
  while (k < g.n[2] && !(centre(g, 2, k) > z)) ++k;
  return k;
}

}  // namespace gen
}  // namespace fppg

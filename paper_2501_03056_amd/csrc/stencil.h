// Culled stencil walk over the particle cell list, shared by the pair-sweep
// kernels (forces, Jacobian products, energy, density loss, neighbour export).
//
// One lane per sorted receiver. The cell key runs fastest along x, so the
// cells of a stencil row along x are contiguous in the sorted order and a
// receiver visits at most (2k+1)^2 contiguous index ranges. Rows and the x-extent of a
// row are culled in cell units against the support radius: a skipped cell is
// at least k cell edges (> 2h, the edge being (2h/k)(1+2^-9) or more) from the
// receiver, so it holds no source and culled sums are bitwise identical to
// full-stencil sums. Along x the cells are kXSplit times narrower (the x
// coordinate in x-cell units is exactly kXSplit times the one in cell units),
// so a row reaches k kXSplit x-cells and ends within half a cell edge of the
// receiver's support sphere. Sources are visited in a fixed order (rows by dz then dy
// ascending, then sorted index).
#pragma once

#include "internal.h"

namespace fppg {

// Receiver cell and its fractional position inside the cell (cell units).
struct Stencil {
  int x, y, z;
  float fx, fy, fz;
};

__device__ __forceinline__ Stencil stencil_of(const float4 p, const GeomDev& G) {
  float tx = (p.x - G.origin[0]) * G.inv_cell_x;
  float ty = (p.y - G.origin[1]) * G.inv_cell;
  float tz = (p.z - G.origin[2]) * G.inv_cell;
  // clamping moves an outside receiver onto the grid box: gaps only shrink
  tx = fminf(fmaxf(tx, 0.0f), float(G.dims[0] - 1));
  ty = fminf(fmaxf(ty, 0.0f), float(G.dims[1] - 1));
  tz = fminf(fmaxf(tz, 0.0f), float(G.dims[2] - 1));
  const float cx = floorf(tx), cy = floorf(ty), cz = floorf(tz);
  return Stencil{int(cx), int(cy), int(cz), tx - cx, ty - cy, tz - cz};
}

// Distance in cell units from a receiver at fraction f of its cell to the
// cell d cells away along one axis.
__device__ __forceinline__ float cell_gap(int d, float f) {
  return d > 0 ? float(d) - f : (d < 0 ? f + float(-d - 1) : 0.0f);
}

// Keys of a receiver's stencil rows. Within one slab row_key is linear in
// (y, z): the row dy, dz away has key base + dz zstep + dy nx, base being the
// receiver's own row. linear: every row of the stencil on the grid lies in
// the receiver's slab (always so with one slab over the whole y range).
struct RowKeys {
  int base, zstep;
  bool linear;
};

__device__ __forceinline__ RowKeys row_keys(const Stencil s, const GeomDev& G, int k) {
  const int S = G.slab;
  const int y0 = int((float(s.y) + 0.5f) * G.inv_slab) * S;
  const int w = min(S, G.dims[1] - y0);
  return RowKeys{int(G.cell_begin) + y0 * G.dims[0] * G.dims[2] + (s.z * w + (s.y - y0)) * G.dims[0],
                 w * G.dims[0], max(s.y - k, 0) >= y0 && min(s.y + k, G.dims[1] - 1) < y0 + w};
}

// Key of the row dy, dz away from the receiver: one multiply-add from the
// plane's base where every active lane's stencil is in its slab (LINEAR),
// row_key otherwise. The same key either way.
template <bool LINEAR>
__device__ __forceinline__ int stencil_row(const GeomDev& G, int plane_base, int dy, int y, int z) {
  return LINEAR ? plane_base + dy * G.dims[0] : row_key(G, y, z);
}

// Visit the source index ranges of the stencil of a receiver, culled to the
// cells within k cell edges (or within sqrt(kk) cell edges, kk <= k^2, for a
// receiver whose pairs reach less far: the multi-resolution force).
template <int K, bool LINEAR, class F>
__device__ __forceinline__ void for_each_row_keyed(const Stencil s, const GeomDev& G, const RowKeys rk,
                                                   const int* __restrict__ cs, F&& f, const float kk) {
#pragma unroll
  for (int dz = -K; dz <= K; ++dz) {
    const int z = s.z + dz;
    if (z < 0 || z >= G.dims[2]) continue;
    const float gz = cell_gap(dz, s.fz);
    const int pb = rk.base + dz * rk.zstep;
#pragma unroll
    for (int dy = -K; dy <= K; ++dy) {
      const int y = s.y + dy;
      if (y < 0 || y >= G.dims[1]) continue;
      const float gy = cell_gap(dy, s.fy);
      const float r2 = kk - (gy * gy + gz * gz);
      if (!(r2 > 0.0f)) continue;
      const float rho = __builtin_amdgcn_sqrtf(r2) * float(kXSplit);   // in x-cell edges
      const int below = min(K * kXSplit, int(ceilf(rho - s.fx + 1.0f)) - 1);   // |dx| with f + |dx| - 1 < rho
      const int above = min(K * kXSplit, int(ceilf(rho + s.fx)) - 1);          // dx with dx - f < rho
      const int x0 = max(s.x - below, 0), x1 = min(s.x + above, G.dims[0] - 1);
      const int row = stencil_row<LINEAR>(G, pb, dy, y, z);
      f(cs[row + x0], cs[row + x1 + 1]);
    }
  }
}

template <int K, class F>
__device__ __forceinline__ void for_each_row(const Stencil s, const GeomDev& G, const int* __restrict__ cs, F&& f,
                                             const float kk = float(K * K)) {
  const RowKeys rk = row_keys(s, G, K);
  if (__ballot(!rk.linear) == 0) for_each_row_keyed<K, true>(s, G, rk, cs, f, kk);
  else for_each_row_keyed<K, false>(s, G, rk, cs, f, kk);
}

// As for_each_row, with the bounds of the five (2k+1) rows of a dz plane
// loaded together before the plane's rows are walked, so that their loads
// overlap (four more registers; used where the occupancy allows it).
template <int K, bool LINEAR, class F>
__device__ __forceinline__ void for_each_row_by_plane_keyed(const Stencil s, const GeomDev& G, const RowKeys rk,
                                                            const int* __restrict__ cs, F&& f, const float kk) {
#pragma unroll
  for (int dz = -K; dz <= K; ++dz) {
    const int z = s.z + dz;
    if (z < 0 || z >= G.dims[2]) continue;
    const float gz = cell_gap(dz, s.fz);
    const int pb = rk.base + dz * rk.zstep;
    int j0[2 * K + 1], j1[2 * K + 1];
#pragma unroll
    for (int dy = -K; dy <= K; ++dy) {
      j0[dy + K] = j1[dy + K] = 0;   // an empty range: a row outside the grid or culled
      const int y = s.y + dy;
      if (y < 0 || y >= G.dims[1]) continue;
      const float gy = cell_gap(dy, s.fy);
      const float r2 = kk - (gy * gy + gz * gz);
      if (!(r2 > 0.0f)) continue;
      const float rho = __builtin_amdgcn_sqrtf(r2) * float(kXSplit);
      const int below = min(K * kXSplit, int(ceilf(rho - s.fx + 1.0f)) - 1);
      const int above = min(K * kXSplit, int(ceilf(rho + s.fx)) - 1);
      const int x0 = max(s.x - below, 0), x1 = min(s.x + above, G.dims[0] - 1);
      const int row = stencil_row<LINEAR>(G, pb, dy, y, z);
      j0[dy + K] = cs[row + x0];
      j1[dy + K] = cs[row + x1 + 1];
    }
#pragma unroll
    for (int q = 0; q < 2 * K + 1; ++q) f(j0[q], j1[q]);
  }
}

template <int K, class F>
__device__ __forceinline__ void for_each_row_by_plane(const Stencil s, const GeomDev& G, const int* __restrict__ cs,
                                                      F&& f, const float kk = float(K * K)) {
  const RowKeys rk = row_keys(s, G, K);
  if (__ballot(!rk.linear) == 0) for_each_row_by_plane_keyed<K, true>(s, G, rk, cs, f, kk);
  else for_each_row_by_plane_keyed<K, false>(s, G, rk, cs, f, kk);
}

// Visit every source index of the stencil, two loads in flight at a time.
// The lanes of a wavefront run a row for as long as its longest lane needs;
// pairs leave at most one step of tail per row (measured faster than groups
// of four, whose tail of up to three single steps per row costs more than the
// extra loads in flight gain, and than groups of three or single steps).
// PLANES: walk the rows with for_each_row_by_plane (same order, same sums).
// The walk advances a pointer (the loop costs one add and one compare per two
// candidates); the index j passed to f is only formed where f uses it.
template <int K, bool PLANES = false, class F>
__device__ __forceinline__ void for_each_source(const Stencil s, const GeomDev& G, const int* __restrict__ cs,
                                                const float4* __restrict__ pos, F&& f,
                                                const float kk = float(K * K)) {
  auto row = [&](int j0, int j1) {
    const float4* q = pos + j0;
    const float4* const e = pos + j1;
    // a pair remains while q < e - 1; that bound is formed from the address
    // (device addresses are far above one float4), not by pointer arithmetic
    const float4* const last = reinterpret_cast<const float4*>(reinterpret_cast<uintptr_t>(e) - sizeof(float4));
    for (; q < last; q += 2) {
      const float4 q0 = q[0], q1 = q[1];
      f(int(q - pos), q0);
      f(int(q - pos) + 1, q1);
    }
    if (q < e) f(int(q - pos), q[0]);
  };
  if (PLANES)
    for_each_row_by_plane<K>(s, G, cs, row, kk);
  else
    for_each_row<K>(s, G, cs, row, kk);
}

// As for_each_source, also loading row j of a second float4 field with the
// position, so that its latency overlaps the pair test (Jacobian products).
template <int K, class F>
__device__ __forceinline__ void for_each_source_with(const Stencil s, const GeomDev& G, const int* __restrict__ cs,
                                                     const float4* __restrict__ pos,
                                                     const float4* __restrict__ aux, F&& f) {
  for_each_row<K>(s, G, cs, [&](int j0, int j1) {
    // byte offsets from the row start, shared by the two fields
    const float4* q = pos + j0;
    const float4* w = aux + j0;
    const int n = j1 - j0;
    int k = 0;
    for (; k + 1 < n; k += 2) {
      const float4 q0 = q[k], q1 = q[k + 1];
      const float4 a0 = w[k], a1 = w[k + 1];
      f(j0 + k, q0, a0);
      f(j0 + k + 1, q1, a1);
    }
    if (k < n) f(j0 + k, q[k], w[k]);
  });
}

__device__ __forceinline__ float pair_d2(float dx, float dy, float dz) {
  return (dx * dx + dy * dy) + dz * dz;   // no contraction in this file
}

}  // namespace fppg

// Facet search grid lookups shared by the projection and the volume layer
// split: cell coordinates of a point and the global index of a search cell.
#pragma once

#include "internal.h"

namespace fppg {

// Search-cell coordinate of y in cell units, clamped to the grid.
__device__ __forceinline__ double search_t(const GeomDev& G, int a, double y) {
  return fmin(fmax((y - G.tg_origin[a]) * G.tg_inv, 0.0), double(G.tg_dims[a] - 1));
}

__device__ __forceinline__ int64_t search_index(const GeomDev& G, int x, int y, int z) {
  return G.tg_begin + (int64_t(z) * G.tg_dims[1] + y) * G.tg_dims[0] + x;
}

}  // namespace fppg

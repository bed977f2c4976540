// Three-layer volume relaxation (section 3.3.4): beneath the surface
// particles, the volume particles closer to the surface than a width W form the
// intermediate layer, which relaxes; the others form the innermost core, which
// stays where it is and acts as a source. fppg_volume_layers re-tags the core
// as fixed particles, once, before the volume relaxation.
//
// Distance: the exact point-triangle distance in FP64 (closest point by the
// Voronoi regions of the triangle, Ericson, Real-Time Collision Detection,
// 2005, section 5.1.5) to the facets registered in the search cells that the
// box [x - W, x + W] touches: a facet closer than W has a point in that box,
// and a facet is registered in every search cell it touches.
#include "search_grid.h"

namespace fppg {

__device__ __forceinline__ double dot3(double ax, double ay, double az, double bx, double by, double bz) {
  return (ax * bx + ay * by) + az * bz;
}

// Squared distance from p to the triangle (A, A + e0, A + e1).
__device__ double facet_dist2(const FacetDev& F, double px, double py, double pz) {
  const double abx = F.e0[0], aby = F.e0[1], abz = F.e0[2];
  const double acx = F.e1[0], acy = F.e1[1], acz = F.e1[2];
  const double apx = px - F.a[0], apy = py - F.a[1], apz = pz - F.a[2];
  const double d1 = dot3(abx, aby, abz, apx, apy, apz), d2 = dot3(acx, acy, acz, apx, apy, apz);
  if (d1 <= 0.0 && d2 <= 0.0) return dot3(apx, apy, apz, apx, apy, apz);          // vertex A
  const double bpx = apx - abx, bpy = apy - aby, bpz = apz - abz;
  const double d3 = dot3(abx, aby, abz, bpx, bpy, bpz), d4 = dot3(acx, acy, acz, bpx, bpy, bpz);
  if (d3 >= 0.0 && d4 <= d3) return dot3(bpx, bpy, bpz, bpx, bpy, bpz);           // vertex B
  const double vc = d1 * d4 - d3 * d2;
  double rx, ry, rz;   // p minus its closest point
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {                                     // edge AB
    const double v = d1 / (d1 - d3);
    rx = apx - v * abx, ry = apy - v * aby, rz = apz - v * abz;
    return dot3(rx, ry, rz, rx, ry, rz);
  }
  const double cpx = apx - acx, cpy = apy - acy, cpz = apz - acz;
  const double d5 = dot3(abx, aby, abz, cpx, cpy, cpz), d6 = dot3(acx, acy, acz, cpx, cpy, cpz);
  if (d6 >= 0.0 && d5 <= d6) return dot3(cpx, cpy, cpz, cpx, cpy, cpz);           // vertex C
  const double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {                                     // edge AC
    const double w = d2 / (d2 - d6);
    rx = apx - w * acx, ry = apy - w * acy, rz = apz - w * acz;
    return dot3(rx, ry, rz, rx, ry, rz);
  }
  const double va = d3 * d6 - d5 * d4;
  if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {                       // edge BC
    const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    rx = bpx - w * (acx - abx), ry = bpy - w * (acy - aby), rz = bpz - w * (acz - abz);
    return dot3(rx, ry, rz, rx, ry, rz);
  }
  const double den = 1.0 / (va + vb + vc);                                        // interior
  const double v = vb * den, w = vc * den;
  rx = apx - v * abx - w * acx, ry = apy - v * aby - w * acy, rz = apz - v * abz - w * acz;
  return dot3(rx, ry, rz, rx, ry, rz);
}

// Is a facet of the search cells around p closer than w (w2 = w * w)?
__device__ bool near_surface(const GeomDev& G, double px, double py, double pz, double w, double w2,
                             const FacetDev* __restrict__ facets, const int* __restrict__ tstart,
                             const int* __restrict__ ttri, const uint8_t* __restrict__ tflag) {
  const double pad = 1e-7;   // cell units
  const int lx = int(floor(search_t(G, 0, px - w) - pad)), hx = int(floor(search_t(G, 0, px + w) + pad));
  const int ly = int(floor(search_t(G, 1, py - w) - pad)), hy = int(floor(search_t(G, 1, py + w) + pad));
  const int lz = int(floor(search_t(G, 2, pz - w) - pad)), hz = int(floor(search_t(G, 2, pz + w) + pad));
  for (int z = max(lz, 0); z <= min(hz, G.tg_dims[2] - 1); ++z)
    for (int y = max(ly, 0); y <= min(hy, G.tg_dims[1] - 1); ++y)
      for (int x = max(lx, 0); x <= min(hx, G.tg_dims[0] - 1); ++x) {
        const int64_t c = search_index(G, x, y, z);
        if (!(tflag[c] & kCellHasFacet)) continue;
        for (int q = tstart[c]; q < tstart[c + 1]; ++q)
          if (facet_dist2(facets[ttri[q]], px, py, pz) < w2) return true;
      }
  return false;
}

__global__ __launch_bounds__(kBlock) void k_volume_layers(float4* __restrict__ pos, int n, double w,
                                                          const GeomDev* __restrict__ geoms, int n_geom,
                                                          const FacetDev* __restrict__ facets,
                                                          const int* __restrict__ tstart,
                                                          const int* __restrict__ ttri,
                                                          const uint8_t* __restrict__ tflag, int* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool core = false;
  if (i < n) {
    const float4 p = pos[i];
    if (tag_of(p.w) == FPPG_TAG_VOLUME && isfinite(p.x) && isfinite(p.y) && isfinite(p.z)) {
      const GeomDev& G = geoms[min(geom_of(p.w), n_geom - 1)];
      core = !near_surface(G, double(p.x), double(p.y), double(p.z), w, w * w, facets, tstart, ttri, tflag);
      if (core) pos[i].w = __int_as_float((__float_as_int(p.w) & ~7) | FPPG_TAG_FIXED);
    }
  }
  const uint64_t m = __ballot(core);
  if (m && (threadIdx.x & 63) == 0) atomicAdd(count, int(__popcll(m)));
}

__global__ void k_zero_i32(int* __restrict__ c) {
  if (threadIdx.x == 0) *c = 0;
}

}  // namespace fppg

using namespace fppg;

extern "C" fppg_status fppg_volume_layers(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, float* pos, double width,
                                          int32_t* count, void* stream) {
  if (!ctx || !geom) return fail(ctx, FPPG_E_ARG, "null ctx/geom");
  if (n != geom->n_active) return fail(ctx, FPPG_E_ARG, "n differs from the active particle count of the geometry");
  if (!count || (n > 0 && !pos)) return fail(ctx, FPPG_E_ARG, "null pos/count");
  if (!aligned(pos, 16)) return fail(ctx, FPPG_E_ARG, "pos must be 16-byte aligned");
  if (!(width >= 0.0) || !std::isfinite(width)) return fail(ctx, FPPG_E_ARG, "width must be finite and >= 0");
  if (geom->has_csg)   // the distance to all facets includes the parts' faces inside the assembly
    return fail(ctx, FPPG_E_UNSUPPORTED, "volume layers of a Boolean assembly are not supported");
  hipStream_t s = static_cast<hipStream_t>(stream);
  k_zero_i32<<<1, 64, 0, s>>>(count);
  if (n > 0)
    k_volume_layers<<<int((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        reinterpret_cast<float4*>(pos), int(n), width, geom->d_geom, geom->n_geom, geom->d_facet, geom->d_tg_start,
        geom->d_tg_tri, geom->d_tg_flag, count);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

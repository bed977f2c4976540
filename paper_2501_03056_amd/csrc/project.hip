// Projection back onto the explicit geometry (section 3.3.3 and 3.3.4).
//
//   k_sort_out   one pass over all particles: volume particles away from the
//                surface (no facet in the 27 search cells around the new
//                position) move directly; surface, feature and near-surface
//                volume particles are appended to three compact worklists
//                (one atomic per wavefront and list)
//   k_surface    FP64 reprojection onto the nearest accepting facet among the
//                27 search cells, revert when none accepts
//   k_feature    FP64 arc-length walk along the feature polyline
//   k_volume     FP64 test of the step segment against the nearby facets;
//                a crossing reverts the move
// The worklist kernels are grid-stride loops over a device-side count, so the
// launch shapes do not depend on the data.
#include "internal.h"

namespace fppg {

constexpr int kListBlocks = 1024;

__device__ __forceinline__ void search_cell(const GeomDev& G, double x, double y, double z, int& cx, int& cy, int& cz) {
  const double tx = (x - G.tg_origin[0]) * G.tg_inv;
  const double ty = (y - G.tg_origin[1]) * G.tg_inv;
  const double tz = (z - G.tg_origin[2]) * G.tg_inv;
  cx = int(floor(fmin(fmax(tx, 0.0), double(G.tg_dims[0] - 1))));
  cy = int(floor(fmin(fmax(ty, 0.0), double(G.tg_dims[1] - 1))));
  cz = int(floor(fmin(fmax(tz, 0.0), double(G.tg_dims[2] - 1))));
}

// Visit the facet lists of the 27 search cells around (cx, cy, cz).
template <class F>
__device__ __forceinline__ void for_each_facet27(const GeomDev& G, int cx, int cy, int cz,
                                                 const int* __restrict__ tstart, const int* __restrict__ ttri, F&& f) {
  for (int dz = -1; dz <= 1; ++dz) {
    const int z = cz + dz;
    if (z < 0 || z >= G.tg_dims[2]) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = cy + dy;
      if (y < 0 || y >= G.tg_dims[1]) continue;
      const int64_t row = G.tg_begin + (int64_t(z) * G.tg_dims[1] + y) * G.tg_dims[0];
      const int x0 = max(cx - 1, 0), x1 = min(cx + 1, G.tg_dims[0] - 1);
      const int b = tstart[row + x0], e = tstart[row + x1 + 1];
      for (int q = b; q < e; ++q) f(ttri[q]);
    }
  }
}

// Barycentric coordinates of a point already on the facet plane: min(la, lb, lc).
__device__ __forceinline__ double bary_min(const FacetDev& F, double px, double py, double pz) {
  const double vx = px - F.a[0], vy = py - F.a[1], vz = pz - F.a[2];
  const double d20 = vx * F.e0[0] + vy * F.e0[1] + vz * F.e0[2];
  const double d21 = vx * F.e1[0] + vy * F.e1[1] + vz * F.e1[2];
  const double lb = (F.d11 * d20 - F.d01 * d21) * F.inv_den;
  const double lc = (F.d00 * d21 - F.d01 * d20) * F.inv_den;
  const double la = 1.0 - lb - lc;
  return fmin(la, fmin(lb, lc));
}

__device__ __forceinline__ void wave_append(bool want, int i, int* __restrict__ list, int* __restrict__ counter) {
  const uint64_t m = __ballot(want);
  if (m == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, __popcll(m));
  base = __shfl(base, leader);
  if (want) list[base + __popcll(m & ((1ull << lane) - 1))] = i;
}

// Add the number of lanes with `pred` to a counter: one atomic per wavefront.
// Called where every active lane of the wavefront takes part.
__device__ __forceinline__ void wave_count(bool pred, unsigned long long* __restrict__ ctr) {
  const uint64_t active = __ballot(1);
  const uint64_t m = __ballot(pred);
  if (m && (threadIdx.x & 63) == __ffsll((long long)active) - 1) atomicAdd(ctr, (unsigned long long)__popcll(m));
}

__global__ void k_zero_counts(int* __restrict__ c) {
  if (threadIdx.x < 16) c[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kBlock) void k_sort_out(float4* __restrict__ pos, const float4* __restrict__ disp, int n,
                                                     const GeomDev* __restrict__ geoms, int n_geom,
                                                     const uint8_t* __restrict__ tflag, uint32_t move_mask,
                                                     int* __restrict__ lists, int* __restrict__ counts, int nlist,
                                                     uint32_t* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool to_surf = false, to_feat = false, to_vol = false;
  if (i < n) {
    const float4 p = pos[i];
    const int tag = tag_of(p.w);
    if (is_moving(tag, move_mask)) {
      if (tag == FPPG_TAG_SURFACE) {
        to_surf = true;
      } else if (tag == FPPG_TAG_FEATURE) {
        to_feat = true;
      } else {
        const float4 d = disp[i];
        const float yx = p.x + d.x, yy = p.y + d.y, yz = p.z + d.z;
        if (!(isfinite(yx) && isfinite(yy) && isfinite(yz))) {
          atomicOr(status, FPPG_S_NONFINITE_POS);
        } else {
          const GeomDev& G = geoms[min(geom_of(p.w), n_geom - 1)];
          int cx, cy, cz;
          search_cell(G, yx, yy, yz, cx, cy, cz);
          const int64_t c = G.tg_begin + (int64_t(cz) * G.tg_dims[1] + cy) * G.tg_dims[0] + cx;
          if (tflag[c] & kCellNearSurface) to_vol = true;
          else pos[i] = make_float4(yx, yy, yz, p.w);
        }
      }
    }
  }
  wave_append(to_surf, i, lists, counts + 0);
  wave_append(to_feat, i, lists + nlist, counts + 1);
  wave_append(to_vol, i, lists + 2 * nlist, counts + 2);
}

__global__ __launch_bounds__(kBlock) void k_surface(float4* __restrict__ pos, int* __restrict__ owner,
                                                    const float4* __restrict__ disp, const GeomDev* __restrict__ geoms,
                                                    int n_geom, const FacetDev* __restrict__ facets,
                                                    const int* __restrict__ tstart, const int* __restrict__ ttri,
                                                    const int* __restrict__ list, const int* __restrict__ counts,
                                                    unsigned long long* __restrict__ counters, uint32_t* status) {
  const int cnt = counts[0];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < cnt; k += gridDim.x * blockDim.x) {
    const int i = list[k];
    const float4 p = pos[i];
    const float4 d = disp[i];
    const GeomDev& G = geoms[min(geom_of(p.w), n_geom - 1)];
    const double yx = double(p.x) + double(d.x), yy = double(p.y) + double(d.y), yz = double(p.z) + double(d.z);
    const double R = G.R;
    double best = INFINITY, bx = 0.0, by = 0.0, bz = 0.0;
    int bt = 0x7fffffff;
    if (isfinite(yx) && isfinite(yy) && isfinite(yz)) {
      int cx, cy, cz;
      search_cell(G, yx, yy, yz, cx, cy, cz);
      for_each_facet27(G, cx, cy, cz, tstart, ttri, [&](int t) {
        const FacetDev& F = facets[t];
        const double dist = (yx - F.a[0]) * F.n[0] + (yy - F.a[1]) * F.n[1] + (yz - F.a[2]) * F.n[2];
        const double ad = fabs(dist);
        if (!(ad <= R) || ad > best || (ad == best && t >= bt)) return;
        const double px = yx - dist * F.n[0], py = yy - dist * F.n[1], pz = yz - dist * F.n[2];
        if (bary_min(F, px, py, pz) >= 0.0) {
          best = ad;
          bt = t;
          bx = px;
          by = py;
          bz = pz;
        }
      });
    } else {
      atomicOr(status, FPPG_S_NONFINITE_POS);
    }
    const bool found = bt != 0x7fffffff;
    if (found) {
      pos[i] = make_float4(float(bx), float(by), float(bz), p.w);
      owner[i] = bt;
    }                                       // else: stays at x (section 3.3.3)
    wave_count(found, &counters[FPPG_C_SURFACE_MOVED]);
    wave_count(!found, &counters[FPPG_C_REVERT_SURFACE]);
  }
}

__global__ __launch_bounds__(kBlock) void k_feature(float4* __restrict__ pos, const int* __restrict__ owner,
                                                    const float4* __restrict__ disp, int* __restrict__ feat_seg,
                                                    double* __restrict__ feat_u, int n_feat, int n_seg,
                                                    const SegDev* __restrict__ segs, const int* __restrict__ list,
                                                    const int* __restrict__ counts,
                                                    unsigned long long* __restrict__ counters, uint32_t* status) {
  const int cnt = counts[1];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < cnt; k += gridDim.x * blockDim.x) {
    const int i = list[k];
    const int slot = owner[i];
    int s = (slot >= 0 && slot < n_feat) ? feat_seg[slot] : -1;
    if (s < 0 || s >= n_seg) {
      atomicOr(status, FPPG_S_BAD_INDEX);   // particle held in place
      continue;
    }
    const float4 d = disp[i];
    const long long bits = (long long)(unsigned)__float_as_int(d.x) | ((long long)__float_as_int(d.y) << 32);
    double u = feat_u[slot] + __longlong_as_double(bits);
    bool ok = isfinite(u);
    // walk along the line; each pass moves one segment, a line has hi - lo segments
    for (int guard = segs[s].hi - segs[s].lo + 2; ok && guard > 0; --guard) {
      const SegDev S = segs[s];
      if (u < 0.0) {
        if (s > S.lo) {
          s -= 1;
          u += segs[s].len;
        } else if (S.closed) {
          s = S.hi - 1;
          u += segs[s].len;
        } else {
          ok = false;
        }
      } else if (u > S.len) {
        if (s < S.hi - 1) {
          u -= S.len;
          s += 1;
        } else if (S.closed) {
          u -= S.len;
          s = S.lo;
        } else {
          ok = false;
        }
      } else {
        break;
      }
    }
    if (ok && u >= 0.0 && u <= segs[s].len) {
      const SegDev S = segs[s];
      const float4 p = pos[i];
      pos[i] = make_float4(float(S.p0[0] + u * S.t[0]), float(S.p0[1] + u * S.t[1]), float(S.p0[2] + u * S.t[2]), p.w);
      feat_seg[slot] = s;
      feat_u[slot] = u;
    } else {
      if (!isfinite(u)) atomicOr(status, FPPG_S_NONFINITE_POS);
      atomicAdd(&counters[FPPG_C_REVERT_FEATURE], 1ull);   // rare: few feature particles
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_volume(float4* __restrict__ pos, const float4* __restrict__ disp,
                                                   const GeomDev* __restrict__ geoms, int n_geom,
                                                   const FacetDev* __restrict__ facets, const int* __restrict__ tstart,
                                                   const int* __restrict__ ttri, const int* __restrict__ list,
                                                   const int* __restrict__ counts,
                                                   unsigned long long* __restrict__ counters) {
  const int cnt = counts[2];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < cnt; k += gridDim.x * blockDim.x) {
    const int i = list[k];
    const float4 p = pos[i];
    const float4 d = disp[i];
    const float fy0 = p.x + d.x, fy1 = p.y + d.y, fy2 = p.z + d.z;   // same binary32 sums as k_sort_out
    const double x0 = p.x, x1 = p.y, x2 = p.z;
    const double y0 = fy0, y1 = fy1, y2 = fy2;
    const GeomDev& G = geoms[min(geom_of(p.w), n_geom - 1)];
    int cx, cy, cz;
    search_cell(G, y0, y1, y2, cx, cy, cz);
    bool crossed = false;
    for_each_facet27(G, cx, cy, cz, tstart, ttri, [&](int t) {
      if (crossed) return;
      const FacetDev& F = facets[t];
      const double sx = (x0 - F.a[0]) * F.n[0] + (x1 - F.a[1]) * F.n[1] + (x2 - F.a[2]) * F.n[2];
      const double sy = (y0 - F.a[0]) * F.n[0] + (y1 - F.a[1]) * F.n[1] + (y2 - F.a[2]) * F.n[2];
      if ((sx > 0.0 && sy > 0.0) || (sx < 0.0 && sy < 0.0)) return;   // segment on one side of the plane
      double px = y0, py = y1, pz = y2;
      if (sx != sy) {
        const double s = sx / (sx - sy);
        px = x0 + s * (y0 - x0);
        py = x1 + s * (y1 - x1);
        pz = x2 + s * (y2 - x2);
      }
      if (bary_min(F, px, py, pz) >= 0.0) crossed = true;
    });
    if (!crossed) pos[i] = make_float4(fy0, fy1, fy2, p.w);
    wave_count(true, &counters[FPPG_C_VOLUME_TESTED]);
    wave_count(crossed, &counters[FPPG_C_REVERT_VOLUME]);
  }
}

static inline int grid_for(int64_t n) { return int((n + kBlock - 1) / kBlock); }

}  // namespace fppg

using namespace fppg;

extern "C" fppg_status fppg_project(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, float* pos, int32_t* owner,
                                    const float* disp, int32_t* feat_seg, double* feat_u, int32_t n_feat,
                                    uint32_t move_mask, int64_t* counters, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !geom) return fail(ctx, FPPG_E_ARG, "null ctx/geom");
  if (n != geom->n_part) return fail(ctx, FPPG_E_ARG, "n differs from the particle count of the geometry descriptors");
  if (n > 0 && (!pos || !owner || !disp)) return fail(ctx, FPPG_E_ARG, "null pos/owner/disp");
  if (n_feat < 0 || (n_feat > 0 && (!feat_seg || !feat_u))) return fail(ctx, FPPG_E_ARG, "bad feature table");
  if (!aligned(pos, 16) || !aligned(disp, 16) || !ws || !aligned(ws, 256))
    return fail(ctx, FPPG_E_ARG, "pos/disp must be 16-byte aligned, ws non-null and 256-byte aligned");
  if (!counters) return fail(ctx, FPPG_E_ARG, "null counters");
  const WsLayout L = ws_layout(geom, n);
  if (ws_bytes < L.project_end) return fail(ctx, FPPG_E_WORKSPACE, "workspace too small for project");
  if (n == 0) return FPPG_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  int* lists = reinterpret_cast<int*>(w + L.list_surf);
  const int nlist = int((L.list_feat - L.list_surf) / 4);
  int* cnt = reinterpret_cast<int*>(w + L.list_count);
  unsigned long long* ctr = reinterpret_cast<unsigned long long*>(counters);
  const int ni = int(n);
  float4* p4 = reinterpret_cast<float4*>(pos);
  const float4* d4 = reinterpret_cast<const float4*>(disp);
  PhaseTimer timer(ctx, 3, s);
  k_zero_counts<<<1, 64, 0, s>>>(cnt);
  k_sort_out<<<grid_for(ni), kBlock, 0, s>>>(p4, d4, ni, geom->d_geom, geom->n_geom, geom->d_tg_flag, move_mask, lists,
                                             cnt, nlist, ctx->d_status);
  k_surface<<<kListBlocks, kBlock, 0, s>>>(p4, owner, d4, geom->d_geom, geom->n_geom, geom->d_facet, geom->d_tg_start,
                                           geom->d_tg_tri, lists, cnt, ctr, ctx->d_status);
  k_feature<<<64, kBlock, 0, s>>>(p4, owner, d4, feat_seg, feat_u, n_feat, int(geom->n_seg), geom->d_seg,
                                  lists + nlist, cnt, ctr, ctx->d_status);
  k_volume<<<kListBlocks, kBlock, 0, s>>>(p4, d4, geom->d_geom, geom->n_geom, geom->d_facet, geom->d_tg_start,
                                          geom->d_tg_tri, lists + 2 * nlist, cnt, ctr);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

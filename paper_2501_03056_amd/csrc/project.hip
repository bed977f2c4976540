// Projection back onto the explicit geometry (section 3.3.3 and 3.3.4), one
// lane per particle in two kernels (volume particles in a lean streaming pass
// that queues the others; surface and feature particles from that queue):
//
//   surface  y = x + dr in FP64; facet search over the search cells in the
//            order of the paper's reprojection: the particle's own cell
//            first, then a neighbouring cell only if its box is within the
//            best accepted plane distance so far (an accepted foot point lies
//            within |d| of y, so every skipped cell is provably unable to hold
//            a better or equal candidate: the result is the argmin over the
//            27 cells). Accept: all barycentric >= 0 and |d| <= R; smallest |d|
//            wins, ties -> lowest facet; none -> revert to x.
//   feature  FP64 arc-length walk along the feature polyline.
//   volume   y = fl32(x + dr); the move is reverted iff the segment [x, y]
//            meets a facet registered in a search cell that the segment's
//            bounding box touches (padded by 1e-7 cell). Away from the
//            surface those cells hold no facet and the move is accepted after
//            one byte of flags.
// Boolean assemblies (section 3.2.3): a foot point, and the point where a
// volume move crosses a facet, count only on the assembly's boundary (FP64
// plane tests of the convex parts): a move across a part's face that lies
// inside the assembly is accepted.
// Reverts are counted per block and added to the caller's counters by one
// small kernel.
#include "search_grid.h"

#include <algorithm>

namespace fppg {

// Barycentric coordinates of a point on the facet plane: min(la, lb, lc).
__device__ __forceinline__ double bary_min(const FacetDev& F, double px, double py, double pz) {
  const double vx = px - F.a[0], vy = py - F.a[1], vz = pz - F.a[2];
  const double d20 = vx * F.e0[0] + vy * F.e0[1] + vz * F.e0[2];
  const double d21 = vx * F.e1[0] + vy * F.e1[1] + vz * F.e1[2];
  const double lb = (F.d11 * d20 - F.d01 * d21) * F.inv_den;
  const double lc = (F.d00 * d21 - F.d01 * d20) * F.inv_den;
  const double la = 1.0 - lb - lc;
  return fmin(la, fmin(lb, lc));
}

__device__ __forceinline__ double gap1(int d, double f) {
  return d > 0 ? double(d) - f : (d < 0 ? f + double(-d - 1) : 0.0);
}

// ---- Boolean assemblies (section 3.2.3) ----------------------------------------------------
// Plane tests of the convex parts in FP64 (n.x - d per plane). A point
// outside a part's bounding box is outside the part; otherwise the planes are
// read eight at a time, so that their loads overlap, and the test stops after
// the first batch that decides it.
template <bool CLOSED>
__device__ __forceinline__ bool in_part(const CsgDev& cs, int k, double x, double y, double z) {
  const PartDev& P = cs.part[k];
  if (x < P.lo[0] || x > P.hi[0] || y < P.lo[1] || y > P.hi[1] || z < P.lo[2] || z > P.hi[2]) return false;
  for (int j = P.plane_begin; j < P.plane_end; j += 8) {
    bool out = false;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (j + u < P.plane_end) {
        const double4 Q = cs.plane[j + u];
        const double v = Q.x * x + Q.y * y + Q.z * z - Q.w;
        out |= CLOSED ? (v > 0.0) : (v >= 0.0);
      }
    }
    if (out) return false;
  }
  return true;
}

__device__ __forceinline__ bool in_part_open(const CsgDev& cs, int k, double x, double y, double z) {
  return in_part<false>(cs, k, x, y, z);
}

__device__ __forceinline__ bool in_part_closed(const CsgDev& cs, int k, double x, double y, double z) {
  return in_part<true>(cs, k, x, y, z);
}

// Is a point of facet t (part k) on the assembly's boundary? Only the parts
// the facet crosses are tested: the facet lies wholly outside (or, for part 0
// of a difference, wholly inside) every other part it must avoid.
__device__ __forceinline__ bool csg_on_boundary(const GeomDev& G, const CsgDev& cs, int t, int k, double x, double y,
                                                double z) {
  const int base = G.part_begin_csg;
  for (uint32_t m = cs.facet_mask[t]; m; m &= m - 1) {
    const int j = base + __ffs(int(m)) - 1;
    if (G.csg_op == FPPG_CSG_DIFFERENCE && j == base && k != base) {
      if (!in_part_closed(cs, j, x, y, z)) return false;   // a cut face counts inside part 0
    } else if (in_part_open(cs, j, x, y, z)) {
      return false;
    }
  }
  return true;
}

struct SurfaceHit {
  double best = INFINITY, x = 0.0, y = 0.0, z = 0.0;
  int t = 0x7fffffff;
};

__device__ __forceinline__ void scan_surface_cell(int64_t c, double yx, double yy, double yz, double R,
                                                  const FacetDev* __restrict__ facets, const int* __restrict__ tstart,
                                                  const int* __restrict__ ttri, SurfaceHit& h, const GeomDev& G,
                                                  const CsgDev& cs) {
  const int b = tstart[c], e = tstart[c + 1];
  for (int q = b; q < e; ++q) {
    const int t = ttri[q];
    const FacetDev& F = facets[t];
    const double dist = (yx - F.a[0]) * F.n[0] + (yy - F.a[1]) * F.n[1] + (yz - F.a[2]) * F.n[2];
    const double ad = fabs(dist);
    if (!(ad <= R) || ad > h.best || (ad == h.best && t >= h.t)) continue;
    const double px = yx - dist * F.n[0], py = yy - dist * F.n[1], pz = yz - dist * F.n[2];
    if (bary_min(F, px, py, pz) >= 0.0 && (G.csg_op == FPPG_CSG_NONE || cs.facet_part[t] < 0 ||
                                           csg_on_boundary(G, cs, t, cs.facet_part[t], px, py, pz))) {
      h.best = ad;
      h.t = t;
      h.x = px;
      h.y = py;
      h.z = pz;
    }
  }
}

// The search from the own cell. If the own cell accepts no facet, *wide is
// set and the caller hands the particle to the parallel search over all 27
// cells (k_project_wide) instead of scanning the neighbours one by one here.
__device__ __forceinline__ SurfaceHit surface_search(const GeomDev& G, double yx, double yy, double yz,
                                                     const FacetDev* __restrict__ facets,
                                                     const int* __restrict__ tstart, const int* __restrict__ ttri,
                                                     const uint8_t* __restrict__ tflag, const CsgDev& cs, bool* wide) {
  SurfaceHit h;
  const double R = G.R;
  const double tx = search_t(G, 0, yx), ty = search_t(G, 1, yy), tz = search_t(G, 2, yz);
  const int cx = int(floor(tx)), cy = int(floor(ty)), cz = int(floor(tz));
  const double fx = tx - cx, fy = ty - cy, fz = tz - cz;
  const int64_t c0 = search_index(G, cx, cy, cz);
  if (tflag[c0] & kCellHasFacet) scan_surface_cell(c0, yx, yy, yz, R, facets, tstart, ttri, h, G, cs);
  *wide = h.t == 0x7fffffff;
  if (*wide) return h;
  const double slack = 1e-7;   // cell units, covers the rounding of the gaps
  for (int dz = -1; dz <= 1; ++dz) {
    const int z = cz + dz;
    if (z < 0 || z >= G.tg_dims[2]) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = cy + dy;
      if (y < 0 || y >= G.tg_dims[1]) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int x = cx + dx;
        if ((dx | dy | dz) == 0 || x < 0 || x >= G.tg_dims[0]) continue;
        const double gx = gap1(dx, fx), gy = gap1(dy, fy), gz = gap1(dz, fz);
        const double lim = fmin(h.best, R) * G.tg_inv + slack;   // the cell must come within |d| of y
        if (gx * gx + gy * gy + gz * gz > lim * lim) continue;
        const int64_t c = search_index(G, x, y, z);
        if (tflag[c] & kCellHasFacet) scan_surface_cell(c, yx, yy, yz, R, facets, tstart, ttri, h, G, cs);
      }
    }
  }
  return h;
}

// Does the segment [x, y] meet a facet registered in cell c (for an
// assembly: at a point of the assembly's boundary)?
__device__ __forceinline__ bool cell_crossed(int64_t c, double x0, double x1, double x2, double y0, double y1, double y2,
                                             const FacetDev* __restrict__ facets, const int* __restrict__ tstart,
                                             const int* __restrict__ ttri, const GeomDev& G, const CsgDev& cs) {
  const int b = tstart[c], e = tstart[c + 1];
  for (int q = b; q < e; ++q) {
    const int t = ttri[q];
    const FacetDev& F = facets[t];
    const double sx = (x0 - F.a[0]) * F.n[0] + (x1 - F.a[1]) * F.n[1] + (x2 - F.a[2]) * F.n[2];
    const double sy = (y0 - F.a[0]) * F.n[0] + (y1 - F.a[1]) * F.n[1] + (y2 - F.a[2]) * F.n[2];
    if ((sx > 0.0 && sy > 0.0) || (sx < 0.0 && sy < 0.0)) continue;   // both ends on one side of the plane
    double px = y0, py = y1, pz = y2;
    if (sx != sy) {
      const double s = sx / (sx - sy);
      px = x0 + s * (y0 - x0);
      py = x1 + s * (y1 - x1);
      pz = x2 + s * (y2 - x2);
    }
    if (bary_min(F, px, py, pz) >= 0.0 &&
        (G.csg_op == FPPG_CSG_NONE || cs.facet_part[t] < 0 || csg_on_boundary(G, cs, t, cs.facet_part[t], px, py, pz)))
      return true;
  }
  return false;
}

// The search cells of the segment's box, widened by 1e-7 cell units and
// clipped to the grid: [lo, hi] per axis (empty where lo > hi).
__device__ __forceinline__ void segment_cells(const GeomDev& G, double x0, double x1, double x2, double y0, double y1,
                                              double y2, int lo[3], int hi[3]) {
  const double pad = 1e-7;   // cell units
  lo[0] = max(int(floor(search_t(G, 0, fmin(x0, y0)) - pad)), 0);
  hi[0] = min(int(floor(search_t(G, 0, fmax(x0, y0)) + pad)), G.tg_dims[0] - 1);
  lo[1] = max(int(floor(search_t(G, 1, fmin(x1, y1)) - pad)), 0);
  hi[1] = min(int(floor(search_t(G, 1, fmax(x1, y1)) + pad)), G.tg_dims[1] - 1);
  lo[2] = max(int(floor(search_t(G, 2, fmin(x2, y2)) - pad)), 0);
  hi[2] = min(int(floor(search_t(G, 2, fmax(x2, y2)) + pad)), G.tg_dims[2] - 1);
}

__device__ __forceinline__ bool segment_crosses(const GeomDev& G, double x0, double x1, double x2, double y0,
                                                double y1, double y2, const FacetDev* __restrict__ facets,
                                                const int* __restrict__ tstart, const int* __restrict__ ttri,
                                                const uint8_t* __restrict__ tflag, const CsgDev& cs) {
  int lo[3], hi[3];
  segment_cells(G, x0, x1, x2, y0, y1, y2, lo, hi);
  for (int z = lo[2]; z <= hi[2]; ++z)
    for (int y = lo[1]; y <= hi[1]; ++y)
      for (int x = lo[0]; x <= hi[0]; ++x) {
        const int64_t c = search_index(G, x, y, z);
        if ((tflag[c] & kCellHasFacet) && cell_crossed(c, x0, x1, x2, y0, y1, y2, facets, tstart, ttri, G, cs))
          return true;
      }
  return false;
}

// Does the segment's box touch a search cell with registered facets? If not,
// segment_crosses is false without a facet test.
__device__ __forceinline__ bool segment_near_facets(const GeomDev& G, double x0, double x1, double x2, double y0,
                                                    double y1, double y2, const uint8_t* __restrict__ tflag) {
  int lo[3], hi[3];
  segment_cells(G, x0, x1, x2, y0, y1, y2, lo, hi);
  for (int z = lo[2]; z <= hi[2]; ++z)
    for (int y = lo[1]; y <= hi[1]; ++y)
      for (int x = lo[0]; x <= hi[0]; ++x)
        if (tflag[search_index(G, x, y, z)] & kCellHasFacet) return true;
  return false;
}

// Arc-length walk of a feature particle; returns false if it leaves an open line.
__device__ __forceinline__ bool feature_walk(const SegDev* __restrict__ segs, int& s, double& u) {
  if (!isfinite(u)) return false;
  for (int guard = segs[s].hi - segs[s].lo + 2; guard > 0; --guard) {
    const SegDev S = segs[s];
    if (u < 0.0) {
      if (s > S.lo) {
        s -= 1;
        u += segs[s].len;
      } else if (S.closed) {
        s = S.hi - 1;
        u += segs[s].len;
      } else {
        return false;
      }
    } else if (u > S.len) {
      if (s < S.hi - 1) {
        u -= S.len;
        s += 1;
      } else if (S.closed) {
        u -= S.len;
        s = S.lo;
      } else {
        return false;
      }
    } else {
      return true;
    }
  }
  return u >= 0.0 && u <= segs[s].len;
}

// Volume particles (and the class dispatch) in a lean kernel: a volume move
// whose box touches no search cell with facets is applied at once (it cannot
// cross the surface); surface and feature particles, and volume moves next to
// facets, whose FP64 tests need several times the registers, go to a queue
// that k_project_heavy takes: the streaming volume pass keeps a high
// occupancy. Each block of the volume pass compacts its queued particles
// (its volume moves, then the others, each in index order) into its own
// kBlock slots of the queue and stores their
// number: no atomics, and the queue is the same on every run.
// ONE_GEOM: a single geometry, whose descriptor is then read with scalar loads
// that do not wait for the particle's position.
template <bool ONE_GEOM>
__global__ __launch_bounds__(kBlock) void k_project_volume(float4* __restrict__ pos, const float4* __restrict__ disp,
                                                           int n, const GeomDev* __restrict__ geoms, int n_geom,
                                                           const uint8_t* __restrict__ tflag, uint32_t move_mask,
                                                           uint32_t* status, uint8_t* __restrict__ accepted,
                                                           const int* __restrict__ list, int n_list,
                                                           int* __restrict__ queue, int* __restrict__ qcount,
                                                           int* __restrict__ hard) {
  if (blockIdx.x == 0 && threadIdx.x == 0) hard[0] = 0;   // the wide-search queue of this projection
  const int i = listed(blockIdx.x * blockDim.x + threadIdx.x, n, list, n_list);
  bool heavy = false, heavy_vol = false;
  if (i < n) {
    const float4 p = pos[i];
    const float4 d = disp[i];   // loaded with the position: one memory round trip for both
    const int tag = tag_of(p.w);
    bool moved = false;
    if (is_moving(tag, move_mask) && isfinite(p.x) && isfinite(p.y) && isfinite(p.z)) {
      if (tag == FPPG_TAG_VOLUME) {
        const GeomDev& G = geoms[ONE_GEOM ? 0 : min(geom_of(p.w), n_geom - 1)];
        const float y0 = p.x + d.x, y1 = p.y + d.y, y2 = p.z + d.z;
        if (!(isfinite(y0) && isfinite(y1) && isfinite(y2))) {
          atomicOr(status, FPPG_S_NONFINITE_POS);
        } else if (segment_near_facets(G, p.x, p.y, p.z, y0, y1, y2, tflag)) {
          heavy = heavy_vol = true;                        // the facet test in k_project_heavy
        } else {
          pos[i] = make_float4(y0, y1, y2, p.w);           // no facet near the move: it stays inside
          moved = true;
        }
      } else {
        heavy = true;
      }
    }
    if (accepted && !heavy) accepted[i] = moved ? 1 : 0;
  }
  // compact the heavy lanes of the block into its queue slots: the queued
  // volume moves first, then the surface and feature particles, each in index
  // order, so that the wavefronts of k_project_heavy mostly run one kind of
  // test (a wavefront whose lanes take both runs both, one after the other)
  __shared__ int s_wcnt[2][kBlock / 64];
  const uint64_t mv = __ballot(heavy_vol), mo = __ballot(heavy && !heavy_vol);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    s_wcnt[0][w] = __popcll(mv);
    s_wcnt[1][w] = __popcll(mo);
  }
  __syncthreads();
  int base_v = 0, base_o = 0, total_v = 0, total_o = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; ++k) {
    base_v += k < w ? s_wcnt[0][k] : 0;
    base_o += k < w ? s_wcnt[1][k] : 0;
    total_v += s_wcnt[0][k];
    total_o += s_wcnt[1][k];
  }
  const uint64_t below = (1ull << lane) - 1;
  if (heavy)
    queue[blockIdx.x * kBlock + (heavy_vol ? base_v + __popcll(mv & below) : total_v + base_o + __popcll(mo & below))] = i;
  if (threadIdx.x == 0) qcount[blockIdx.x] = total_v + total_o;
}

// Facet tests of the queued volume moves (segment_crosses, the decision the
// volume pass defers), surface reprojection and feature walks of the queued
// particles: block b
// takes the queues of volume-pass blocks [b, b + 1) * group, read as one list
// (the counts' prefix sums in LDS). group is 1 when every moving particle
// goes to the queue (no volume particle moves: dense queues, one block each)
// and kHeavyGroupMax otherwise (a few queued particles per volume block, packed
// into fuller wavefronts).
__global__ __launch_bounds__(kBlock) void k_project_heavy(float4* __restrict__ pos, int* __restrict__ owner,
                                                          const float4* __restrict__ disp,
                                                          int* __restrict__ feat_seg, double* __restrict__ feat_u,
                                                          int n_feat, int n_seg, const SegDev* __restrict__ segs,
                                                          const GeomDev* __restrict__ geoms, int n_geom,
                                                          const FacetDev* __restrict__ facets,
                                                          const int* __restrict__ tstart,
                                                          const int* __restrict__ ttri,
                                                          const uint8_t* __restrict__ tflag,
                                                          uint32_t* status, uint8_t* __restrict__ accepted,
                                                          const int* __restrict__ queue,
                                                          const int* __restrict__ qcount, int n_vblocks, int group,
                                                          int4* __restrict__ part, CsgDev cs, int* __restrict__ hard) {
  __shared__ int s_pre[kHeavyGroupMax + 1];
  __shared__ int s_rev[3];
  const int b0 = blockIdx.x * group;
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int k = 0; k < group; ++k) {
      s_pre[k] = acc;
      acc += b0 + k < n_vblocks ? qcount[b0 + k] : 0;
    }
    s_pre[group] = acc;
    s_rev[0] = s_rev[1] = s_rev[2] = 0;
  }
  __syncthreads();
  const int cnt = s_pre[group];
  int rs = 0, rf = 0, rv = 0;   // this lane's surface, feature and volume reverts
  for (int q = threadIdx.x; q < cnt; q += kBlock) {
    bool rev_s = false, rev_f = false, rev_v = false;
    {
      int k = 0;
      while (k + 1 < group && s_pre[k + 1] <= q) ++k;
      const int i = queue[(b0 + k) * kBlock + (q - s_pre[k])];
      const float4 p = pos[i];
      const int tag = tag_of(p.w);
      const float4 d = disp[i];
      const GeomDev& G = geoms[min(geom_of(p.w), n_geom - 1)];
      bool moved = false;
      if (tag == FPPG_TAG_VOLUME) {   // a move next to facets (finite, queued by the volume pass)
        const float y0 = p.x + d.x, y1 = p.y + d.y, y2 = p.z + d.z;
        if (segment_crosses(G, p.x, p.y, p.z, y0, y1, y2, facets, tstart, ttri, tflag, cs)) {
          rev_v = true;                                    // would leave the volume: stays at x
        } else {
          pos[i] = make_float4(y0, y1, y2, p.w);
          moved = true;
        }
      } else if (tag == FPPG_TAG_SURFACE) {
        const double yx = double(p.x) + double(d.x), yy = double(p.y) + double(d.y), yz = double(p.z) + double(d.z);
        if (!(isfinite(yx) && isfinite(yy) && isfinite(yz))) {
          atomicOr(status, FPPG_S_NONFINITE_POS);
        } else {
          bool wide = false;
          const SurfaceHit h = surface_search(G, yx, yy, yz, facets, tstart, ttri, tflag, cs, &wide);
          if (wide) {
            hard[1 + atomicAdd(&hard[0], 1)] = i;          // decided by k_project_wide
            continue;
          }
          pos[i] = make_float4(float(h.x), float(h.y), float(h.z), p.w);
          owner[i] = h.t;
          moved = true;
        }
      } else {   // feature
        const int slot = owner[i];
        int s = (slot >= 0 && slot < n_feat) ? feat_seg[slot] : -1;
        if (s < 0 || s >= n_seg) {
          atomicOr(status, FPPG_S_BAD_INDEX);
        } else {
          const long long bits = (long long)(unsigned)__float_as_int(d.x) | ((long long)__float_as_int(d.y) << 32);
          double u = feat_u[slot] + __longlong_as_double(bits);
          if (feature_walk(segs, s, u)) {
            const SegDev S = segs[s];
            pos[i] = make_float4(float(S.p0[0] + u * S.t[0]), float(S.p0[1] + u * S.t[1]),
                                 float(S.p0[2] + u * S.t[2]), p.w);
            feat_seg[slot] = s;
            feat_u[slot] = u;
            moved = true;
          } else {
            if (!isfinite(u)) atomicOr(status, FPPG_S_NONFINITE_POS);
            rev_f = true;
          }
        }
      }
      if (accepted) accepted[i] = moved ? 1 : 0;
    }
    rs += rev_s;
    rf += rev_f;
    rv += rev_v;
  }
  if (rs) atomicAdd(&s_rev[0], rs);
  if (rf) atomicAdd(&s_rev[1], rf);
  if (rv) atomicAdd(&s_rev[2], rv);
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = make_int4(s_rev[0], s_rev[1], s_rev[2], 0);
}

// Surface particles whose own search cell accepts no facet: one wavefront
// per particle, lane c (< 27) scanning cell c of the 3 x 3 x 3 block around y
// when it lies within R, then the wavefront's smallest (|d|, facet): the same
// argmin as the one-by-one search, in the time of one cell instead of 27.
__global__ __launch_bounds__(kBlock) void k_project_wide(float4* __restrict__ pos, int* __restrict__ owner,
                                                         const float4* __restrict__ disp,
                                                         const GeomDev* __restrict__ geoms, int n_geom,
                                                         const FacetDev* __restrict__ facets,
                                                         const int* __restrict__ tstart, const int* __restrict__ ttri,
                                                         const uint8_t* __restrict__ tflag,
                                                         uint8_t* __restrict__ accepted, const int* __restrict__ hard,
                                                         CsgDev cs, unsigned long long* __restrict__ counters) {
  const int lane = threadIdx.x & 63;
  const int wave = int((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int nwaves = int((gridDim.x * blockDim.x) >> 6);
  const int cnt = hard[0];
  int reverts = 0;
  for (int q = wave; q < cnt; q += nwaves) {
    const int i = hard[1 + q];
    const float4 p = pos[i];
    const float4 d = disp[i];
    const GeomDev& G = geoms[min(geom_of(p.w), n_geom - 1)];
    const double yx = double(p.x) + double(d.x), yy = double(p.y) + double(d.y), yz = double(p.z) + double(d.z);
    const double R = G.R;
    const double tx = search_t(G, 0, yx), ty = search_t(G, 1, yy), tz = search_t(G, 2, yz);
    const int cx = int(floor(tx)), cy = int(floor(ty)), cz = int(floor(tz));
    SurfaceHit h;
    if (lane < 27) {
      const int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = lane / 9 - 1;
      const int x = cx + dx, y = cy + dy, z = cz + dz;
      if (x >= 0 && x < G.tg_dims[0] && y >= 0 && y < G.tg_dims[1] && z >= 0 && z < G.tg_dims[2]) {
        const double gx = gap1(dx, tx - cx), gy = gap1(dy, ty - cy), gz = gap1(dz, tz - cz);
        const double lim = R * G.tg_inv + 1e-7;   // cell units: the cell must come within R of y
        const int64_t c = search_index(G, x, y, z);
        if (gx * gx + gy * gy + gz * gz <= lim * lim && (tflag[c] & kCellHasFacet))
          scan_surface_cell(c, yx, yy, yz, R, facets, tstart, ttri, h, G, cs);
      }
    }
    double b = h.best;
    int t = h.t;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(b, o);
      const int ot = __shfl_xor(t, o);
      if (ob < b || (ob == b && ot < t)) {
        b = ob;
        t = ot;
      }
    }
    if (t != 0x7fffffff) {
      const int src = __ffsll((long long)__ballot(h.t == t && h.best == b)) - 1;
      const double fx = __shfl(h.x, src), fy = __shfl(h.y, src), fz = __shfl(h.z, src);
      if (lane == 0) {
        pos[i] = make_float4(float(fx), float(fy), float(fz), p.w);
        owner[i] = t;
        if (accepted) accepted[i] = 1;
      }
    } else if (lane == 0) {
      ++reverts;                                          // no facet accepts: stays at x (section 3.3.3)
      if (accepted) accepted[i] = 0;
    }
  }
  if (lane == 0 && reverts) atomicAdd(&counters[FPPG_C_REVERT_SURFACE], (unsigned long long)reverts);
}

// Sum the per-block revert counts into the caller's counters (one block).
__global__ __launch_bounds__(kBlock) void k_project_counts(const int4* __restrict__ part, int n_part,
                                                           unsigned long long* __restrict__ counters) {
  __shared__ unsigned long long s[3][kBlock];
  unsigned long long a = 0, b = 0, c = 0;
  for (int k = threadIdx.x; k < n_part; k += kBlock) {
    const int4 v = part[k];
    a += unsigned(v.x);
    b += unsigned(v.y);
    c += unsigned(v.z);
  }
  s[0][threadIdx.x] = a;
  s[1][threadIdx.x] = b;
  s[2][threadIdx.x] = c;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int r = 0; r < 3; ++r) s[r][threadIdx.x] += s[r][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (s[0][0]) atomicAdd(&counters[FPPG_C_REVERT_SURFACE], s[0][0]);
    if (s[1][0]) atomicAdd(&counters[FPPG_C_REVERT_FEATURE], s[1][0]);
    if (s[2][0]) atomicAdd(&counters[FPPG_C_REVERT_VOLUME], s[2][0]);
  }
}

static inline int grid_for(int64_t n) { return int((n + kBlock - 1) / kBlock); }

}  // namespace fppg

using namespace fppg;

namespace {

static fppg_status project_impl(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, float* pos, int32_t* owner,
                                const float* disp, int32_t* feat_seg, double* feat_u, int32_t n_feat,
                                uint32_t move_mask, int64_t* counters, const int32_t* list, int32_t n_list,
                                uint8_t* accepted, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !geom) return fail(ctx, FPPG_E_ARG, "null ctx/geom");
  if (n != geom->n_active) return fail(ctx, FPPG_E_ARG, "n differs from the active particle count of the geometry");
  if (n > 0 && (!pos || !owner || !disp)) return fail(ctx, FPPG_E_ARG, "null pos/owner/disp");
  if (n_feat < 0 || (n_feat > 0 && (!feat_seg || !feat_u))) return fail(ctx, FPPG_E_ARG, "bad feature table");
  if (!aligned(pos, 16) || !aligned(disp, 16)) return fail(ctx, FPPG_E_ARG, "pos/disp must be 16-byte aligned");
  if (!counters) return fail(ctx, FPPG_E_ARG, "null counters");
  if (list && (n_list < 0 || n_list > n)) return fail(ctx, FPPG_E_ARG, "n_list must be in [0, n]");
  if (n == 0) return FPPG_OK;
  const WsLayout L = ws_layout(geom, n);
  if (!ws || !aligned(ws, 256)) return fail(ctx, FPPG_E_ARG, "ws is null or not 256-byte aligned");
  if (ws_bytes < L.proj_end) return fail(ctx, FPPG_E_WORKSPACE, "workspace too small for project");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = int(n);
  const int nr = list ? int(n_list) : ni;
  if (nr == 0) return FPPG_OK;
  int* qcount = reinterpret_cast<int*>(static_cast<char*>(ws) + L.proj_count);
  int4* part = reinterpret_cast<int4*>(static_cast<char*>(ws) + L.proj_part);
  int* queue = reinterpret_cast<int*>(static_cast<char*>(ws) + L.proj_queue);
  int* hard = reinterpret_cast<int*>(static_cast<char*>(ws) + L.proj_hard);
  unsigned long long* ctr = reinterpret_cast<unsigned long long*>(counters);
  float4* p4 = reinterpret_cast<float4*>(pos);
  const float4* d4 = reinterpret_cast<const float4*>(disp);
  PhaseTimer timer(ctx, 3, s);
  const int vb = grid_for(nr);
  if (geom->n_geom == 1)
    k_project_volume<true><<<vb, kBlock, 0, s>>>(p4, d4, ni, geom->d_geom, 1, geom->d_tg_flag, move_mask,
                                                 ctx->d_status, accepted, list, nr, queue, qcount, hard);
  else
    k_project_volume<false><<<vb, kBlock, 0, s>>>(p4, d4, ni, geom->d_geom, geom->n_geom, geom->d_tg_flag,
                                                  move_mask, ctx->d_status, accepted, list, nr, queue, qcount, hard);
  const int group = (move_mask >> FPPG_TAG_VOLUME) & 1u ? kHeavyGroupMax : 1;
  const int hb = (vb + group - 1) / group;
  k_project_heavy<<<hb, kBlock, 0, s>>>(p4, owner, d4, feat_seg, feat_u, n_feat, int(geom->n_seg), geom->d_seg,
                                        geom->d_geom, geom->n_geom, geom->d_facet, geom->d_tg_start, geom->d_tg_tri,
                                        geom->d_tg_flag, ctx->d_status, accepted, queue, qcount, vb, group,
                                        part, geom->csg(), hard);
  k_project_counts<<<1, kBlock, 0, s>>>(part, hb, ctr);
  // the wide searches: every wavefront loops over the queue, whose length the device holds
  k_project_wide<<<std::max(1, std::min(hb, 256)), kBlock, 0, s>>>(p4, owner, d4, geom->d_geom, geom->n_geom,
                                                                  geom->d_facet, geom->d_tg_start, geom->d_tg_tri,
                                                                  geom->d_tg_flag, accepted, hard, geom->csg(), ctr);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

}  // namespace

extern "C" fppg_status fppg_project(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, float* pos, int32_t* owner,
                                    const float* disp, int32_t* feat_seg, double* feat_u, int32_t n_feat,
                                    uint32_t move_mask, int64_t* counters, const int32_t* list, int32_t n_list,
                                    void* ws, size_t ws_bytes, void* stream) {
  return project_impl(ctx, geom, n, pos, owner, disp, feat_seg, feat_u, n_feat, move_mask, counters, list, n_list,
                      nullptr, ws, ws_bytes, stream);
}

extern "C" fppg_status fppg_project_record(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, float* pos,
                                           int32_t* owner, const float* disp, int32_t* feat_seg, double* feat_u,
                                           int32_t n_feat, uint32_t move_mask, int64_t* counters, uint8_t* accepted,
                                           void* ws, size_t ws_bytes, void* stream) {
  if (n > 0 && !accepted) return fail(ctx, FPPG_E_ARG, "null accepted");
  return project_impl(ctx, geom, n, pos, owner, disp, feat_seg, feat_u, n_feat, move_mask, counters, nullptr, 0,
                      accepted, ws, ws_bytes, stream);
}

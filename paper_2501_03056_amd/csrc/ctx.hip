// Context, errors, workspace layout and device-resident geometry of libfppg.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

namespace fppg {

fppg_status fail(fppg_ctx* ctx, fppg_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

fppg_status hip_fail(fppg_ctx* ctx, hipError_t e, const char* what) {
  if (ctx) ctx->err = std::string(what) + ": " + hipGetErrorString(e);
  return FPPG_E_HIP;
}

static size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

WsLayout ws_layout(const Geom* g, int64_t n) {
  WsLayout L{};
  const size_t N = size_t(n > 0 ? n : 1);
  const size_t nc = size_t(g->ncell > 0 ? g->ncell : 1);
  size_t o = 0;
  L.key = o;      o += up256(4 * N);
  L.rank = o;     o += up256(4 * N);
  L.tmp_id = o;   o += up256(4 * N);
  L.tmp_src = o;  o += up256(4 * N);
  L.tmp_key = o;  o += up256(4 * N);
  L.count = o;    o += up256(4 * (nc + 2));
  L.blocksum = o; o += up256(4 * size_t(scan_blocksum_len(nc + 1)));
  L.big = o;      o += up256(4 * (N / 65 + 1));   // cells of more than 64 particles: at most N / 65
  L.build_end = o;
  o = 0;
  L.accel = o;    o += up256(16 * N);
  L.step_end = o;
  o = 0;
  const size_t nbl = (N + kBlock - 1) / kBlock;
  L.list_cnt = o;  o += up256(4 * (nbl + 1));
  L.list_offs = o; o += up256(4 * (nbl + 2));
  L.list_bsum = o; o += up256(4 * size_t(scan_blocksum_len(nbl + 1)));
  L.list_end = o;
  o = 0;
  const size_t nvb = (N + kBlock - 1) / kBlock;   // blocks of the volume pass
  L.proj_count = o; o += up256(4 * nvb);
  L.proj_part = o;  o += up256(16 * nvb);   // one per k_project_heavy block (at most one per volume block)
  L.proj_queue = o; o += up256(4 * (N + kBlock));   // every entry lies below (launch blocks) * kBlock
  L.proj_hard = o;  o += up256(4 * (N + 1));          // count, then the particles the parallel search takes
  L.proj_end = o;
  // relax_energy: one FP64 partial per block of kBlock; vec_dot: kDotPartials
  L.reduce_end = up256(8 * std::max<size_t>((N + kBlock - 1) / kBlock + 1, kDotPartials));
  L.total = std::max(std::max(std::max(L.build_end, L.list_end), std::max(L.step_end, L.reduce_end)), L.proj_end);
  return L;
}

// ---- facet search grid -------------------------------------------------------------------

struct SearchGrid {
  double origin[3], cell, inv;
  int32_t dims[3];
};

// The facet search grid of one geometry: cells of edge R (1 + 2^-6) over the
// mesh's box widened by two cells. Its facets are registered on the device
// (register.hip: subdivision, separating-axis test against the cells widened
// by a relative pad of 1e-6 cell, so that a point on a facet whose cell index
// is computed with rounding still finds the facet in that cell). Facets of an
// assembly that never lie on its boundary are left out.
static fppg_status search_grid_params(fppg_ctx* ctx, const fppg_geom_desc& d, SearchGrid& sg) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int32_t v = 0; v < d.n_vert; ++v)
    for (int q = 0; q < 3; ++q) {
      lo[q] = std::min(lo[q], d.vert[3 * v + q]);
      hi[q] = std::max(hi[q], d.vert[3 * v + q]);
    }
  sg.cell = double(d.proj_radius) * (1.0 + 1.0 / 64.0);
  sg.inv = 1.0 / sg.cell;
  int64_t ncell = 1;
  for (int q = 0; q < 3; ++q) {
    sg.origin[q] = lo[q] - 2.0 * sg.cell;
    double ext = (hi[q] - lo[q]) * sg.inv;
    if (!(ext < 1e6)) return fail(ctx, FPPG_E_CAPACITY, "facet search grid too large (proj_radius too small)");
    sg.dims[q] = int32_t(std::ceil(ext)) + 5;
    ncell *= sg.dims[q];
  }
  if (ncell > (int64_t(1) << 30)) return fail(ctx, FPPG_E_CAPACITY, "facet search grid exceeds 2^30 cells");
  return FPPG_OK;
}

static int bits_for(uint64_t v) {
  int b = 0;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

template <class T>
static fppg_status upload(fppg_ctx* ctx, T** dst, const std::vector<T>& src) {
  size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
  FPPG_HIP(ctx, hipMalloc(reinterpret_cast<void**>(dst), bytes));
  if (!src.empty()) FPPG_HIP(ctx, hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return FPPG_OK;
}

static void free_geom(Geom* g) {
  if (!g) return;
  hipFree(g->d_geom);
  hipFree(g->d_facet);
  hipFree(g->d_n32);
  hipFree(g->d_seg);
  hipFree(g->d_tri_vert);
  hipFree(g->d_seg_vert);
  hipFree(g->d_tg_start);
  hipFree(g->d_tg_tri);
  hipFree(g->d_tg_flag);
  hipFree(g->d_facet_part);
  hipFree(g->d_part);
  hipFree(g->d_plane);
  hipFree(g->d_facet_mask);
}

// Planes of the convex parts of an assembly (section 3.2.3): every facet of a
// part gives a plane (n, d), n the unit outward normal and d = n.A; planes
// equal within 1e-12 are stored once. A part is accepted only if it is convex:
// every vertex of its facets within 1e-9 (1 + size) of the inner side of each
// of its planes.
static fppg_status build_parts(fppg_ctx* ctx, const fppg_geom_desc& d, int32_t g, int32_t tri_off,
                               std::vector<int32_t>& facet_part, std::vector<PartDev>& parts,
                               std::vector<double4>& planes, GeomDev& G, std::vector<uint8_t>& facet_class,
                               std::vector<uint8_t>& facet_mask) {
  G.csg_op = d.csg_op;
  G.part_begin_csg = G.part_end_csg = int32_t(parts.size());
  facet_class.clear();
  facet_mask.insert(facet_mask.end(), size_t(d.n_tri), uint8_t(0));
  if (d.csg_op == FPPG_CSG_NONE) {
    facet_part.insert(facet_part.end(), size_t(d.n_tri), -1);
    return FPPG_OK;
  }
  const std::string where = "geometry " + std::to_string(g) + ": ";
  if (d.csg_op != FPPG_CSG_UNION && d.csg_op != FPPG_CSG_DIFFERENCE)
    return fail(ctx, FPPG_E_ARG, where + "csg_op must be 0, 1 or 2");
  if (d.n_part < 1 || d.n_part > 8 || !d.part_tri_begin || d.part_tri_begin[0] != 0 ||
      d.part_tri_begin[d.n_part] != d.n_tri)
    return fail(ctx, FPPG_E_ARG, where + "part_tri_begin must run from 0 to n_tri over 1 to 8 parts");
  for (int32_t k = 0; k < d.n_part; ++k) {
    const int32_t b = d.part_tri_begin[k], e = d.part_tri_begin[k + 1];
    if (e <= b) return fail(ctx, FPPG_E_ARG, where + "every part needs a facet (part_tri_begin increasing)");
    const int32_t p0 = int32_t(planes.size());
    double lo = INFINITY, hi = -INFINITY;
    PartDev pd;
    for (int q = 0; q < 3; ++q) {
      pd.lo[q] = INFINITY;
      pd.hi[q] = -INFINITY;
    }
    for (int32_t t = b; t < e; ++t) {
      const double* A = d.vert + 3 * d.tri[3 * t];
      const double* B = d.vert + 3 * d.tri[3 * t + 1];
      const double* C = d.vert + 3 * d.tri[3 * t + 2];
      const double e0[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]}, e1[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
      double n[3] = {e0[1] * e1[2] - e0[2] * e1[1], e0[2] * e1[0] - e0[0] * e1[2], e0[0] * e1[1] - e0[1] * e1[0]};
      const double ln = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      for (int q = 0; q < 3; ++q) n[q] /= ln;
      const double dd = n[0] * A[0] + n[1] * A[1] + n[2] * A[2];
      bool dup = false;
      for (int32_t j = p0; j < int32_t(planes.size()) && !dup; ++j)
        dup = std::fabs(planes[j].x - n[0]) <= 1e-12 && std::fabs(planes[j].y - n[1]) <= 1e-12 &&
              std::fabs(planes[j].z - n[2]) <= 1e-12 && std::fabs(planes[j].w - dd) <= 1e-12;
      if (!dup) planes.push_back(make_double4(n[0], n[1], n[2], dd));
      for (int q = 0; q < 3; ++q) {
        lo = std::min(lo, std::min(A[q], std::min(B[q], C[q])));
        hi = std::max(hi, std::max(A[q], std::max(B[q], C[q])));
        pd.lo[q] = std::min(pd.lo[q], std::min(A[q], std::min(B[q], C[q])));
        pd.hi[q] = std::max(pd.hi[q], std::max(A[q], std::max(B[q], C[q])));
      }
      facet_part.push_back(int32_t(parts.size()));
    }
    const double tol = 1e-9 * (1.0 + (hi - lo));
    for (int32_t t = b; t < e; ++t)
      for (int c = 0; c < 3; ++c) {
        const double* V = d.vert + 3 * d.tri[3 * t + c];
        for (int32_t j = p0; j < int32_t(planes.size()); ++j)
          if (planes[j].x * V[0] + planes[j].y * V[1] + planes[j].z * V[2] - planes[j].w > tol)
            return fail(ctx, FPPG_E_ARG, where + "part " + std::to_string(k) + " is not convex");
      }
    pd.plane_begin = p0;
    pd.plane_end = int32_t(planes.size());
    for (int q = 0; q < 3; ++q) {   // widened so that the box never decides what the planes would not
      pd.lo[q] -= 1e-12 * (1.0 + std::fabs(pd.lo[q]));
      pd.hi[q] += 1e-12 * (1.0 + std::fabs(pd.hi[q]));
    }
    parts.push_back(pd);
  }
  G.part_end_csg = int32_t(parts.size());
  // Classify every facet against the other parts once, so that the per-point
  // test is needed only where a facet crosses another part's surface. With
  // V the three corners: "V strictly inside part j" (every plane < -tol) holds
  // for the whole facet (convexity); "a plane of j has every corner >= tol"
  // separates the whole facet from j. A facet that lies in a part it must
  // avoid (or outside part 0 for a cut part) is never on the boundary and is
  // left out of the facet search grid; one that is separated from every part
  // it must avoid (and inside part 0 for a cut part) is always on it and gets
  // part -1; any other keeps its part index for the per-point test.
  const int32_t pb = G.part_begin_csg;
  auto side = [&](int32_t j, const double* const V[3], double tol) {   // -1 all inside, +1 separated, 0 mixed
    const PartDev& r = parts[j];
    bool inside = true;
    for (int32_t q = r.plane_begin; q < r.plane_end; ++q) {
      const double4 P = planes[q];
      double mx = -INFINITY, mn = INFINITY;
      for (int c = 0; c < 3; ++c) {
        const double v = P.x * V[c][0] + P.y * V[c][1] + P.z * V[c][2] - P.w;
        mx = std::max(mx, v);
        mn = std::min(mn, v);
      }
      if (mn >= tol) return 1;
      if (mx >= -tol) inside = false;
    }
    return inside ? -1 : 0;
  };
  for (int32_t k = 0; k < d.n_part; ++k) {
    for (int32_t t = d.part_tri_begin[k]; t < d.part_tri_begin[k + 1]; ++t) {
      const double* V[3] = {d.vert + 3 * d.tri[3 * t], d.vert + 3 * d.tri[3 * t + 1], d.vert + 3 * d.tri[3 * t + 2]};
      double ext = 0.0;
      for (int q = 0; q < 3; ++q) ext = std::max(ext, std::fabs(V[0][q]) + std::fabs(V[1][q]) + std::fabs(V[2][q]));
      const double tol = 1e-12 * (1.0 + ext);
      int cls = 1;   // 0 never, 1 always, 2 per point
      uint8_t mask = 0;   // the parts a point of the facet must be tested against
      for (int32_t j = 0; j < d.n_part && cls != 0; ++j) {
        if (j == k) continue;
        const int sd = side(pb + j, V, tol);
        if (d.csg_op == FPPG_CSG_DIFFERENCE && j == 0 && k > 0) {   // must lie in part 0
          if (sd == 1) cls = 0;
          else if (sd == 0) cls = 2;
        } else {                                                   // must avoid part j
          if (sd == -1) cls = 0;
          else if (sd == 0) cls = 2;
        }
        if (sd == 0) mask |= uint8_t(1u << j);
      }
      facet_class.push_back(uint8_t(cls));
      facet_mask[facet_mask.size() - size_t(d.n_tri) + size_t(t)] = cls == 2 ? mask : 0;
      if (cls != 2) facet_part[facet_part.size() - size_t(d.n_tri) + size_t(t)] = -1;
    }
  }
  (void)tri_off;
  return FPPG_OK;
}

static fppg_status geom_create(fppg_ctx* ctx, const fppg_geom_desc* descs, int32_t n_geom,
                               fppg_geom** out) {
  if (!ctx || !out) return fail(ctx, FPPG_E_ARG, "null ctx/out");
  *out = nullptr;
  if (!descs || n_geom < 1 || n_geom > kMaxGeom) return fail(ctx, FPPG_E_ARG, "n_geom out of range");
  const int32_t k = descs[0].k;
  if (k != 1 && k != 2) return fail(ctx, FPPG_E_UNSUPPORTED, "stencil half-width k must be 1 or 2");
  std::vector<GeomDev> gd(n_geom);
  std::vector<FacetDev> facets;
  std::vector<float4> n32;
  std::vector<SegDev> segs;
  std::vector<int4> tri_vert;
  std::vector<int2> seg_vert;
  std::vector<int32_t> facet_part;
  std::vector<PartDev> parts;
  std::vector<double4> planes;
  std::vector<uint8_t> facet_class;   // of the current geometry's facets (assemblies only)
  std::vector<uint8_t> facet_mask;
  int32_t vert_off = 0;
  std::vector<RegItem> reg_items;  // facets to register in the search grids
  std::vector<RegGrid> reg_grids;  // one per geometry
  int64_t ncell = 0, part = 0, tg_cells = 0;
  bool any_levels = false;
  int32_t tri_off = 0, seg_off = 0;
  for (int32_t g = 0; g < n_geom; ++g) {
    const fppg_geom_desc& d = descs[g];
    GeomDev& G = gd[g];
    if (d.k != k) return fail(ctx, FPPG_E_UNSUPPORTED, "stencil half-width differs across the batch");
    if (!(d.h > 0.f) || !(d.proj_radius > 0.f) || !(d.inv_cell > 0.f) || !std::isfinite(d.inv_cell))
      return fail(ctx, FPPG_E_ARG, "geometry " + std::to_string(g) + ": h, proj_radius, inv_cell must be > 0");
    if (d.part_begin != part || d.part_end < d.part_begin)
      return fail(ctx, FPPG_E_ARG, "geometry " + std::to_string(g) + ": particle ranges must tile [0, n) in order");
    const float rc = 2.0f * d.h;
    if (double(1.0f / d.inv_cell) * k < double(rc) * (1.0 + 1.0 / 512.0) ||
        1.0 / double(d.inv_cell) * k < double(rc) * (1.0 + 1.0 / 512.0))
      return fail(ctx, FPPG_E_ARG, "geometry " + std::to_string(g) + ": cell edge smaller than (2h/k)(1+2^-9)");
    int64_t nc = 1;
    for (int q = 0; q < 3; ++q) {
      if (d.dims[q] < 1 || d.dims[q] >= (1 << 20)) return fail(ctx, FPPG_E_ARG, "dims must be in [1, 2^20)");
      G.origin[q] = d.origin[q];
      G.dims[q] = d.dims[q] * (q == 0 ? kXSplit : 1);
      nc *= G.dims[q];
    }
    G.inv_cell = d.inv_cell;
    G.inv_cell_x = d.inv_cell * float(kXSplit);
    G.k = k;
    G.h = d.h;
    G.rc2 = rc * rc;
    G.R = d.proj_radius;
    const double hd = d.h;
    G.kcoef = float(105.0 / (16.0 * M_PI * hd * hd * hd * hd * hd));
    if (d.max_level < 0 || d.max_level > 3)
      return fail(ctx, FPPG_E_ARG, "geometry " + std::to_string(g) + ": max_level must lie in [0, 3]");
    G.max_level = d.max_level;
    any_levels = any_levels || d.max_level > 0;
    G.cell_begin = ncell;
    G.part_begin = d.part_begin;
    G.part_end = d.part_end;
    ncell += nc;
    if (ncell >= (int64_t(1) << 31) - 1) return fail(ctx, FPPG_E_CAPACITY, "more than 2^31 particle cells");
    part = d.part_end;
    // mesh
    if (d.n_tri < 0 || d.n_vert < 0 || (d.n_tri > 0 && (!d.tri || !d.vert)))
      return fail(ctx, FPPG_E_ARG, "geometry " + std::to_string(g) + ": bad mesh arrays");
    for (int64_t i = 0; i < int64_t(d.n_tri) * 3; ++i)
      if (d.tri[i] < 0 || d.tri[i] >= d.n_vert) return fail(ctx, FPPG_E_ARG, "facet vertex index out of range");
    G.tri_begin = tri_off;
    G.tri_end = tri_off + d.n_tri;
    for (int32_t t = 0; t < d.n_tri; ++t) {
      const double* A = d.vert + 3 * d.tri[3 * t];
      const double* B = d.vert + 3 * d.tri[3 * t + 1];
      const double* C = d.vert + 3 * d.tri[3 * t + 2];
      FacetDev f;
      for (int q = 0; q < 3; ++q) {
        f.a[q] = A[q];
        f.e0[q] = B[q] - A[q];
        f.e1[q] = C[q] - A[q];
      }
      double nn[3] = {f.e0[1] * f.e1[2] - f.e0[2] * f.e1[1], f.e0[2] * f.e1[0] - f.e0[0] * f.e1[2],
                      f.e0[0] * f.e1[1] - f.e0[1] * f.e1[0]};
      double ln = std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
      if (!(ln > 0)) return fail(ctx, FPPG_E_ARG, "degenerate facet " + std::to_string(t));
      for (int q = 0; q < 3; ++q) f.n[q] = nn[q] / ln;
      f.d00 = f.e0[0] * f.e0[0] + f.e0[1] * f.e0[1] + f.e0[2] * f.e0[2];
      f.d01 = f.e0[0] * f.e1[0] + f.e0[1] * f.e1[1] + f.e0[2] * f.e1[2];
      f.d11 = f.e1[0] * f.e1[0] + f.e1[1] * f.e1[1] + f.e1[2] * f.e1[2];
      f.inv_den = 1.0 / (f.d00 * f.d11 - f.d01 * f.d01);
      facets.push_back(f);
      n32.push_back(make_float4(float(f.n[0]), float(f.n[1]), float(f.n[2]), 0.f));
      tri_vert.push_back(make_int4(vert_off + d.tri[3 * t], vert_off + d.tri[3 * t + 1], vert_off + d.tri[3 * t + 2], 0));
    }
    // parts of a Boolean assembly
    {
      const fppg_status pst = build_parts(ctx, d, g, tri_off, facet_part, parts, planes, G, facet_class,
                                          facet_mask);
      if (pst != FPPG_OK) return pst;
    }
    // feature segments
    G.seg_begin = seg_off;
    if (d.n_line < 0 || (d.n_line > 0 && (!d.line_seg_begin || !d.seg_p || !d.line_closed)))
      return fail(ctx, FPPG_E_ARG, "bad feature-line arrays");
    int32_t nseg = d.n_line > 0 ? d.line_seg_begin[d.n_line] : 0;
    for (int32_t l = 0; l < d.n_line; ++l) {
      int32_t b = d.line_seg_begin[l], e = d.line_seg_begin[l + 1];
      if (b < 0 || e < b || e > nseg) return fail(ctx, FPPG_E_ARG, "line_seg_begin not monotone");
      for (int32_t s = b; s < e; ++s) {
        SegDev sd;
        const double* p = d.seg_p + 6 * s;
        double v[3] = {p[3] - p[0], p[4] - p[1], p[5] - p[2]};
        sd.len = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (!(sd.len > 0)) return fail(ctx, FPPG_E_ARG, "zero-length feature segment");
        for (int q = 0; q < 3; ++q) {
          sd.p0[q] = p[q];
          sd.t[q] = v[q] / sd.len;
        }
        sd.lo = seg_off + b;
        sd.hi = seg_off + e;
        sd.closed = d.line_closed[l] ? 1 : 0;
        sd.pad = 0;
        segs.push_back(sd);
        int2 sv = make_int2(-1, -1);
        if (d.seg_vert) {
          const int32_t a = d.seg_vert[2 * s], b2 = d.seg_vert[2 * s + 1];
          if (a >= d.n_vert || b2 >= d.n_vert) return fail(ctx, FPPG_E_ARG, "seg_vert index out of range");
          sv = make_int2(a >= 0 ? vert_off + a : -1, b2 >= 0 ? vert_off + b2 : -1);
        }
        seg_vert.push_back(sv);
      }
    }
    seg_off += nseg;
    G.seg_end = seg_off;
    // facet search grid
    SearchGrid sg;
    fppg_status st = search_grid_params(ctx, d, sg);
    if (st != FPPG_OK) return st;
    {
      RegGrid rg{};
      for (int q = 0; q < 3; ++q) {
        rg.o[q] = sg.origin[q];
        rg.dims[q] = sg.dims[q];
      }
      rg.cell = sg.cell;
      rg.inv = sg.inv;
      rg.pad = 1e-6 * sg.cell;
      rg.key_begin = tg_cells;
      for (int32_t t = 0; t < d.n_tri; ++t) {
        if (!facet_class.empty() && facet_class[t] == 0) continue;   // an assembly's facet never on its boundary
        RegItem it{};
        for (int q = 0; q < 3; ++q) {
          it.a[q] = d.vert[3 * d.tri[3 * t] + q];
          it.b[q] = d.vert[3 * d.tri[3 * t + 1] + q];
          it.c[q] = d.vert[3 * d.tri[3 * t + 2] + q];
        }
        it.facet = tri_off + t;
        it.grid = int(reg_grids.size());
        reg_items.push_back(it);
      }
      reg_grids.push_back(rg);
    }
    tri_off += d.n_tri;
    vert_off += d.n_vert;
    for (int q = 0; q < 3; ++q) {
      G.tg_origin[q] = sg.origin[q];
      G.tg_dims[q] = sg.dims[q];
    }
    G.tg_inv = sg.inv;
    G.slab = (d.slab <= 0 || d.slab > d.dims[1]) ? d.dims[1] : d.slab;
    G.inv_slab = 1.0f / float(G.slab);
    G.tg_begin = tg_cells;
    tg_cells += int64_t(sg.dims[0]) * sg.dims[1] * sg.dims[2];
    if (tg_cells >= (int64_t(1) << 31)) return fail(ctx, FPPG_E_CAPACITY, "facet search grids exceed 2^31 cells");
  }
  // the search grids of all geometries registered on the device in one pass
  RegPairs reg{};
  {
    const fppg_status rst = register_facets(ctx, reg_items, reg_grids, false, bits_for(uint64_t(std::max<int64_t>(tg_cells - 1, 0))),
                                            bits_for(uint64_t(std::max(tri_off - 1, 0))), &reg, nullptr);
    if (rst != FPPG_OK) return rst;
  }
  int* d_tg_start = nullptr;
  int* d_tg_tri = nullptr;
  uint8_t* d_tg_flag = nullptr;
  {
    const fppg_status cst = registration_csr(ctx, reg, tg_cells, &d_tg_start, &d_tg_tri, &d_tg_flag, nullptr);
    hipFree(reg.keys);
    hipFree(reg.facets);
    if (cst != FPPG_OK) return cst;
  }
  Geom* geo = new (std::nothrow) fppg_geom();
  if (!geo) {
    hipFree(d_tg_start);
    hipFree(d_tg_tri);
    hipFree(d_tg_flag);
    return fail(ctx, FPPG_E_CAPACITY, "out of host memory");
  }
  geo->n_geom = n_geom;
  geo->k = k;
  geo->ncell = ncell;
  geo->n_tri = tri_off;
  geo->n_seg = seg_off;
  geo->tg_cells = tg_cells;
  geo->tg_entries = reg.n;
  geo->d_tg_start = d_tg_start;
  geo->d_tg_tri = d_tg_tri;
  geo->d_tg_flag = d_tg_flag;
  geo->n_part = part;
  geo->n_active = part;
  geo->n_vert = vert_off;
  geo->host = gd;
  geo->device = ctx->device;
  geo->has_csg = !parts.empty();
  geo->has_levels = any_levels;
  fppg_status st = FPPG_OK;
  if ((st = upload(ctx, &geo->d_geom, gd)) != FPPG_OK || (st = upload(ctx, &geo->d_facet, facets)) != FPPG_OK ||
      (st = upload(ctx, &geo->d_n32, n32)) != FPPG_OK || (st = upload(ctx, &geo->d_seg, segs)) != FPPG_OK ||
      (st = upload(ctx, &geo->d_tri_vert, tri_vert)) != FPPG_OK ||
      (st = upload(ctx, &geo->d_seg_vert, seg_vert)) != FPPG_OK ||
      (st = upload(ctx, &geo->d_facet_part, facet_part)) != FPPG_OK || (st = upload(ctx, &geo->d_part, parts)) != FPPG_OK ||
      (st = upload(ctx, &geo->d_plane, planes)) != FPPG_OK ||
      (st = upload(ctx, &geo->d_facet_mask, facet_mask)) != FPPG_OK) {
    free_geom(geo);
    delete static_cast<fppg_geom*>(geo);
    return st;
  }
  *out = static_cast<fppg_geom*>(geo);
  return FPPG_OK;
}

}  // namespace fppg

using namespace fppg;

extern "C" {

const char* fppg_status_str(fppg_status s) {
  switch (s) {
    case FPPG_OK: return "ok";
    case FPPG_E_ARG: return "invalid argument";
    case FPPG_E_HIP: return "HIP runtime error";
    case FPPG_E_WORKSPACE: return "workspace too small";
    case FPPG_E_CAPACITY: return "capacity exceeded";
    case FPPG_E_UNSUPPORTED: return "unsupported configuration";
    case FPPG_E_NODEVICE: return "no usable gfx950 device";
    default: return "unknown status";
  }
}

const char* fppg_last_error(const fppg_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

#ifndef FPPG_SOURCE_HASH
#define FPPG_SOURCE_HASH "unknown"
#endif
// The marker makes the hash readable from the file without loading it.
__attribute__((used)) static const char kSourceHashRecord[] = "FPPG_SOURCE_HASH:" FPPG_SOURCE_HASH;

const char* fppg_source_hash(void) { return kSourceHashRecord + 17; }

fppg_status fppg_create(int32_t device, fppg_ctx** out) {
  if (!out) return FPPG_E_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return FPPG_E_NODEVICE;
  if (device < 0 || device >= count) return FPPG_E_ARG;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return FPPG_E_NODEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FPPG_E_NODEVICE;
  if (hipSetDevice(device) != hipSuccess) return FPPG_E_NODEVICE;
  fppg_ctx* ctx = new (std::nothrow) fppg_ctx();
  if (!ctx) return FPPG_E_CAPACITY;
  ctx->device = device;
  if (hipMalloc(reinterpret_cast<void**>(&ctx->d_status), 64) != hipSuccess ||
      hipMemset(ctx->d_status, 0, 64) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&ctx->d_tickets), 64) != hipSuccess) {
    hipFree(ctx->d_status);
    delete ctx;
    return FPPG_E_HIP;
  }
  const fppg_status st = init_dot_scratch(ctx);   // the device is current here
  if (st != FPPG_OK) {
    hipFree(ctx->d_status);
    hipFree(ctx->d_tickets);
    delete ctx;
    return st;
  }
  *out = ctx;
  return FPPG_OK;
}

static void destroy_events(fppg_ctx* ctx) {
  for (auto& p : ctx->prof) {
    for (auto e : p.start) hipEventDestroy(e);
    for (auto e : p.stop) hipEventDestroy(e);
    p.start.clear();
    p.stop.clear();
    p.used = 0;
    p.ms = 0.0;
    p.launches = 0;
  }
  ctx->profiling = 0;
}

void fppg_destroy(fppg_ctx* ctx) {
  if (!ctx) return;
  destroy_events(ctx);
  hipFree(ctx->d_status);
  hipFree(ctx->d_tickets);
  delete ctx;
}

fppg_status fppg_profile(fppg_ctx* ctx, uint32_t phases) {
  if (!ctx) return FPPG_E_ARG;
  FPPG_HIP(ctx, hipSetDevice(ctx->device));
  destroy_events(ctx);
  phases &= (1u << FPPG_NPHASES) - 1u;
  if (!phases) return FPPG_OK;
  for (auto& p : ctx->prof) {
    p.start.resize(kProfSlots);
    p.stop.resize(kProfSlots);
    for (int i = 0; i < kProfSlots; ++i) {
      FPPG_HIP(ctx, hipEventCreate(&p.start[i]));
      FPPG_HIP(ctx, hipEventCreate(&p.stop[i]));
    }
  }
  ctx->profiling = phases;
  return FPPG_OK;
}

fppg_status fppg_profile_read(fppg_ctx* ctx, double* ms, int64_t* launches) {
  if (!ctx || !ms || !launches) return fail(ctx, FPPG_E_ARG, "null argument");
  for (int ph = 0; ph < FPPG_NPHASES; ++ph) {
    PhaseProf& p = ctx->prof[ph];
    for (int i = 0; i < p.used; ++i) {
      FPPG_HIP(ctx, hipEventSynchronize(p.stop[i]));
      float t = 0.f;
      FPPG_HIP(ctx, hipEventElapsedTime(&t, p.start[i], p.stop[i]));
      p.ms += t;
      p.launches++;
    }
    p.used = 0;
    ms[ph] = p.ms;
    launches[ph] = p.launches;
  }
  return FPPG_OK;
}

fppg_status fppg_read_status(fppg_ctx* ctx, void* stream, uint32_t* flags) {
  if (!ctx || !flags) return fail(ctx, FPPG_E_ARG, "null ctx/flags");
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t v = 0;
  FPPG_HIP(ctx, hipMemcpyAsync(&v, ctx->d_status, 4, hipMemcpyDeviceToHost, s));
  FPPG_HIP(ctx, hipStreamSynchronize(s));
  FPPG_HIP(ctx, hipMemsetAsync(ctx->d_status, 0, 4, s));
  FPPG_HIP(ctx, hipStreamSynchronize(s));
  *flags = v;
  return FPPG_OK;
}

fppg_status fppg_geom_create(fppg_ctx* ctx, const fppg_geom_desc* descs, int32_t n_geom, fppg_geom** out) {
  if (ctx) FPPG_HIP(ctx, hipSetDevice(ctx->device));
  return geom_create(ctx, descs, n_geom, out);
}

void fppg_geom_destroy(fppg_geom* geom) {
  if (!geom) return;
  free_geom(geom);
  delete geom;
}

fppg_status fppg_geom_info(const fppg_geom* g, int64_t* ncell, int64_t* n_tri, int64_t* n_seg,
                           int64_t* search_cells, int64_t* search_entries) {
  if (!g) return FPPG_E_ARG;
  if (ncell) *ncell = g->ncell;
  if (n_tri) *n_tri = g->n_tri;
  if (n_seg) *n_seg = g->n_seg;
  if (search_cells) *search_cells = g->tg_cells;
  if (search_entries) *search_entries = g->tg_entries;
  return FPPG_OK;
}

fppg_status fppg_geom_search_grid(fppg_ctx* ctx, const fppg_geom* g, int32_t* start, int32_t* tri, uint8_t* flag,
                                  void* stream) {
  if (!ctx || !g) return fail(ctx, FPPG_E_ARG, "null ctx/geom");
  if (g->device != ctx->device) return fail(ctx, FPPG_E_ARG, "geometry and context on different devices");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (start) FPPG_HIP(ctx, hipMemcpyAsync(start, g->d_tg_start, size_t(g->tg_cells + 1) * 4, hipMemcpyDeviceToDevice, s));
  if (tri && g->tg_entries > 0)
    FPPG_HIP(ctx, hipMemcpyAsync(tri, g->d_tg_tri, size_t(g->tg_entries) * 4, hipMemcpyDeviceToDevice, s));
  if (flag) FPPG_HIP(ctx, hipMemcpyAsync(flag, g->d_tg_flag, size_t(g->tg_cells), hipMemcpyDeviceToDevice, s));
  return FPPG_OK;
}

fppg_status fppg_workspace_size(const fppg_geom* g, int64_t n, size_t* bytes) {
  if (!g || !bytes || n < 0) return FPPG_E_ARG;
  *bytes = ws_layout(g, n).total;
  return FPPG_OK;
}

}  // extern "C"

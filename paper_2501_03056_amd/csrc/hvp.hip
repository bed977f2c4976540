// Sweeps over the same culled stencil as the force kernel (stencil.h) for
// the additions to the method: Jacobian-vector products of the force field
// (Newton-Krylov relaxation, reverse-mode differentiation), the pair energy
// (Newton line search), and the neighbour-set export used by the tests.
// Compiled without floating-point contraction, like the force kernel, so the
// neighbour predicate is the same binary32 expression.
#include "stencil.h"

#include <cfloat>
#include <type_traits>

namespace fppg {

// ---- pair energy (line search of Newton-Krylov relaxation) --------------------------------

// E = sum over moving receivers i and their sources j of c_ij W(r_ij), with
// c_ij = 1/2 when j moves too (the pair is then counted from both ends) and 1
// otherwise; W (Eq. 16) evaluated in FP64 from the binary32 positions. For a
// single moving class with fixed other sources, a = -grad E.
template <int K>
__global__ __launch_bounds__(kBlock) void k_energy(const float4* __restrict__ pos, int n, const int* __restrict__ cs,
                                                   const GeomDev* __restrict__ geoms, int n_geom, uint32_t move_mask,
                                                   double* __restrict__ partial) {
  const int i = xcd_chunk(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (i < n) {
    const float4 p = pos[i];
    const int tag = tag_of(p.w);
    if (is_moving(tag, move_mask) && isfinite(p.x) && isfinite(p.y) && isfinite(p.z)) {
      const GeomDev& G = geoms[min(geom_of(p.w), n_geom - 1)];
      const int rk = rank_of(tag);
      const double h = G.h;
      const double alpha = 21.0 / (16.0 * M_PI * h * h * h);
      const float rc2 = G.rc2;
      for_each_source<K>(stencil_of(p, G), G, cs, pos, [&](int j, const float4 q) {
        if (!(pair_d2(p.x - q.x, p.y - q.y, p.z - q.z) < rc2) || j == i) return;
        const int tj = tag_of(q.w);
        if (rank_of(tj) > rk) return;
        const double dx = double(p.x) - double(q.x), dy = double(p.y) - double(q.y), dz = double(p.z) - double(q.z);
        const double qq = sqrt(dx * dx + dy * dy + dz * dz) / h;
        const double t = fmax(1.0 - 0.5 * qq, 0.0);
        const double w = alpha * (t * t) * (t * t) * (2.0 * qq + 1.0);
        e += is_moving(tj, move_mask) ? 0.5 * w : w;
      });
    }
  }
  const double t = block_sum256(e);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// ---- Jacobian-vector products -----------------------------------------------------------

// M(r) w = K [ t^3 w - (3/2h) t^2 (r.w) r / |r| ],  t = 1 - |r|/2h  (0 outside the support).
// 1/|r| from the hardware reciprocal square root (about 1 ulp) and |r| = d2/|r|:
// one transcendental and no division per pair. r = 0 (coincident particles)
// gives rsq = inf; the r r^T/|r| term is then 0 by the guard.
__device__ __forceinline__ void pair_jac_apply(float dx, float dy, float dz, float d2, float inv2h, float k3, float w0,
                                               float w1, float w2, float& o0, float& o1, float& o2, float scale) {
  const float inv_r = d2 > 0.0f ? __builtin_amdgcn_rsqf(d2) : 0.0f;
  const float r = d2 * inv_r;
  const float t = fmaf(-r, inv2h, 1.0f);   // a pair has r < 2h; non-pairs carry weight 0
  const float t2 = t * t;
  const float c1 = scale * (t2 * t);
  const float rw = fmaf(dz, w2, fmaf(dy, w1, dx * w0));
  const float c2 = scale * (k3 * t2) * (rw * inv_r);
  o0 = fmaf(-c2, dx, fmaf(c1, w0, o0));
  o1 = fmaf(-c2, dy, fmaf(c1, w1, o1));
  o2 = fmaf(-c2, dz, fmaf(c1, w2, o2));
}

// Tangent projection and scale of the product's row (fppg_relax_hvp_projected).
struct ProjectOut {
  const int* owner;
  const int* feat_seg;
  int n_feat, n_tri, n_seg;
  const float4* n32;
  const SegDev* segs;
  float scale;
  uint32_t* status;
};

template <int K, bool TRANSPOSE, bool PROJECT = false>
__global__ __launch_bounds__(kBlock) void k_jvp(const float4* __restrict__ pos, int n, const int* __restrict__ cs,
                                                const GeomDev* __restrict__ geoms, int n_geom, uint32_t move_mask,
                                                const float4* __restrict__ v, float4* __restrict__ out, int remap,
                                                ProjectOut po = ProjectOut{}) {
  // the blocks' XCD mapping is the context's force launch setting
  // (launch_chunk; per-lane sums whichever it is)
  const int i = launch_chunk(remap, int(blockIdx.x), int(gridDim.x)) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 p = pos[i];
  const int tag = tag_of(p.w);
  const bool mov_i = is_moving(tag, move_mask);
  float o0 = 0.0f, o1 = 0.0f, o2 = 0.0f;
  // a quarantined (non-finite) particle is nobody's neighbour: its row is 0
  if ((mov_i || TRANSPOSE) && isfinite(p.x) && isfinite(p.y) && isfinite(p.z)) {
    const int g = min(geom_of(p.w), n_geom - 1);
    const GeomDev& G = geoms[g];
    const int rk = rank_of(tag);
    const uint32_t T = tag < FPPG_TAG_VOLUME ? uint32_t(tag) : 7u;   // tag_j <= T <=> rank_j <= rank_i
    const float rc2 = G.rc2;
    const float inv2h = 0.5f / G.h;
    const float k3 = 3.0f * inv2h;
    const float4 vi = v[i];
    // Branch-free body: a candidate that is not a pair gets weight 0 (all
    // inputs are finite, so the unused terms stay finite), so the loads of
    // both rows are issued up front and no exec mask is juggled per
    // candidate. M(r) is linear in w, so the two terms of the transposed
    // product share one application.
    const Stencil st = stencil_of(p, G);
    if (!TRANSPOSE) {
      // J v: every source's term M(r)(v_i - v_j). The receiver itself needs no
      // test: there w = v_i - v_i = 0 and r = 0, so its term is exactly 0 (the
      // clamp of d2 keeps 1/|r| finite). Wavefronts of volume receivers only
      // (which take every class) skip the class test. As in the force kernel,
      // t = 1 - r/2h is clamped to [0, 1] by the FMA's output modifier and no
      // neighbour test is needed: both terms carry t^2, zero at and beyond
      // 2h; next to the predicate's pairs the product differs only by pairs
      // within rounding of r = 2h, whose terms are below 2^-46 of a
      // unit-distance term.
      auto body = [&](auto ranked) {
        for_each_source_with<K>(st, G, cs, pos, v, [&](int, const float4 q, const float4 vj) {
          const float dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
          const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
          const float inv_r = __builtin_amdgcn_rsqf(fmaxf(d2, FLT_MIN));
          const float t0 = __builtin_amdgcn_fmed3f(fmaf(-(d2 * inv_r), inv2h, 1.0f), 0.0f, 1.0f);
          const float t = decltype(ranked)::value ? (((__float_as_uint(q.w) & 7u) <= T) ? t0 : 0.0f) : t0;
          const float t2 = t * t;
          const float c1 = t2 * t;
          const float w0 = vi.x - vj.x, w1 = vi.y - vj.y, w2 = vi.z - vj.z;
          const float rw = fmaf(dz, w2, fmaf(dy, w1, dx * w0));
          const float c2 = (k3 * t2) * (rw * inv_r);
          o0 = fmaf(-c2, dx, fmaf(c1, w0, o0));
          o1 = fmaf(-c2, dy, fmaf(c1, w1, o1));
          o2 = fmaf(-c2, dz, fmaf(c1, w2, o2));
        });
      };
      if (__ballot(mov_i && tag < FPPG_TAG_VOLUME) != 0) body(std::true_type{});
      else body(std::false_type{});
    } else {
      for_each_source_with<K>(st, G, cs, pos, v, [&](int j, const float4 q, const float4 vj) {
        const float dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
        const float d2 = pair_d2(dx, dy, dz);
        const uint32_t tj = __float_as_uint(q.w) & 7u;
        // bitwise, not short-circuit, so that nothing here branches
        const bool pair = (d2 < rc2) & (j != i);
        const float s1 = (pair & mov_i & (tj <= T)) ? 1.0f : 0.0f;
        const float s2 = (pair & is_moving(int(tj), move_mask) & (rk <= rank_of(int(tj)))) ? -1.0f : 0.0f;
        pair_jac_apply(dx, dy, dz, d2, inv2h, k3, fmaf(s1, vi.x, s2 * vj.x), fmaf(s1, vi.y, s2 * vj.y),
                       fmaf(s1, vi.z, s2 * vj.z), o0, o1, o2, 1.0f);
      });
    }
    o0 *= G.kcoef;
    o1 *= G.kcoef;
    o2 *= G.kcoef;
  }
  float4 r = make_float4(o0, o1, o2, 0.0f);
  if (PROJECT) {
    r = tangent_apply(r, tag, i, move_mask, po.owner, po.feat_seg, po.n_feat, po.n_tri, po.n_seg, po.n32, po.segs,
                      po.status);
    r.x *= po.scale;
    r.y *= po.scale;
    r.z *= po.scale;
  }
  out[i] = r;
}

// ---- neighbour export (tests) -------------------------------------------------------------

template <int K>
__global__ __launch_bounds__(kBlock) void k_neighbors(const float4* __restrict__ pos, int n, const int* __restrict__ cs,
                                                      const GeomDev* __restrict__ geoms, int n_geom,
                                                      int* __restrict__ count, int* __restrict__ list, int cap) {
  const int i = xcd_chunk(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 p = pos[i];
  const GeomDev& G = geoms[min(geom_of(p.w), n_geom - 1)];
  int c = 0;
  const float rc2 = G.rc2;
  for_each_source<K>(stencil_of(p, G), G, cs, pos, [&](int j, const float4 q) {
    const float d2 = pair_d2(p.x - q.x, p.y - q.y, p.z - q.z);
    if (d2 < rc2 && j != i) {
      if (c < cap) list[int64_t(i) * cap + c] = j;
      ++c;
    }
  });
  count[i] = c;
}

static inline int grid_for(int64_t n) { return int((n + kBlock - 1) / kBlock); }

static fppg_status check_common(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                const int32_t* cs) {
  if (!ctx || !geom) return fail(ctx, FPPG_E_ARG, "null ctx/geom");
  if (n != geom->n_active) return fail(ctx, FPPG_E_ARG, "n differs from the active particle count of the geometry");
  if (n > 0 && (!pos || !cs)) return fail(ctx, FPPG_E_ARG, "null pos/cell_start");
  if (!aligned(pos, 16)) return fail(ctx, FPPG_E_ARG, "pos must be 16-byte aligned");
  if (geom->has_levels)   // these sweeps use one smoothing length per geometry
    return fail(ctx, FPPG_E_UNSUPPORTED, "Jacobian, energy and neighbour sweeps of a multi-resolution geometry are not supported");
  return FPPG_OK;
}

}  // namespace fppg

using namespace fppg;

extern "C" fppg_status fppg_relax_hvp(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                      const int32_t* cell_start, uint32_t move_mask, int32_t transpose,
                                      const float* v, float* Jv, void* stream) {
  fppg_status st = check_common(ctx, geom, n, pos, cell_start);
  if (st != FPPG_OK) return st;
  if (n > 0 && (!v || !Jv)) return fail(ctx, FPPG_E_ARG, "null v/Jv");
  if (!aligned(v, 16) || !aligned(Jv, 16)) return fail(ctx, FPPG_E_ARG, "v/Jv must be 16-byte aligned");
  if (v == Jv && n > 0) return fail(ctx, FPPG_E_ARG, "Jv must not alias v");
  if (n == 0) return FPPG_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = int(n);
  const float4* p4 = reinterpret_cast<const float4*>(pos);
  const float4* v4 = reinterpret_cast<const float4*>(v);
  float4* o4 = reinterpret_cast<float4*>(Jv);
  PhaseTimer timer(ctx, 4, s);
  if (geom->k == 1) {
    if (transpose) k_jvp<1, true><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, move_mask, v4, o4, ctx->xcd_remap);
    else k_jvp<1, false><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, move_mask, v4, o4, ctx->xcd_remap);
  } else {
    if (transpose) k_jvp<2, true><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, move_mask, v4, o4, ctx->xcd_remap);
    else k_jvp<2, false><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, move_mask, v4, o4, ctx->xcd_remap);
  }
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

extern "C" fppg_status fppg_relax_hvp_projected(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                                const int32_t* cell_start, const int32_t* owner,
                                                const int32_t* feat_seg, int32_t n_feat, uint32_t move_mask,
                                                const float* v, float scale, float* out, void* stream) {
  fppg_status st = check_common(ctx, geom, n, pos, cell_start);
  if (st != FPPG_OK) return st;
  if (n > 0 && (!v || !out || !owner)) return fail(ctx, FPPG_E_ARG, "null v/out/owner");
  if (n_feat < 0 || (n_feat > 0 && !feat_seg)) return fail(ctx, FPPG_E_ARG, "bad feature table");
  if (!aligned(v, 16) || !aligned(out, 16)) return fail(ctx, FPPG_E_ARG, "v/out must be 16-byte aligned");
  if (v == out && n > 0) return fail(ctx, FPPG_E_ARG, "out must not alias v");
  if (n == 0) return FPPG_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = int(n);
  const ProjectOut po{owner, feat_seg, n_feat, int(geom->n_tri), int(geom->n_seg), geom->d_n32, geom->d_seg, scale,
                      ctx->d_status};
  const float4* p4 = reinterpret_cast<const float4*>(pos);
  const float4* v4 = reinterpret_cast<const float4*>(v);
  float4* o4 = reinterpret_cast<float4*>(out);
  PhaseTimer timer(ctx, 4, s);
  if (geom->k == 1)
    k_jvp<1, false, true><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, move_mask, v4, o4, ctx->xcd_remap, po);
  else
    k_jvp<2, false, true><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, move_mask, v4, o4, ctx->xcd_remap, po);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

extern "C" fppg_status fppg_relax_energy(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                         const int32_t* cell_start, uint32_t move_mask, double* out, void* ws,
                                         size_t ws_bytes, void* stream) {
  fppg_status st = check_common(ctx, geom, n, pos, cell_start);
  if (st != FPPG_OK) return st;
  if (!out || !ws || !aligned(ws, 256)) return fail(ctx, FPPG_E_ARG, "null out or null/misaligned ws");
  const int nb = std::max(1, grid_for(n));
  if (ws_bytes < size_t(nb) * sizeof(double)) return fail(ctx, FPPG_E_WORKSPACE, "workspace too small for relax_energy");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* partial = static_cast<double*>(ws);
  const float4* p4 = reinterpret_cast<const float4*>(pos);
  if (geom->k == 1) k_energy<1><<<nb, kBlock, 0, s>>>(p4, int(n), cell_start, geom->d_geom, geom->n_geom, move_mask, partial);
  else k_energy<2><<<nb, kBlock, 0, s>>>(p4, int(n), cell_start, geom->d_geom, geom->n_geom, move_mask, partial);
  FPPG_HIP(ctx, hipGetLastError());
  return sum_partials(ctx, partial, nb, out, s);
}

extern "C" fppg_status fppg_debug_neighbors(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                            const int32_t* cell_start, int32_t* count, int32_t* list, int32_t cap,
                                            void* stream) {
  fppg_status st = check_common(ctx, geom, n, pos, cell_start);
  if (st != FPPG_OK) return st;
  if (cap < 0 || (n > 0 && (!count || (cap > 0 && !list)))) return fail(ctx, FPPG_E_ARG, "bad count/list/cap");
  if (n == 0) return FPPG_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = int(n);
  const float4* p4 = reinterpret_cast<const float4*>(pos);
  if (geom->k == 1) k_neighbors<1><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, count, list, cap);
  else k_neighbors<2><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, count, list, cap);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

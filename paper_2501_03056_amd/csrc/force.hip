// Pair sweeps over the cell list: relaxation force + amax (Eq. 15-17), the
// displacement update (Eq. 22-25), the Jacobian-vector products of the force
// field, and the neighbour-set export used by the tests.
//
// One lane per sorted receiver. With x-fastest cell keys the cells of a
// stencil row along x are contiguous in the sorted order, so a receiver
// visits at most (2k+1)^2 contiguous index ranges. Rows and the x-extent of a
// row are culled in cell units against the support radius: a skipped cell is
// at least k cell edges (> 2h, the edge being (2h/k)(1+2^-9) or more) from the
// receiver, so it holds no source and the culled sums are bitwise identical to
// the full-stencil sums. Sources are summed in a fixed order (rows by dz then
// dy ascending, then sorted index): the sums are deterministic.
//
// The neighbour predicate is the binary32 expression
// fl32(fl32(fl32(dx*dx) + fl32(dy*dy)) + fl32(dz*dz)) < rc2; this file is
// compiled without floating-point contraction so that the compiler cannot fuse
// it, and the accumulations use explicit fmaf.
#include "stencil.h"

namespace fppg {

__global__ void k_zero_f32(float* __restrict__ a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

// ---- forces + amax ---------------------------------------------------------------------

// One source: K-less pair term (1 - r/2h)^3 r_ij if j is a source of i.
// RANKED: check rank(tag_j) <= rank(tag_i) as tag_j <= T (T = rank, or 7 for
// volume receivers which take every class). The receiver itself contributes
// r = 0, so it needs no test (the count subtracts it).
template <bool RANKED, bool COUNT>
__device__ __forceinline__ void add_pair(const float4 p, const float4 q, float rc2, float inv2h, uint32_t T,
                                         float& ax, float& ay, float& az, float& cnt) {
  const float dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
  const float d2 = pair_d2(dx, dy, dz);
  bool src = d2 < rc2;
  if (RANKED) src = src & ((__float_as_uint(q.w) & 7u) <= T);
  const float t = fmaxf(fmaf(-__builtin_amdgcn_sqrtf(d2), inv2h, 1.0f), 0.0f);
  const float w = src ? t * t * t : 0.0f;
  ax = fmaf(w, dx, ax);
  ay = fmaf(w, dy, ay);
  az = fmaf(w, dz, az);
  if (COUNT) cnt += src ? 1.0f : 0.0f;
}

template <int K, bool COUNT>
__global__ __launch_bounds__(kBlock) void k_force(const float4* __restrict__ pos, int n,
                                                  const int* __restrict__ cs, const GeomDev* __restrict__ geoms,
                                                  int n_geom, uint32_t move_mask, float4* __restrict__ accel,
                                                  unsigned* __restrict__ amax_bits, uint32_t* status) {
  const int i = xcd_chunk(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  float anorm = 0.0f;
  int g = 0;
  bool mov = false;
  float4 p = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  int tag = 0;
  if (i < n) {
    p = pos[i];
    tag = tag_of(p.w);
    g = min(geom_of(p.w), n_geom - 1);
    mov = is_moving(tag, move_mask);
    if (mov && !(isfinite(p.x) && isfinite(p.y) && isfinite(p.z))) {
      atomicOr(status, FPPG_S_NONFINITE_ACCEL);   // quarantined particle: no force, no move
      mov = false;
    }
  }
  // wavefronts of volume receivers only skip the class test
  const bool ranked = __ballot(mov && tag < FPPG_TAG_VOLUME) != 0;
  float ax = 0.0f, ay = 0.0f, az = 0.0f, cnt = 0.0f;
  if (mov) {
    const GeomDev& G = geoms[g];
    const float rc2 = G.rc2;
    const float inv2h = 0.5f / G.h;
    const uint32_t T = tag < FPPG_TAG_VOLUME ? uint32_t(tag) : 7u;
    const Stencil st = stencil_of(p, G);
    if (ranked)
      for_each_source<K>(st, G, cs, pos, [&](int, const float4 q) { add_pair<true, COUNT>(p, q, rc2, inv2h, T, ax, ay, az, cnt); });
    else
      for_each_source<K>(st, G, cs, pos, [&](int, const float4 q) { add_pair<false, COUNT>(p, q, rc2, inv2h, T, ax, ay, az, cnt); });
    ax *= G.kcoef;
    ay *= G.kcoef;
    az *= G.kcoef;
    if (COUNT) cnt -= 1.0f;   // the receiver itself
    anorm = sqrtf(ax * ax + ay * ay + az * az);
    if (!isfinite(anorm)) {
      atomicOr(status, FPPG_S_NONFINITE_ACCEL);
      ax = ay = az = 0.0f;
      anorm = 0.0f;
    }
  }
  if (i < n) accel[i] = make_float4(ax, ay, az, cnt);
  // per-geometry max of |a|: wave max, block max, one atomic per block and geometry
  __shared__ float s_max[kBlock / 64];
  __shared__ int s_geo[kBlock / 64];
  const int g0 = __shfl(g, 0);
  const bool mixed = __ballot(anorm > 0.0f && g != g0) != 0;
  if (mixed && anorm > 0.0f) atomicMax(&amax_bits[g], __float_as_uint(anorm));   // wave spans geometries
  float m = mixed ? 0.0f : anorm;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) {
    s_max[threadIdx.x >> 6] = m;
    s_geo[threadIdx.x >> 6] = g0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < kBlock / 64; ++w) {
      float mm = s_max[w];
      if (!(mm > 0.0f)) continue;
      for (int w2 = w + 1; w2 < kBlock / 64; ++w2)
        if (s_geo[w2] == s_geo[w]) {
          mm = fmaxf(mm, s_max[w2]);
          s_max[w2] = 0.0f;
        }
      atomicMax(&amax_bits[s_geo[w]], __float_as_uint(mm));
    }
  }
}

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

// ---- displacement (Eq. 22-25) ------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_update(const float4* __restrict__ pos, const float4* __restrict__ accel,
                                                   const int* __restrict__ owner, const int* __restrict__ feat_seg,
                                                   int n, int n_feat, int n_tri, int n_seg,
                                                   const GeomDev* __restrict__ geoms, int n_geom,
                                                   const float* __restrict__ amax, const float4* __restrict__ n32,
                                                   const SegDev* __restrict__ segs, uint32_t move_mask,
                                                   float4* __restrict__ disp, uint32_t* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 p = pos[i];
  const int tag = tag_of(p.w);
  float4 d = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (is_moving(tag, move_mask)) {
    const int g = min(geom_of(p.w), n_geom - 1);
    const float am = amax[g];
    const float tau = am > 0.0f ? (geoms[g].h * 0.0625f) / am : 0.0f;   // dt^2 = (h/16)/amax
    const float4 a = accel[i];
    float rx = tau * a.x, ry = tau * a.y, rz = tau * a.z;               // v reset: dr = a dt^2
    if (tag == FPPG_TAG_SURFACE) {
      const int o = owner[i];
      if (o < 0 || o >= n_tri) {
        atomicOr(status, FPPG_S_BAD_INDEX);
        rx = ry = rz = 0.0f;
      } else {
        const float4 nn = n32[o];
        const float s = rx * nn.x + ry * nn.y + rz * nn.z;              // Eq. 25 on the displacement
        rx -= s * nn.x;
        ry -= s * nn.y;
        rz -= s * nn.z;
      }
      d = make_float4(rx, ry, rz, 0.0f);
    } else if (tag == FPPG_TAG_FEATURE) {
      const int o = owner[i];
      const int sg = (o >= 0 && o < n_feat) ? feat_seg[o] : -1;
      if (sg < 0 || sg >= n_seg) {
        atomicOr(status, FPPG_S_BAD_INDEX);
      } else {
        const SegDev S = segs[sg];
        const double du = double(rx) * S.t[0] + double(ry) * S.t[1] + double(rz) * S.t[2];
        const long long bits = __double_as_longlong(du);
        d = make_float4(__int_as_float(int(bits & 0xffffffffll)), __int_as_float(int(bits >> 32)), 0.0f, 0.0f);
      }
    } else {
      d = make_float4(rx, ry, rz, 0.0f);
    }
  }
  disp[i] = d;
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
  const float t = fmaxf(fmaf(-r, inv2h, 1.0f), 0.0f);
  const float t2 = t * t;
  const float c1 = scale * (t2 * t);
  const float rw = fmaf(dz, w2, fmaf(dy, w1, dx * w0));
  const float c2 = scale * (k3 * t2) * (rw * inv_r);
  o0 = fmaf(-c2, dx, fmaf(c1, w0, o0));
  o1 = fmaf(-c2, dy, fmaf(c1, w1, o1));
  o2 = fmaf(-c2, dz, fmaf(c1, w2, o2));
}

template <int K, bool TRANSPOSE>
__global__ __launch_bounds__(kBlock) void k_jvp(const float4* __restrict__ pos, int n, const int* __restrict__ cs,
                                                const GeomDev* __restrict__ geoms, int n_geom, uint32_t move_mask,
                                                const float4* __restrict__ v, float4* __restrict__ out) {
  const int i = xcd_chunk(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 p = pos[i];
  const int tag = tag_of(p.w);
  const bool mov_i = is_moving(tag, move_mask);
  float o0 = 0.0f, o1 = 0.0f, o2 = 0.0f;
  if (mov_i || TRANSPOSE) {
    const int g = min(geom_of(p.w), n_geom - 1);
    const GeomDev& G = geoms[g];
    const int rk = rank_of(tag);
    const float rc2 = G.rc2;
    const float inv2h = 0.5f / G.h;
    const float k3 = 3.0f * inv2h;
    const float4 vi = v[i];
    for_each_source_with<K>(stencil_of(p, G), G, cs, pos, v, [&](int j, const float4 q, const float4 vj) {
      const float dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
      const float d2 = pair_d2(dx, dy, dz);
      if (!(d2 < rc2) || j == i) return;
      const int tj = tag_of(q.w);
      const int rj = rank_of(tj);
      if (!TRANSPOSE) {
        if (rj <= rk) pair_jac_apply(dx, dy, dz, d2, inv2h, k3, vi.x - vj.x, vi.y - vj.y, vi.z - vj.z, o0, o1, o2, 1.0f);
      } else {
        if (mov_i && rj <= rk) pair_jac_apply(dx, dy, dz, d2, inv2h, k3, vi.x, vi.y, vi.z, o0, o1, o2, 1.0f);
        if (is_moving(tj, move_mask) && rk <= rj)
          pair_jac_apply(dx, dy, dz, d2, inv2h, k3, vj.x, vj.y, vj.z, o0, o1, o2, -1.0f);
      }
    });
    o0 *= G.kcoef;
    o1 *= G.kcoef;
    o2 *= G.kcoef;
  }
  out[i] = make_float4(o0, o1, o2, 0.0f);
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
  if (n != geom->n_part) return fail(ctx, FPPG_E_ARG, "n differs from the particle count of the geometry descriptors");
  if (n > 0 && (!pos || !cs)) return fail(ctx, FPPG_E_ARG, "null pos/cell_start");
  if (!aligned(pos, 16)) return fail(ctx, FPPG_E_ARG, "pos must be 16-byte aligned");
  return FPPG_OK;
}

}  // namespace fppg

using namespace fppg;

extern "C" fppg_status fppg_relax_step(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                       const int32_t* owner, const int32_t* cell_start, const int32_t* feat_seg,
                                       int32_t n_feat, uint32_t move_mask, uint32_t flags, float* accel,
                                       float* amax, float* disp, void* ws, size_t ws_bytes, void* stream) {
  fppg_status st = check_common(ctx, geom, n, pos, cell_start);
  if (st != FPPG_OK) return st;
  if (!amax || !disp || !owner) return fail(ctx, FPPG_E_ARG, "null amax/disp/owner");
  if (n_feat < 0 || (n_feat > 0 && !feat_seg)) return fail(ctx, FPPG_E_ARG, "bad feature table");
  if (!aligned(disp, 16) || (accel && !aligned(accel, 16))) return fail(ctx, FPPG_E_ARG, "accel/disp must be 16-byte aligned");
  const WsLayout L = ws_layout(geom, n);
  float4* acc = reinterpret_cast<float4*>(accel);
  if (!acc) {
    if (!ws || !aligned(ws, 256)) return fail(ctx, FPPG_E_ARG, "accel is NULL and ws is null or misaligned");
    if (ws_bytes < L.step_end) return fail(ctx, FPPG_E_WORKSPACE, "workspace too small for relax_step");
    acc = reinterpret_cast<float4*>(static_cast<char*>(ws) + L.accel);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = int(n);
  const bool count = (flags & FPPG_F_COUNT_PAIRS) != 0;
  k_zero_f32<<<grid_for(geom->n_geom), kBlock, 0, s>>>(amax, geom->n_geom);
  if (ni > 0) {
    const float4* p4 = reinterpret_cast<const float4*>(pos);
    unsigned* ab = reinterpret_cast<unsigned*>(amax);
    {
    PhaseTimer timer(ctx, 1, s);
    if (geom->k == 1) {
      if (count) k_force<1, true><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, move_mask, acc, ab, ctx->d_status);
      else k_force<1, false><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, move_mask, acc, ab, ctx->d_status);
    } else {
      if (count) k_force<2, true><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, move_mask, acc, ab, ctx->d_status);
      else k_force<2, false><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, move_mask, acc, ab, ctx->d_status);
    }
    }
    PhaseTimer timer(ctx, 2, s);
    k_update<<<grid_for(ni), kBlock, 0, s>>>(p4, acc, owner, feat_seg, ni, n_feat, int(geom->n_tri), int(geom->n_seg),
                                             geom->d_geom, geom->n_geom, amax, geom->d_n32, geom->d_seg, move_mask,
                                             reinterpret_cast<float4*>(disp), ctx->d_status);
  }
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

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
    if (transpose) k_jvp<1, true><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, move_mask, v4, o4);
    else k_jvp<1, false><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, move_mask, v4, o4);
  } else {
    if (transpose) k_jvp<2, true><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, move_mask, v4, o4);
    else k_jvp<2, false><<<grid_for(ni), kBlock, 0, s>>>(p4, ni, cell_start, geom->d_geom, geom->n_geom, move_mask, v4, o4);
  }
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

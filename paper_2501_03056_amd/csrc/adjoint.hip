// Reverse-mode pieces for differentiating a relaxation run with respect to
// the mesh vertices (not in the paper):
//
//   k_density / k_loss_grad   uniformity loss L = mean_{i moving} (rho_i/rho0 - 1)^2,
//                             rho_i = W(0) + sum_{j: pred(i,j)} W(r_ij) over all classes,
//                             and dL/dx (gather form, no atomics)
//   k_step_adjoint            one step's adjoint through the projection and the
//                             tangential displacement, with the FP64 derivatives of
//                             x' with respect to the owner facets' vertices
//   k_fixed_adjoint           the positions of particles that do not move as functions
//                             of the mesh (singular point = its vertex, feature particle
//                             at arc length u of its segment)
//   k_permute                 carries adjoint rows between the sort orders of steps
//
// Vertex gradients are accumulated as 64-bit fixed point (2^-40 units) with
// integer atomics: integer addition is associative, so the sums do not depend
// on the order of the atomics (deterministic), and converted to double at the
// end. Their range is |sum| < 2^23; leaving it raises FPPG_S_FIXED_RANGE.
#include "stencil.h"

#include <cmath>

namespace fppg {

constexpr double kFixScale = 1099511627776.0;   // 2^40
constexpr double kFixLimit = 8388608.0;         // 2^23: 2^63 units of 2^-40

// One contribution to a fixed-point sum. A contribution of magnitude 2^23 or
// more is dropped, and a signed overflow of the running sum is detected from
// the value the atomic returns; both raise FPPG_S_FIXED_RANGE. The overflow
// test sees the partial sums in the order the atomics took, so it can also
// fire when only a partial sum left the range (conservative).
__device__ __forceinline__ void fix_add(unsigned long long* __restrict__ acc, int idx, double v, uint32_t* status) {
  if (v == 0.0) return;
  if (!(fabs(v) < kFixLimit)) {
    atomicOr(status, FPPG_S_FIXED_RANGE);
    return;
  }
  const long long inc = llrint(v * kFixScale);
  const long long old = (long long)atomicAdd(&acc[idx], (unsigned long long)inc);
  const long long sum = (long long)((unsigned long long)old + (unsigned long long)inc);
  if (((old ^ sum) & (inc ^ sum)) < 0) atomicOr(status, FPPG_S_FIXED_RANGE);
}

__device__ __forceinline__ void fix_add3(unsigned long long* __restrict__ acc, uint32_t* status, int vert, double x,
                                         double y, double z) {
  if (vert < 0) return;
  fix_add(acc, 3 * vert, x, status);
  fix_add(acc, 3 * vert + 1, y, status);
  fix_add(acc, 3 * vert + 2, z, status);
}

// ---- uniformity loss -----------------------------------------------------------------------

template <int K>
__global__ __launch_bounds__(kBlock) void k_density(const float4* __restrict__ pos, int n, const int* __restrict__ cs,
                                                    const GeomDev* __restrict__ geoms, int n_geom, uint32_t move_mask,
                                                    double rho0, double* __restrict__ rho,
                                                    double* __restrict__ partial_loss, double* __restrict__ partial_cnt) {
  const int i = xcd_chunk(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  double l = 0.0, c = 0.0;
  if (i < n) {
    const float4 p = pos[i];
    const GeomDev& G = geoms[min(geom_of(p.w), n_geom - 1)];
    const double h = G.h;
    const double alpha = 21.0 / (16.0 * M_PI * h * h * h);
    const float rc2 = G.rc2;
    double s = alpha;   // W(0)
    if (isfinite(p.x) && isfinite(p.y) && isfinite(p.z)) {
      for_each_source<K>(stencil_of(p, G), G, cs, pos, [&](int j, const float4 q) {
        if (!(pair_d2(p.x - q.x, p.y - q.y, p.z - q.z) < rc2) || j == i) return;
        const double dx = double(p.x) - double(q.x), dy = double(p.y) - double(q.y), dz = double(p.z) - double(q.z);
        const double qq = sqrt(dx * dx + dy * dy + dz * dz) / h;
        const double t = fmax(1.0 - 0.5 * qq, 0.0);
        s += alpha * (t * t) * (t * t) * (2.0 * qq + 1.0);
      });
    }
    rho[i] = s;
    if (is_moving(tag_of(p.w), move_mask)) {
      const double e = s / rho0 - 1.0;
      l = e * e;
      c = 1.0;
    }
  }
  const double tl = block_sum256(l);
  const double tc = block_sum256(c);
  if (threadIdx.x == 0) {
    partial_loss[blockIdx.x] = tl;
    partial_cnt[blockIdx.x] = tc;
  }
}

// dL/dx_k = sum_{j in N(k)} (g_k [k moves] + g_j [j moves]) W'(r_kj) e_kj,  g_i = 2 (rho_i/rho0 - 1) / (rho0 N)
// with W'(r) e = -K (1 - q/2)^3 (x_k - x_j), K = 5 alpha / h^2.
template <int K>
__global__ __launch_bounds__(kBlock) void k_loss_grad(const float4* __restrict__ pos, int n, const int* __restrict__ cs,
                                                      const GeomDev* __restrict__ geoms, int n_geom, uint32_t move_mask,
                                                      double rho0, const double* __restrict__ rho,
                                                      const double* __restrict__ stats, float4* __restrict__ grad) {
  const int i = xcd_chunk(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 p = pos[i];
  const GeomDev& G = geoms[min(geom_of(p.w), n_geom - 1)];
  const double cnt = fmax(stats[1], 1.0);
  const double scale = 2.0 / (rho0 * cnt);
  const double gi = is_moving(tag_of(p.w), move_mask) ? scale * (rho[i] / rho0 - 1.0) : 0.0;
  const double h = G.h;
  const double Kc = 105.0 / (16.0 * M_PI * h * h * h * h * h);
  const float rc2 = G.rc2;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  if (isfinite(p.x) && isfinite(p.y) && isfinite(p.z)) {
    for_each_source<K>(stencil_of(p, G), G, cs, pos, [&](int j, const float4 q) {
      if (!(pair_d2(p.x - q.x, p.y - q.y, p.z - q.z) < rc2) || j == i) return;
      const double gj = is_moving(tag_of(q.w), move_mask) ? scale * (rho[j] / rho0 - 1.0) : 0.0;
      const double dx = double(p.x) - double(q.x), dy = double(p.y) - double(q.y), dz = double(p.z) - double(q.z);
      const double t = fmax(1.0 - 0.5 * sqrt(dx * dx + dy * dy + dz * dz) / h, 0.0);
      const double f = -(gi + gj) * Kc * t * t * t;
      gx += f * dx;
      gy += f * dy;
      gz += f * dz;
    });
  }
  grad[i] = make_float4(float(gx), float(gy), float(gz), 0.0f);
}

// ---- one step's adjoint ------------------------------------------------------------------

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// Given the adjoint nbar of a facet's unit normal, add the vertex adjoints.
__device__ __forceinline__ void normal_to_vertices(const FacetDev& F, int4 tv, const double nbar[3],
                                                   unsigned long long* __restrict__ vbar, uint32_t* status,
                                                   double extraA[3]) {
  double N[3];
  cross3(F.e0, F.e1, N);
  const double len = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
  const double nn = F.n[0] * nbar[0] + F.n[1] * nbar[1] + F.n[2] * nbar[2];
  double Nbar[3];
  for (int q = 0; q < 3; ++q) Nbar[q] = (nbar[q] - F.n[q] * nn) / len;
  double e0b[3], e1b[3];
  cross3(F.e1, Nbar, e0b);   // dN = de0 x e1 + e0 x de1
  cross3(Nbar, F.e0, e1b);
  fix_add3(vbar, status, tv.x, extraA[0] - e0b[0] - e1b[0], extraA[1] - e0b[1] - e1b[1], extraA[2] - e0b[2] - e1b[2]);
  fix_add3(vbar, status, tv.y, e0b[0], e0b[1], e0b[2]);
  fix_add3(vbar, status, tv.z, e1b[0], e1b[1], e1b[2]);
}

__global__ __launch_bounds__(kBlock) void k_step_adjoint(
    const float4* __restrict__ pos, const uint8_t* __restrict__ accepted, const int* __restrict__ owner,
    const int* __restrict__ owner_next, const float4* __restrict__ accel, const float* __restrict__ amax, int n,
    int n_tri, const GeomDev* __restrict__ geoms, int n_geom, const FacetDev* __restrict__ facets,
    const int4* __restrict__ tri_vert, const int* __restrict__ fseg_before, const int* __restrict__ fseg_after,
    const double* __restrict__ fu_after, int n_feat, int n_seg, const SegDev* __restrict__ segs,
    const int2* __restrict__ seg_vert, uint32_t move_mask, const float4* __restrict__ xbar_next,
    float4* __restrict__ ybar, float4* __restrict__ xbar, unsigned long long* __restrict__ vbar, uint32_t* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 p = pos[i];
  const float4 xb = xbar_next[i];
  const int tag = tag_of(p.w);
  const bool reverted = accepted[i] == 0;
  float4 yb_out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  float4 xb_out = xb;
  if (is_moving(tag, move_mask) && !reverted) {
    const int g = min(geom_of(p.w), n_geom - 1);
    const double tau = amax[g] > 0.0f ? (double(geoms[g].h) * 0.0625) / double(amax[g]) : 0.0;
    if (tag == FPPG_TAG_FEATURE) {
      const int slot = owner[i];
      const int s0 = (slot >= 0 && slot < n_feat) ? fseg_before[slot] : -1;
      const int s2 = (slot >= 0 && slot < n_feat) ? fseg_after[slot] : -1;
      if (s0 >= 0 && s0 < n_seg && s2 >= 0 && s2 < n_seg) {
        const SegDev A = segs[s0], B = segs[s2];
        const float4 a4 = accel[i];
        const double a[3] = {a4.x, a4.y, a4.z};
        // x' = P0_s2 + u' t_s2 with u' = u + dt^2 a.t_s0 + c and u = t_s0.(x - P0_s0)
        const double gu = B.t[0] * xb.x + B.t[1] * xb.y + B.t[2] * xb.z;   // adjoint of u'
        const double u2 = fu_after[slot];
        {
          const double w[3] = {u2 * xb.x, u2 * xb.y, u2 * xb.z};             // adjoint of t_s2
          const double wt = w[0] * B.t[0] + w[1] * B.t[1] + w[2] * B.t[2];
          double d[3];
          for (int q = 0; q < 3; ++q) d[q] = (w[q] - wt * B.t[q]) / B.len;
          const int2 sv = seg_vert[s2];
          fix_add3(vbar, status, sv.y, d[0], d[1], d[2]);
          fix_add3(vbar, status, sv.x, xb.x - d[0], xb.y - d[1], xb.z - d[2]);
        }
        {
          // t_s0 through du = dt^2 a.t_s0, and P0_s0 through u = t_s0.(x - P0_s0)
          const double w[3] = {tau * gu * a[0], tau * gu * a[1], tau * gu * a[2]};
          const double wt = w[0] * A.t[0] + w[1] * A.t[1] + w[2] * A.t[2];
          double d[3];
          for (int q = 0; q < 3; ++q) d[q] = (w[q] - wt * A.t[q]) / A.len;
          const int2 sv = seg_vert[s0];
          fix_add3(vbar, status, sv.y, d[0], d[1], d[2]);
          fix_add3(vbar, status, sv.x, -d[0] - gu * A.t[0], -d[1] - gu * A.t[1], -d[2] - gu * A.t[2]);
        }
        if (s2 != s0) {
          // the walk's direction, recomputed as the forward computed du
          const float am = amax[g];
          const float tauf = am > 0.0f ? (geoms[g].h * 0.0625f) / am : 0.0f;
          const double du = double(tauf * a4.x) * A.t[0] + double(tauf * a4.y) * A.t[1] + double(tauf * a4.z) * A.t[2];
          const bool fwd = du > 0.0;
          int k = s0;
          for (int guard = 0; k != s2 && guard <= A.hi - A.lo; ++guard) {
            if (!fwd) k = k > A.lo ? k - 1 : (A.closed ? A.hi - 1 : -1);
            if (k < 0) break;
            // u' -= L_k (walked off forwards) or += L_k (walked onto backwards); dL_k = t_k.(dP1 - dP0)
            const double sg = fwd ? -gu : gu;
            const SegDev C = segs[k];
            const int2 sv = seg_vert[k];
            fix_add3(vbar, status, sv.y, sg * C.t[0], sg * C.t[1], sg * C.t[2]);
            fix_add3(vbar, status, sv.x, -sg * C.t[0], -sg * C.t[1], -sg * C.t[2]);
            if (fwd) k = k + 1 < A.hi ? k + 1 : (A.closed ? A.lo : -1);
            if (k < 0) break;
          }
        }
        yb_out = make_float4(float(tau * gu * A.t[0]), float(tau * gu * A.t[1]), float(tau * gu * A.t[2]), 0.0f);
        xb_out = make_float4(float(gu * A.t[0]), float(gu * A.t[1]), float(gu * A.t[2]), 0.0f);
      }
    } else if (tag == FPPG_TAG_VOLUME) {
      yb_out = make_float4(float(tau * xb.x), float(tau * xb.y), float(tau * xb.z), 0.0f);
    } else {
      const int o = owner[i], t = owner_next[i];
      if (o >= 0 && o < n_tri && t >= 0 && t < n_tri) {
        const FacetDev& Fo = facets[o];
        const FacetDev& Ft = facets[t];
        const float4 a4 = accel[i];
        const double a[3] = {a4.x, a4.y, a4.z};
        const double an = a[0] * Fo.n[0] + a[1] * Fo.n[1] + a[2] * Fo.n[2];
        const double y[3] = {double(p.x) + tau * (a[0] - an * Fo.n[0]), double(p.y) + tau * (a[1] - an * Fo.n[1]),
                             double(p.z) + tau * (a[2] - an * Fo.n[2])};
        const double xbv[3] = {xb.x, xb.y, xb.z};
        // projection onto facet t: x' = y - d n, d = (y - A) . n
        const double nx = Ft.n[0] * xbv[0] + Ft.n[1] * xbv[1] + Ft.n[2] * xbv[2];
        double ym[3], yb[3];
        for (int q = 0; q < 3; ++q) {
          ym[q] = y[q] - Ft.a[q];
          yb[q] = xbv[q] - Ft.n[q] * nx;
        }
        const double d = ym[0] * Ft.n[0] + ym[1] * Ft.n[1] + ym[2] * Ft.n[2];
        double nbar_t[3], Adir[3];
        for (int q = 0; q < 3; ++q) {
          nbar_t[q] = -d * xbv[q] - ym[q] * nx;
          Adir[q] = Ft.n[q] * nx;
        }
        normal_to_vertices(Ft, tri_vert[t], nbar_t, vbar, status, Adir);
        // tangential displacement with the owner normal: y = x + tau (a - (a.n) n)
        const double ny = Fo.n[0] * yb[0] + Fo.n[1] * yb[1] + Fo.n[2] * yb[2];
        double nbar_o[3], zero[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < 3; ++q) nbar_o[q] = -tau * (a[q] * ny + an * yb[q]);
        normal_to_vertices(Fo, tri_vert[o], nbar_o, vbar, status, zero);
        yb_out = make_float4(float(tau * (yb[0] - Fo.n[0] * ny)), float(tau * (yb[1] - Fo.n[1] * ny)),
                             float(tau * (yb[2] - Fo.n[2] * ny)), 0.0f);
        xb_out = make_float4(float(yb[0]), float(yb[1]), float(yb[2]), 0.0f);
      }
    }
  }
  ybar[i] = yb_out;
  xbar[i] = xb_out;
}

__global__ __launch_bounds__(kBlock) void k_fixed_adjoint(const float4* __restrict__ pos, const int* __restrict__ owner,
                                                          const int* __restrict__ feat_seg,
                                                          const double* __restrict__ feat_u, int n, int n_feat,
                                                          int n_seg, int n_vert, const SegDev* __restrict__ segs,
                                                          const int2* __restrict__ seg_vert, uint32_t move_mask,
                                                          const float4* __restrict__ xbar,
                                                          unsigned long long* __restrict__ vbar, uint32_t* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int tag = tag_of(pos[i].w);
  // singular points never move; every feature particle starts on its segment
  if (tag != FPPG_TAG_SINGULAR && tag != FPPG_TAG_FEATURE) return;
  const float4 xb = xbar[i];
  if (tag == FPPG_TAG_SINGULAR) {
    const int v = owner[i];
    if (v >= 0 && v < n_vert) fix_add3(vbar, status, v, xb.x, xb.y, xb.z);
  } else if (tag == FPPG_TAG_FEATURE) {
    const int slot = owner[i];
    const int s = (slot >= 0 && slot < n_feat) ? feat_seg[slot] : -1;
    if (s < 0 || s >= n_seg) return;
    const SegDev S = segs[s];
    const int2 sv = seg_vert[s];
    // x = P0 + u (P1 - P0)/|P1 - P0|:  dP1 = (u/L)(I - t t^T) xb,  dP0 = xb - dP1
    const double u = feat_u[slot];
    const double tx = S.t[0] * xb.x + S.t[1] * xb.y + S.t[2] * xb.z;
    const double c = u / S.len;
    const double p1[3] = {c * (xb.x - S.t[0] * tx), c * (xb.y - S.t[1] * tx), c * (xb.z - S.t[2] * tx)};
    fix_add3(vbar, status, sv.y, p1[0], p1[1], p1[2]);
    fix_add3(vbar, status, sv.x, xb.x - p1[0], xb.y - p1[1], xb.z - p1[2]);
  }
}

__global__ __launch_bounds__(kBlock) void k_permute(const float4* __restrict__ src, const int* __restrict__ index, int n,
                                                    int scatter, float4* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = index[i];
  if (j < 0 || j >= n) return;
  if (scatter) dst[j] = src[i];
  else dst[i] = src[j];
}

__global__ __launch_bounds__(kBlock) void k_fixed_to_double(const unsigned long long* __restrict__ in, int n,
                                                            double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = double((long long)in[i]) / kFixScale;
}

// out = {sum e^2, N}  ->  {sum e^2 / N, N}
__global__ void k_scale_loss(double* out) { out[0] = out[0] / fmax(out[1], 1.0); }

static inline int grid_for(int64_t n) { return int((n + kBlock - 1) / kBlock); }

}  // namespace fppg

using namespace fppg;

extern "C" fppg_status fppg_lattice_density(double dx, double h, double* out) {
  if (!out || !(dx > 0.0) || !(h > 0.0) || !std::isfinite(dx) || !std::isfinite(h)) return FPPG_E_ARG;
  const double m_real = std::ceil(2.0 * h / dx);
  if (m_real > 1024.0) return FPPG_E_ARG;   // (2m+1)^3 lattice points: keep the sum bounded
  const int m = int(m_real) + 1;
  const double alpha = 21.0 / (16.0 * M_PI * h * h * h);
  // Wendland C2 (Eq. 16-17): alpha (1 - q/2)^4 (2q + 1) for q = r/h < 2, summed
  // over the points (i, j, k) dx of the cubic lattice, the origin included
  double sum = 0.0;
  for (int i = -m; i <= m; ++i)
    for (int j = -m; j <= m; ++j)
      for (int k = -m; k <= m; ++k) {
        const double x = i * dx, y = j * dx, z = k * dx;
        const double q = std::sqrt(x * x + y * y + z * z) / h;
        if (q >= 2.0) continue;
        const double t = 1.0 - 0.5 * q;
        sum += alpha * (t * t) * (t * t) * (2.0 * q + 1.0);
      }
  *out = sum;
  return FPPG_OK;
}

extern "C" fppg_status fppg_uniformity_loss(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                            const int32_t* cell_start, uint32_t move_mask, double rho0, double* out,
                                            float* grad, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !geom) return fail(ctx, FPPG_E_ARG, "null ctx/geom");
  if (geom->has_levels)
    return fail(ctx, FPPG_E_UNSUPPORTED, "the uniformity loss of a multi-resolution geometry is not supported");
  if (n != geom->n_active || n < 1) return fail(ctx, FPPG_E_ARG, "n differs from the active particle count of the geometry");
  if (!pos || !cell_start || !out || !ws || !aligned(pos, 16) || !aligned(ws, 256) || (grad && !aligned(grad, 16)))
    return fail(ctx, FPPG_E_ARG, "null or misaligned argument");
  if (!(rho0 > 0.0)) return fail(ctx, FPPG_E_ARG, "rho0 must be > 0");
  const int nb = grid_for(n);
  const size_t need = size_t(n) * 8 + 2 * size_t(nb) * 8 + 64;
  if (ws_bytes < need) return fail(ctx, FPPG_E_WORKSPACE, "workspace too small for uniformity_loss");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* rho = static_cast<double*>(ws);
  double* pl = rho + n;
  double* pc = pl + nb;
  const float4* p4 = reinterpret_cast<const float4*>(pos);
  if (geom->k == 1) k_density<1><<<nb, kBlock, 0, s>>>(p4, int(n), cell_start, geom->d_geom, geom->n_geom, move_mask, rho0, rho, pl, pc);
  else k_density<2><<<nb, kBlock, 0, s>>>(p4, int(n), cell_start, geom->d_geom, geom->n_geom, move_mask, rho0, rho, pl, pc);
  FPPG_HIP(ctx, hipGetLastError());
  fppg_status st = sum_partials(ctx, pl, nb, out, s);
  if (st != FPPG_OK) return st;
  st = sum_partials(ctx, pc, nb, out + 1, s);
  if (st != FPPG_OK) return st;
  k_scale_loss<<<1, 1, 0, s>>>(out);
  if (grad) {
    float4* g4 = reinterpret_cast<float4*>(grad);
    if (geom->k == 1) k_loss_grad<1><<<nb, kBlock, 0, s>>>(p4, int(n), cell_start, geom->d_geom, geom->n_geom, move_mask, rho0, rho, out, g4);
    else k_loss_grad<2><<<nb, kBlock, 0, s>>>(p4, int(n), cell_start, geom->d_geom, geom->n_geom, move_mask, rho0, rho, out, g4);
  }
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

extern "C" fppg_status fppg_step_adjoint(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                         const uint8_t* accepted, const int32_t* owner, const int32_t* owner_next,
                                         const float* accel, const float* amax, const int32_t* fseg_before,
                                         const int32_t* fseg_after, const double* fu_after, int32_t n_feat,
                                         uint32_t move_mask, const float* xbar_next, float* ybar, float* xbar,
                                         int64_t* vbar_fixed, void* stream) {
  if (!ctx || !geom) return fail(ctx, FPPG_E_ARG, "null ctx/geom");
  if (n != geom->n_active) return fail(ctx, FPPG_E_ARG, "n differs from the active particle count of the geometry");
  if (n_feat < 0 || (n_feat > 0 && (!fseg_before || !fseg_after || !fu_after)))
    return fail(ctx, FPPG_E_ARG, "bad feature tables");
  if (n > 0 && (!pos || !accepted || !owner || !owner_next || !accel || !amax || !xbar_next || !ybar || !xbar ||
                !vbar_fixed))
    return fail(ctx, FPPG_E_ARG, "null argument");
  if (!aligned(pos, 16) || !aligned(accel, 16) || !aligned(xbar_next, 16) ||
      !aligned(ybar, 16) || !aligned(xbar, 16))
    return fail(ctx, FPPG_E_ARG, "misaligned argument");
  if (n > 0 && xbar == xbar_next) return fail(ctx, FPPG_E_ARG, "xbar must not alias xbar_next");
  if (n == 0) return FPPG_OK;
  k_step_adjoint<<<grid_for(n), kBlock, 0, static_cast<hipStream_t>(stream)>>>(
      reinterpret_cast<const float4*>(pos), accepted, owner, owner_next,
      reinterpret_cast<const float4*>(accel), amax, int(n), int(geom->n_tri), geom->d_geom, geom->n_geom,
      geom->d_facet, geom->d_tri_vert, fseg_before, fseg_after, fu_after, n_feat, int(geom->n_seg), geom->d_seg,
      geom->d_seg_vert, move_mask, reinterpret_cast<const float4*>(xbar_next),
      reinterpret_cast<float4*>(ybar), reinterpret_cast<float4*>(xbar),
      reinterpret_cast<unsigned long long*>(vbar_fixed), ctx->d_status);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

extern "C" fppg_status fppg_fixed_adjoint(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                          const int32_t* owner, const int32_t* feat_seg, const double* feat_u,
                                          int32_t n_feat, uint32_t move_mask, const float* xbar, int64_t* vbar_fixed,
                                          void* stream) {
  if (!ctx || !geom) return fail(ctx, FPPG_E_ARG, "null ctx/geom");
  if (n != geom->n_active) return fail(ctx, FPPG_E_ARG, "n differs from the active particle count of the geometry");
  if (n > 0 && (!pos || !owner || !xbar || !vbar_fixed)) return fail(ctx, FPPG_E_ARG, "null argument");
  if (n_feat < 0 || (n_feat > 0 && (!feat_seg || !feat_u))) return fail(ctx, FPPG_E_ARG, "bad feature table");
  if (!aligned(pos, 16) || !aligned(xbar, 16)) return fail(ctx, FPPG_E_ARG, "misaligned argument");
  if (n == 0) return FPPG_OK;
  k_fixed_adjoint<<<grid_for(n), kBlock, 0, static_cast<hipStream_t>(stream)>>>(
      reinterpret_cast<const float4*>(pos), owner, feat_seg, feat_u, int(n), n_feat, int(geom->n_seg),
      int(geom->n_vert), geom->d_seg, geom->d_seg_vert, move_mask, reinterpret_cast<const float4*>(xbar),
      reinterpret_cast<unsigned long long*>(vbar_fixed), ctx->d_status);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

extern "C" fppg_status fppg_vec_permute(fppg_ctx* ctx, int64_t n, const float* src, const int32_t* index,
                                        int32_t scatter, float* dst, void* stream) {
  if (!ctx) return FPPG_E_ARG;
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(ctx, FPPG_E_ARG, "n out of range");
  if (n > 0 && (!src || !index || !dst)) return fail(ctx, FPPG_E_ARG, "null argument");
  if (!aligned(src, 16) || !aligned(dst, 16) || (n > 0 && src == dst)) return fail(ctx, FPPG_E_ARG, "misaligned or aliased");
  if (n == 0) return FPPG_OK;
  k_permute<<<grid_for(n), kBlock, 0, static_cast<hipStream_t>(stream)>>>(
      reinterpret_cast<const float4*>(src), index, int(n), scatter ? 1 : 0, reinterpret_cast<float4*>(dst));
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

extern "C" fppg_status fppg_fixed_to_double(fppg_ctx* ctx, int64_t count, const int64_t* in, double* out,
                                            void* stream) {
  if (!ctx) return FPPG_E_ARG;
  if (count < 0 || count >= (int64_t(1) << 31) || (count > 0 && (!in || !out)))
    return fail(ctx, FPPG_E_ARG, "bad argument");
  if (count == 0) return FPPG_OK;
  k_fixed_to_double<<<grid_for(count), kBlock, 0, static_cast<hipStream_t>(stream)>>>(
      reinterpret_cast<const unsigned long long*>(in), int(count), out);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

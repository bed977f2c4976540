// Vector kernels for Newton-Krylov relaxation on particle fields (float4
// arrays, x/y/z used, w ignored): FP64 dot products with a fixed summation
// order (deterministic), y = alpha x + beta y, projection onto the tangent
// spaces of the constrained particles, and the conversion of a direction into
// the displacement format of fppg_project.
#include "internal.h"

namespace fppg {

constexpr int kRedBlock = 256;   // block_sum256 assumes 256 threads

__global__ __launch_bounds__(kRedBlock) void k_dot_partial(const float4* __restrict__ a, const float4* __restrict__ b,
                                                           int n, int per_block, double* __restrict__ partial) {
  const int base = blockIdx.x * per_block;
  const int end = min(n, base + per_block);
  double s = 0.0;
  for (int i = base + threadIdx.x; i < end; i += kRedBlock) {
    const float4 x = a[i], y = b[i];
    s += double(x.x) * double(y.x) + double(x.y) * double(y.y) + double(x.z) * double(y.z);
  }
  const double t = block_sum256(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(kRedBlock) void k_sum_partials(const double* __restrict__ partial, int nb,
                                                            double* __restrict__ out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += kRedBlock) s += partial[i];
  const double t = block_sum256(s);
  if (threadIdx.x == 0) *out = t;
}

__global__ __launch_bounds__(kBlock) void k_axpby(int n, float alpha, const float4* __restrict__ x, float beta,
                                                  float4* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // beta = 0 ignores the old y and alpha = 0 ignores x (BLAS convention), so
  // uninitialised memory, NaN included, never leaks into the result
  float4 b = beta != 0.0f ? y[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const float4 a = alpha != 0.0f ? x[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  b.x = fmaf(alpha, a.x, beta * b.x);
  b.y = fmaf(alpha, a.y, beta * b.y);
  b.z = fmaf(alpha, a.z, beta * b.z);
  y[i] = b;
}

// v <- P v (tangent_apply, internal.h).
__global__ __launch_bounds__(kBlock) void k_tangent(const float4* __restrict__ pos, const int* __restrict__ owner,
                                                    const int* __restrict__ feat_seg, int n, int n_feat, int n_tri,
                                                    int n_seg, const float4* __restrict__ n32,
                                                    const SegDev* __restrict__ segs, uint32_t move_mask,
                                                    float4* __restrict__ v, uint32_t* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  v[i] = tangent_apply(v[i], tag_of(pos[i].w), i, move_mask, owner, feat_seg, n_feat, n_tri, n_seg, n32, segs,
                       status);
}

// out = a x + b y + c z (a term with a zero coefficient is not read), then
// acc += phi out when acc is given: the direction and iterate updates of MINRES.
__global__ __launch_bounds__(kBlock) void k_combine3(int n, float a, const float4* __restrict__ x, float b,
                                                     const float4* __restrict__ y, float c,
                                                     const float4* __restrict__ z, float4* __restrict__ out,
                                                     float phi, float4* __restrict__ acc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 zero = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const float4 X = a != 0.0f ? x[i] : zero, Y = b != 0.0f ? y[i] : zero, Z = c != 0.0f ? z[i] : zero;
  float4 o;
  o.x = fmaf(c, Z.x, fmaf(b, Y.x, a * X.x));
  o.y = fmaf(c, Z.y, fmaf(b, Y.y, a * X.y));
  o.z = fmaf(c, Z.z, fmaf(b, Y.z, a * X.z));
  o.w = 0.0f;
  out[i] = o;
  if (acc) {
    float4 s = acc[i];
    s.x = fmaf(phi, o.x, s.x);
    s.y = fmaf(phi, o.y, s.y);
    s.z = fmaf(phi, o.z, s.z);
    acc[i] = s;
  }
}

// disp = alpha P v in the format of fppg_project (feature: FP64 du = alpha v.t).
__global__ __launch_bounds__(kBlock) void k_displace(const float4* __restrict__ pos, const int* __restrict__ owner,
                                                     const int* __restrict__ feat_seg, int n, int n_feat, int n_tri,
                                                     int n_seg, const float4* __restrict__ n32,
                                                     const SegDev* __restrict__ segs, uint32_t move_mask,
                                                     const float4* __restrict__ v, float alpha,
                                                     float4* __restrict__ disp, uint32_t* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int tag = tag_of(pos[i].w);
  float4 d = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (is_moving(tag, move_mask)) {
    const float4 x = v[i];
    float rx = alpha * x.x, ry = alpha * x.y, rz = alpha * x.z;
    if (tag == FPPG_TAG_SURFACE) {
      const int o = owner[i];
      if (o < 0 || o >= n_tri) {
        atomicOr(status, FPPG_S_BAD_INDEX);
        rx = ry = rz = 0.0f;
      } else {
        const float4 nn = n32[o];
        const float s = rx * nn.x + ry * nn.y + rz * nn.z;
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

static inline int grid_for(int64_t n) { return int((n + kBlock - 1) / kBlock); }

__global__ void k_zero_u32(unsigned* __restrict__ a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0u;
}

// Scratch of fppg_vec_dot_noalloc: the per-block partial sums of one dot
// product, in a static device array (each device holds its own copy for the
// life of the process). Host code never passes `scratch` itself to a kernel
// (its host-side name is not a device address): init_dot_scratch resolves the
// device address once per context, with the context's device current.
static __device__ __align__(256) double scratch[kDotPartials];

fppg_status init_dot_scratch(fppg_ctx* ctx) {
  void* p = nullptr;
  FPPG_HIP(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) return fail(ctx, FPPG_E_HIP, "static dot-product scratch has no device address");
  ctx->dot_scratch = static_cast<double*>(p);
  return FPPG_OK;
}

fppg_status sum_partials(fppg_ctx* ctx, const double* partial, int nb, double* out, hipStream_t s) {
  k_sum_partials<<<1, kRedBlock, 0, s>>>(partial, nb, out);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

// Deterministic FP64 dot over n float4 rows into out[0] (device).
fppg_status dot_into(fppg_ctx* ctx, int n, const float4* a, const float4* b, double* out, double* partial,
                     int max_blocks, hipStream_t s) {
  int nb = std::max(1, std::min(max_blocks, (n + kRedBlock * 8 - 1) / (kRedBlock * 8)));
  const int per_block = (n + nb - 1) / nb;
  if (n > 0) nb = (n + per_block - 1) / per_block;
  k_dot_partial<<<nb, kRedBlock, 0, s>>>(a, b, n, per_block, partial);
  k_sum_partials<<<1, kRedBlock, 0, s>>>(partial, n > 0 ? nb : 1, out);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

}  // namespace fppg

using namespace fppg;

extern "C" fppg_status fppg_vec_dot(fppg_ctx* ctx, int64_t n, const float* a, const float* b, double* out, void* ws,
                                    size_t ws_bytes, void* stream) {
  if (!ctx) return FPPG_E_ARG;
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(ctx, FPPG_E_ARG, "n out of range");
  if (!out || !ws || (n > 0 && (!a || !b))) return fail(ctx, FPPG_E_ARG, "null argument");
  if (!aligned(a, 16) || !aligned(b, 16) || !aligned(ws, 256)) return fail(ctx, FPPG_E_ARG, "misaligned argument");
  if (ws_bytes < kDotPartials * sizeof(double)) return fail(ctx, FPPG_E_WORKSPACE, "workspace too small for vec_dot");
  if (n == 0) {
    double* p = static_cast<double*>(ws);
    k_sum_partials<<<1, kRedBlock, 0, static_cast<hipStream_t>(stream)>>>(p, 0, out);
    FPPG_HIP(ctx, hipGetLastError());
    return FPPG_OK;
  }
  return dot_into(ctx, int(n), reinterpret_cast<const float4*>(a), reinterpret_cast<const float4*>(b), out,
                  static_cast<double*>(ws), kDotPartials, static_cast<hipStream_t>(stream));
}

extern "C" fppg_status fppg_vec_dot_noalloc(fppg_ctx* ctx, int64_t n, const float* a, const float* b, double* out,
                                            void* stream) {
  if (!ctx) return FPPG_E_ARG;
  if (!ctx->dot_scratch) return fail(ctx, FPPG_E_HIP, "context has no dot-product scratch");
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(ctx, FPPG_E_ARG, "n out of range (0 <= n < 2^31)");
  if (!out || (n > 0 && (!a || !b))) return fail(ctx, FPPG_E_ARG, "null argument");
  if (!aligned(a, 16) || !aligned(b, 16)) return fail(ctx, FPPG_E_ARG, "misaligned argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n == 0) {   // no partial is read: the sum over none is 0
    k_sum_partials<<<1, kRedBlock, 0, s>>>(ctx->dot_scratch, 0, out);
    FPPG_HIP(ctx, hipGetLastError());
    return FPPG_OK;
  }
  // the same kernels and block partition as fppg_vec_dot (at most kDotPartials
  // blocks, every partial written before it is summed), with the partials in
  // the static scratch: the result is bitwise that of fppg_vec_dot
  return dot_into(ctx, int(n), reinterpret_cast<const float4*>(a), reinterpret_cast<const float4*>(b), out,
                  ctx->dot_scratch, kDotPartials, s);
}

extern "C" fppg_status fppg_vec_axpby(fppg_ctx* ctx, int64_t n, float alpha, const float* x, float beta, float* y,
                                      void* stream) {
  if (!ctx) return FPPG_E_ARG;
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(ctx, FPPG_E_ARG, "n out of range");
  if (n > 0 && (!x || !y)) return fail(ctx, FPPG_E_ARG, "null argument");
  if (!aligned(x, 16) || !aligned(y, 16)) return fail(ctx, FPPG_E_ARG, "misaligned argument");
  if (n == 0) return FPPG_OK;
  k_axpby<<<grid_for(n), kBlock, 0, static_cast<hipStream_t>(stream)>>>(int(n), alpha, reinterpret_cast<const float4*>(x),
                                                                         beta, reinterpret_cast<float4*>(y));
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

__global__ __launch_bounds__(kBlock) void k_clamp(float4* __restrict__ v, int n, float cap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float4 x = v[i];
  const float m = sqrtf(x.x * x.x + x.y * x.y + x.z * x.z);
  if (m > cap) {
    const float s = cap / m;
    x.x *= s;
    x.y *= s;
    x.z *= s;
    v[i] = x;
  }
}

extern "C" fppg_status fppg_vec_clamp(fppg_ctx* ctx, int64_t n, float* v, float cap, void* stream) {
  if (!ctx) return FPPG_E_ARG;
  if (n < 0 || n >= (int64_t(1) << 31) || !(cap > 0.0f)) return fail(ctx, FPPG_E_ARG, "bad n or cap");
  if (n > 0 && (!v || !aligned(v, 16))) return fail(ctx, FPPG_E_ARG, "null or misaligned argument");
  if (n == 0) return FPPG_OK;
  k_clamp<<<grid_for(n), kBlock, 0, static_cast<hipStream_t>(stream)>>>(reinterpret_cast<float4*>(v), int(n), cap);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

__global__ __launch_bounds__(kBlock) void k_maxnorm(const float4* __restrict__ a, int n, unsigned* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float m = 0.0f;
  if (i < n) {
    const float4 x = a[i];
    m = sqrtf(x.x * x.x + x.y * x.y + x.z * x.z);
    if (!(m >= 0.0f)) m = INFINITY;   // NaN counts as unbounded
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0 && m > 0.0f) atomicMax(out, __float_as_uint(m));
}

extern "C" fppg_status fppg_vec_maxnorm(fppg_ctx* ctx, int64_t n, const float* a, float* out, void* stream) {
  if (!ctx) return FPPG_E_ARG;
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(ctx, FPPG_E_ARG, "n out of range");
  if (!out || (n > 0 && !a) || !aligned(a, 16)) return fail(ctx, FPPG_E_ARG, "null or misaligned argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  k_zero_u32<<<1, 64, 0, s>>>(reinterpret_cast<unsigned*>(out), 1);
  if (n > 0) k_maxnorm<<<grid_for(n), kBlock, 0, s>>>(reinterpret_cast<const float4*>(a), int(n), reinterpret_cast<unsigned*>(out));
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

extern "C" fppg_status fppg_tangent_project(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                            const int32_t* owner, const int32_t* feat_seg, int32_t n_feat,
                                            uint32_t move_mask, float* v, void* stream) {
  if (!ctx || !geom) return fail(ctx, FPPG_E_ARG, "null ctx/geom");
  if (n != geom->n_active) return fail(ctx, FPPG_E_ARG, "n differs from the active particle count of the geometry");
  if (n > 0 && (!pos || !owner || !v)) return fail(ctx, FPPG_E_ARG, "null argument");
  if (n_feat < 0 || (n_feat > 0 && !feat_seg)) return fail(ctx, FPPG_E_ARG, "bad feature table");
  if (!aligned(pos, 16) || !aligned(v, 16)) return fail(ctx, FPPG_E_ARG, "misaligned argument");
  if (n == 0) return FPPG_OK;
  k_tangent<<<grid_for(n), kBlock, 0, static_cast<hipStream_t>(stream)>>>(
      reinterpret_cast<const float4*>(pos), owner, feat_seg, int(n), n_feat, int(geom->n_tri), int(geom->n_seg),
      geom->d_n32, geom->d_seg, move_mask, reinterpret_cast<float4*>(v), ctx->d_status);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

extern "C" fppg_status fppg_vec_combine3(fppg_ctx* ctx, int64_t n, float a, const float* x, float b,
                                         const float* y, float c, const float* z, float* out, float phi,
                                         float* acc, void* stream) {
  if (!ctx) return FPPG_E_ARG;
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(ctx, FPPG_E_ARG, "n out of range");
  if (n > 0 && (!out || (a != 0.0f && !x) || (b != 0.0f && !y) || (c != 0.0f && !z)))
    return fail(ctx, FPPG_E_ARG, "null argument");
  if (!aligned(x, 16) || !aligned(y, 16) || !aligned(z, 16) || !aligned(out, 16) || !aligned(acc, 16))
    return fail(ctx, FPPG_E_ARG, "misaligned argument");
  if (n > 0 && (out == x || out == y || out == z || (acc && (acc == out || acc == x || acc == y || acc == z))))
    return fail(ctx, FPPG_E_ARG, "out and acc must not alias the inputs or each other");
  if (n == 0) return FPPG_OK;
  k_combine3<<<grid_for(n), kBlock, 0, static_cast<hipStream_t>(stream)>>>(
      int(n), a, reinterpret_cast<const float4*>(x), b, reinterpret_cast<const float4*>(y), c,
      reinterpret_cast<const float4*>(z), reinterpret_cast<float4*>(out), phi, reinterpret_cast<float4*>(acc));
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

extern "C" fppg_status fppg_displace(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                     const int32_t* owner, const int32_t* feat_seg, int32_t n_feat, uint32_t move_mask,
                                     const float* v, float alpha, float* disp, void* stream) {
  if (!ctx || !geom) return fail(ctx, FPPG_E_ARG, "null ctx/geom");
  if (n != geom->n_active) return fail(ctx, FPPG_E_ARG, "n differs from the active particle count of the geometry");
  if (n > 0 && (!pos || !owner || !v || !disp)) return fail(ctx, FPPG_E_ARG, "null argument");
  if (n_feat < 0 || (n_feat > 0 && !feat_seg)) return fail(ctx, FPPG_E_ARG, "bad feature table");
  if (!aligned(pos, 16) || !aligned(v, 16) || !aligned(disp, 16)) return fail(ctx, FPPG_E_ARG, "misaligned argument");
  if (n == 0) return FPPG_OK;
  k_displace<<<grid_for(n), kBlock, 0, static_cast<hipStream_t>(stream)>>>(
      reinterpret_cast<const float4*>(pos), owner, feat_seg, int(n), n_feat, int(geom->n_tri), int(geom->n_seg),
      geom->d_n32, geom->d_seg, move_mask, reinterpret_cast<const float4*>(v), alpha, reinterpret_cast<float4*>(disp),
      ctx->d_status);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

// Relaxation force + amax (Eq. 15-17) and the displacement update (Eq. 22-25).
//
// One lane per sorted receiver over the culled stencil of stencil.h. Sources
// are summed in a fixed order (rows by dz then dy ascending, then sorted
// index): the sums are deterministic.
//
// The neighbour predicate is the binary32 expression
// fl32(fl32(fl32(dx*dx) + fl32(dy*dy)) + fl32(dz*dz)) < rc2; this file is
// compiled without floating-point contraction so that the compiler cannot fuse
// it, and the accumulations use explicit fmaf.
#include "stencil.h"

#include <algorithm>

namespace fppg {

__global__ void k_zero_f32(float* __restrict__ a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

// ---- forces + amax ---------------------------------------------------------------------

// One source: K-less pair term (1 - r/2h)^3 r_ij with 1 - r/2h clamped to
// [0, 1], which is zero at and beyond the support radius, so that the sum
// needs no neighbour test: a candidate beyond 2h adds exact zeros. Next to the
// sum over the predicate's neighbours (the binary32 test |r|^2 < fl32(2h)^2)
// it differs only by pairs within rounding of r = 2h, whose terms are below
// 2^-69 of a unit-distance term. r^2 is taken with two FMAs and the clamp is
// the FMA's output modifier: 14 VALU instructions per candidate.
// RANKED: sources of a class above the receiver's (tag_j > T; T = 7 for volume
// receivers, which take every class) add nothing. The receiver itself adds
// r = 0. COUNT: counts the predicate's neighbours (the receiver subtracted
// by the caller) for the pair statistics.
template <bool RANKED, bool COUNT>
__device__ __forceinline__ void add_pair(const float4 p, const float4 q, float rc2, float inv2h, uint32_t T,
                                         float& ax, float& ay, float& az, float& cnt) {
  const float dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
  const float t = __builtin_amdgcn_fmed3f(fmaf(-__builtin_amdgcn_sqrtf(r2), inv2h, 1.0f), 0.0f, 1.0f);
  float w = t * t * t;
  bool src = true;
  if (RANKED) {
    src = (__float_as_uint(q.w) & 7u) <= T;
    w = src ? w : 0.0f;
  }
  ax = fmaf(w, dx, ax);
  ay = fmaf(w, dy, ay);
  az = fmaf(w, dz, az);
  if (COUNT) cnt += (src && pair_d2(dx, dy, dz) < rc2) ? 1.0f : 0.0f;
}

// Multi-resolution pair term: the source's level l_j (pos.w bits 3-4) gives
// h_j = h 2^-l_j, the pair's support h_i + h_j = 2 h_ij, and the term is
// (h / h_ij)^5 (1 - r / 2h_ij)^3 r_ij, so that the geometry's K(h) applied at
// the end gives K(h_ij) per pair (K scales as h^-5). The predicate of the
// counting variant is |r|^2 < fl32(fl32(h_i + h_j)^2).
template <bool RANKED, bool COUNT>
__device__ __forceinline__ void add_pair_mr(const float4 p, const float4 q, float h, float hi, uint32_t T,
                                            float& ax, float& ay, float& az, float& cnt) {
  const float dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
  const int lj = int((__float_as_uint(q.w) >> 3) & 3u);
  const float hs = hi + ldexpf(h, -lj);
  const float inv = __builtin_amdgcn_rcpf(hs);
  const float t = __builtin_amdgcn_fmed3f(fmaf(-__builtin_amdgcn_sqrtf(r2), inv, 1.0f), 0.0f, 1.0f);
  const float ratio = (2.0f * h) * inv;
  const float ratio2 = ratio * ratio;
  float w = (t * t * t) * (ratio2 * ratio2 * ratio);
  bool src = true;
  if (RANKED) {
    src = (__float_as_uint(q.w) & 7u) <= T;
    w = src ? w : 0.0f;
  }
  ax = fmaf(w, dx, ax);
  ay = fmaf(w, dy, ay);
  az = fmaf(w, dz, az);
  if (COUNT) cnt += (src && pair_d2(dx, dy, dz) < hs * hs) ? 1.0f : 0.0f;
}

// The B receivers of chunk blk (launch slots blk * B ...): forces, and the
// chunk's contribution to amax. Called by every thread of a block.
template <int K, bool COUNT, int B, bool MR = false>
__device__ __forceinline__ void force_chunk(int blk, const float4* __restrict__ pos, int n,
                                            const int* __restrict__ cs, const GeomDev* __restrict__ geoms,
                                            int n_geom, uint32_t move_mask, float4* __restrict__ accel,
                                            unsigned* __restrict__ amax_bits, uint32_t* status,
                                            const int* __restrict__ list, int n_list) {
  const int i = listed(blk * B + threadIdx.x, n, list, n_list);
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
    if (MR) {
      // pairs of receiver i reach at most h_i + h = 2h (1 + 2^-l_i) / 2: the
      // stencil is culled to that radius, K (1 + 2^-l_i) / 2 cell edges
      const int li = int((__float_as_uint(p.w) >> 3) & 3u);
      const float hi = ldexpf(G.h, -li);
      const float rad = float(K) * (0.5f + ldexpf(0.5f, -li));
      if (ranked)
        for_each_source<K, true>(st, G, cs, pos, [&](int, const float4 q) { add_pair_mr<true, COUNT>(p, q, G.h, hi, T, ax, ay, az, cnt); }, rad * rad);
      else
        for_each_source<K, true>(st, G, cs, pos, [&](int, const float4 q) { add_pair_mr<false, COUNT>(p, q, G.h, hi, T, ax, ay, az, cnt); }, rad * rad);
    } else if (ranked)
      for_each_source<K, true>(st, G, cs, pos, [&](int, const float4 q) { add_pair<true, COUNT>(p, q, rc2, inv2h, T, ax, ay, az, cnt); });
    else
      for_each_source<K, true>(st, G, cs, pos, [&](int, const float4 q) { add_pair<false, COUNT>(p, q, rc2, inv2h, T, ax, ay, az, cnt); });
    ax *= G.kcoef;
    ay *= G.kcoef;
    az *= G.kcoef;
    if (COUNT) cnt -= 1.0f;   // the receiver itself
    anorm = sqrtf(ax * ax + ay * ay + az * az);
    // multi-resolution: amax takes |a_i| 2^l_i, so that dt^2 moves particle i at most h_i / 16
    if (MR) anorm = ldexpf(anorm, int((__float_as_uint(p.w) >> 3) & 3u));
    if (!isfinite(anorm)) {
      atomicOr(status, FPPG_S_NONFINITE_ACCEL);
      ax = ay = az = 0.0f;
      anorm = 0.0f;
    }
  }
  if (i < n) accel[i] = make_float4(ax, ay, az, cnt);
  // per-geometry max of |a|: wave max, block max, one atomic per block and geometry
  __shared__ float s_max[B / 64];
  __shared__ int s_geo[B / 64];
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
    for (int w = 0; w < B / 64; ++w) {
      float mm = s_max[w];
      if (!(mm > 0.0f)) continue;
      for (int w2 = w + 1; w2 < B / 64; ++w2)
        if (s_geo[w2] == s_geo[w]) {
          mm = fmaxf(mm, s_max[w2]);
          s_max[w2] = 0.0f;
        }
      atomicMax(&amax_bits[s_geo[w]], __float_as_uint(mm));
    }
  }
  __syncthreads();   // s_max / s_geo are reused by the block's next chunk
}

// One block per chunk of B receivers. remap: the XCD mapping of the blocks
// (launch_chunk: round-robin, one contiguous range per XCD, or runs of
// chunks). None changes a result (per-lane sums, max-reduced amax).
template <int K, bool COUNT, int B, bool MR = false>
__global__ __launch_bounds__(B) void k_force(const float4* __restrict__ pos, int n,
                                             const int* __restrict__ cs, const GeomDev* __restrict__ geoms,
                                             int n_geom, uint32_t move_mask, float4* __restrict__ accel,
                                             unsigned* __restrict__ amax_bits, uint32_t* status,
                                             const int* __restrict__ list, int n_list, int remap) {
  const int blk = launch_chunk(remap, int(blockIdx.x), int(gridDim.x));
  force_chunk<K, COUNT, B, MR>(blk, pos, n, cs, geoms, n_geom, move_mask, accel, amax_bits, status, list, n_list);
}

// Persistent schedule: a grid of resident blocks takes chunks by tickets.
// Block b starts on the ticket counter of XCD b % 8 (workgroups are dealt to
// the XCDs round-robin), which hands out that XCD's contiguous range of
// chunks, as xcd_chunk splits them; a block whose range is used up takes
// tickets from the next XCD's range, and so on, and leaves once all eight
// are used up (every block exits after at most nchunks + 8 ticket draws in
// all). tickets [8] must be zero at launch. Each chunk is processed exactly as
// by k_force, so the results are the same bit for bit.
template <int K, bool COUNT, int B>
__global__ __launch_bounds__(B) void k_force_tickets(const float4* __restrict__ pos, int n,
                                                     const int* __restrict__ cs, const GeomDev* __restrict__ geoms,
                                                     int n_geom, uint32_t move_mask, float4* __restrict__ accel,
                                                     unsigned* __restrict__ amax_bits, uint32_t* status,
                                                     const int* __restrict__ list, int n_list, int nchunks,
                                                     int* __restrict__ tickets) {
  __shared__ int s_chunk;
  const int q = nchunks / kNumXcd, r = nchunks % kNumXcd;
  const int home = int(blockIdx.x) % kNumXcd;
  int step = 0;   // ranges used up so far (thread 0)
  for (;;) {
    if (threadIdx.x == 0) {
      int c = -1;
      while (step < kNumXcd) {
        const int x = (home + step) % kNumXcd;
        const int t = atomicAdd(&tickets[x], 1);
        if (t < q + (x < r ? 1 : 0)) {
          c = x * q + min(x, r) + t;
          break;
        }
        ++step;
      }
      s_chunk = c;
    }
    __syncthreads();
    const int c = s_chunk;
    __syncthreads();
    if (c < 0) break;
    force_chunk<K, COUNT, B>(c, pos, n, cs, geoms, n_geom, move_mask, accel, amax_bits, status, list, n_list);
  }
}

__global__ void k_zero_tickets(int* __restrict__ t) {
  if (threadIdx.x < kNumXcd) t[threadIdx.x] = 0;
}

// ---- displacement (Eq. 22-25) ------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_update(const float4* __restrict__ pos, const float4* __restrict__ accel,
                                                   const int* __restrict__ owner, const int* __restrict__ feat_seg,
                                                   int n, int n_feat, int n_tri, int n_seg,
                                                   const GeomDev* __restrict__ geoms, int n_geom,
                                                   const float* __restrict__ amax, const float4* __restrict__ n32,
                                                   const SegDev* __restrict__ segs, uint32_t move_mask,
                                                   float4* __restrict__ disp, uint32_t* status,
                                                   const int* __restrict__ list, int n_list) {
  const int i = listed(blockIdx.x * blockDim.x + threadIdx.x, n, list, n_list);
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

static inline int grid_for(int64_t n) { return int((n + kBlock - 1) / kBlock); }

// Launch of the force kernel in the context's schedule: one block per chunk,
// or the persistent ticket schedule with as many resident blocks as fit.
struct ForceLaunch {
  int block;
  int remap;   // XCD mapping of the workgroups (launch_chunk)
  bool persistent;
  int* tickets;
  fppg_ctx* ctx;   // occupancy of the persistent kernel, queried once per context
};

template <int K, bool COUNT, int B>
static void launch_force_b(const ForceLaunch& fl, int nr, hipStream_t s, const float4* p4, int n, const int* cs,
                           const GeomDev* g, int n_geom, uint32_t mm, float4* acc, unsigned* ab, uint32_t* st,
                           const int* list) {
  const int nchunks = (nr + B - 1) / B;
  if (!fl.persistent) {
    k_force<K, COUNT, B><<<nchunks, B, 0, s>>>(p4, n, cs, g, n_geom, mm, acc, ab, st, list, nr, fl.remap);
    return;
  }
  int& per_cu = fl.ctx->resident[K - 1][B == 128 ? 0 : (B == 256 ? 1 : 2)];
  if (!per_cu) {   // queried outside graph capture too: host calls only, no stream work
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_force_tickets<K, COUNT, B>, B, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    hipDeviceProp_t prop;
    fl.ctx->num_cu = hipGetDeviceProperties(&prop, fl.ctx->device) == hipSuccess ? prop.multiProcessorCount : 256;
  }
  const int grid = std::max(1, std::min(nchunks, fl.ctx->num_cu * per_cu));
  k_zero_tickets<<<1, 64, 0, s>>>(fl.tickets);
  k_force_tickets<K, COUNT, B><<<grid, B, 0, s>>>(p4, n, cs, g, n_geom, mm, acc, ab, st, list, nr, nchunks,
                                                  fl.tickets);
}

template <int K, bool COUNT>
static void launch_force_k(const ForceLaunch& fl, int nr, hipStream_t s, const float4* p4, int n, const int* cs,
                           const GeomDev* g, int n_geom, uint32_t mm, float4* acc, unsigned* ab, uint32_t* st,
                           const int* list) {
  if (fl.block == 128) launch_force_b<K, COUNT, 128>(fl, nr, s, p4, n, cs, g, n_geom, mm, acc, ab, st, list);
  else if (fl.block == 512) launch_force_b<K, COUNT, 512>(fl, nr, s, p4, n, cs, g, n_geom, mm, acc, ab, st, list);
  else launch_force_b<K, COUNT, 256>(fl, nr, s, p4, n, cs, g, n_geom, mm, acc, ab, st, list);
}

template <int K, bool COUNT>
static void launch_force_mr(int remap, int nr, hipStream_t s, const float4* p4, int n, const int* cs,
                            const GeomDev* g, int n_geom, uint32_t mm, float4* acc, unsigned* ab, uint32_t* st,
                            const int* list) {
  k_force<K, COUNT, 256, true><<<(nr + 255) / 256, 256, 0, s>>>(p4, n, cs, g, n_geom, mm, acc, ab, st, list, nr, remap);
}

// A multi-resolution geometry takes the level-aware variant (256 threads, one
// block per chunk, whatever the launch shape set for the single-resolution kernel).
static void launch_force(int k, bool count, bool mr, const ForceLaunch& fl, int nr, hipStream_t s, const float4* p4,
                         int n, const int* cs, const GeomDev* g, int n_geom, uint32_t mm, float4* acc, unsigned* ab,
                         uint32_t* st, const int* list) {
  if (mr) {
    if (k == 1) {
      if (count) launch_force_mr<1, true>(fl.remap, nr, s, p4, n, cs, g, n_geom, mm, acc, ab, st, list);
      else launch_force_mr<1, false>(fl.remap, nr, s, p4, n, cs, g, n_geom, mm, acc, ab, st, list);
    } else {
      if (count) launch_force_mr<2, true>(fl.remap, nr, s, p4, n, cs, g, n_geom, mm, acc, ab, st, list);
      else launch_force_mr<2, false>(fl.remap, nr, s, p4, n, cs, g, n_geom, mm, acc, ab, st, list);
    }
    return;
  }
  if (k == 1) {
    if (count) launch_force_k<1, true>(fl, nr, s, p4, n, cs, g, n_geom, mm, acc, ab, st, list);
    else launch_force_k<1, false>(fl, nr, s, p4, n, cs, g, n_geom, mm, acc, ab, st, list);
  } else {
    if (count) launch_force_k<2, true>(fl, nr, s, p4, n, cs, g, n_geom, mm, acc, ab, st, list);
    else launch_force_k<2, false>(fl, nr, s, p4, n, cs, g, n_geom, mm, acc, ab, st, list);
  }
}

static fppg_status check_common(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                const int32_t* cs) {
  if (!ctx || !geom) return fail(ctx, FPPG_E_ARG, "null ctx/geom");
  if (n != geom->n_active) return fail(ctx, FPPG_E_ARG, "n differs from the active particle count of the geometry");
  if (n > 0 && (!pos || !cs)) return fail(ctx, FPPG_E_ARG, "null pos/cell_start");
  if (!aligned(pos, 16)) return fail(ctx, FPPG_E_ARG, "pos must be 16-byte aligned");
  return FPPG_OK;
}

}  // namespace fppg

using namespace fppg;

extern "C" fppg_status fppg_relax_step(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                       const int32_t* owner, const int32_t* cell_start, const int32_t* feat_seg,
                                       int32_t n_feat, uint32_t move_mask, uint32_t flags, float* accel,
                                       float* amax, float* disp, const int32_t* list, int32_t n_list, void* ws,
                                       size_t ws_bytes, void* stream) {
  fppg_status st = check_common(ctx, geom, n, pos, cell_start);
  if (st != FPPG_OK) return st;
  if (list && (n_list < 0 || n_list > n)) return fail(ctx, FPPG_E_ARG, "n_list must be in [0, n]");
  const bool forces_only = (flags & FPPG_F_FORCES_ONLY) != 0;
  if (forces_only && !accel) return fail(ctx, FPPG_E_ARG, "FPPG_F_FORCES_ONLY needs accel");
  if (!amax || (n > 0 && ((!disp && !forces_only) || !owner))) return fail(ctx, FPPG_E_ARG, "null amax/disp/owner");
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
  const int nr = list ? int(n_list) : ni;   // launch slots
  const bool count = (flags & FPPG_F_COUNT_PAIRS) != 0;
  k_zero_f32<<<grid_for(geom->n_geom), kBlock, 0, s>>>(amax, geom->n_geom);
  if (nr > 0) {
    const float4* p4 = reinterpret_cast<const float4*>(pos);
    unsigned* ab = reinterpret_cast<unsigned*>(amax);
    {
    PhaseTimer timer(ctx, 1, s);
    const ForceLaunch fl{ctx->force_block, ctx->xcd_remap, ctx->persistent, ctx->d_tickets, ctx};
    launch_force(geom->k, count, geom->has_levels, fl, nr, s, p4, ni, cell_start, geom->d_geom, geom->n_geom,
                 move_mask, acc, ab,
                 ctx->d_status, list);
    }
    if (!forces_only) {
    PhaseTimer timer(ctx, 2, s);
    k_update<<<grid_for(nr), kBlock, 0, s>>>(p4, acc, owner, feat_seg, ni, n_feat, int(geom->n_tri), int(geom->n_seg),
                                             geom->d_geom, geom->n_geom, amax, geom->d_n32, geom->d_seg, move_mask,
                                             reinterpret_cast<float4*>(disp), ctx->d_status, list, nr);
    }
  }
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

extern "C" fppg_status fppg_set_launch(fppg_ctx* ctx, int32_t force_block, int32_t xcd_remap) {
  if (!ctx) return FPPG_E_ARG;
  if (force_block != 128 && force_block != 256 && force_block != 512)
    return fail(ctx, FPPG_E_ARG, "force_block must be 128, 256 or 512");
  if (xcd_remap < 0 || xcd_remap > 2) return fail(ctx, FPPG_E_ARG, "xcd_remap must be 0, 1 or 2");
  ctx->force_block = force_block;
  ctx->xcd_remap = xcd_remap;
  return FPPG_OK;
}

extern "C" fppg_status fppg_set_schedule(fppg_ctx* ctx, int32_t persistent) {
  if (!ctx) return FPPG_E_ARG;
  if (persistent != 0 && persistent != 1) return fail(ctx, FPPG_E_ARG, "persistent must be 0 or 1");
  ctx->persistent = persistent != 0;
  return FPPG_OK;
}

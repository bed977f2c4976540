// Particle generation front end (sections 3.1.1, 3.1.2 and 3.2.1): classify
// the cells of a uniform background grid of edge dx as surface, internal or
// external, then seed a volume particle at the centre of every internal cell
// and a surface particle at the projection of every surface cell's centre
// onto its nearest facet.
//
//   surface cells   one wavefront per facet walks the cells of the facet's
//                   bounding box (widened by a cell) and applies the
//                   separating-axis triangle-box test (box normals, facet
//                   normal, the 9 products of box axes and facet edges),
//                   closed: touching counts. The paper first subdivides
//                   facets until their box spans at most one cell; a cell
//                   meets a facet iff it meets one of its sub-triangles, so
//                   walking the whole box gives the same cells.
//   ray parity      one wavefront per facet walks the columns under the
//                   facet's xy box; a column whose centre lies in the
//                   facet's xy projection (counter-clockwise, a point on an
//                   edge counted only for edges pointing down in y, or along
//                   -x when horizontal, each edge function evaluated with the
//                   endpoints in lexicographic order so that two facets
//                   sharing an edge see opposite values) toggles the parity
//                   bit of the first cell whose centre lies above the
//                   crossing; a prefix XOR up each column gives the parity
//                   of the crossings below every centre. Internal = odd and
//                   not surface. Vertical facets (zero projected area) are
//                   not crossed.
//   surface mapping among the facets meeting a surface cell, the projection
//                   of the centre along the facet normal whose foot lies
//                   inside the facet (barycentric >= 0) with the smallest
//                   |plane distance| (ties: lowest facet), by two passes of
//                   64-bit / 32-bit atomicMin per cell; none: discarded.
//   output          particles in cell order (z, y, x; x fastest) by a
//                   three-phase count / scan / write (per-block counts, the
//                   multi-block exclusive scan of the cell rebuild).
//
// All arithmetic is FP64 with the sums of three products taken left to
// right and no contraction (the build's -ffp-contract=off), so the classes
// are those of the plain definition evaluated in the same order.
#include "gen_common.h"

namespace fppg {

namespace gen {

__global__ __launch_bounds__(kWave) void k_surface_cells(const double* __restrict__ vert, const int* __restrict__ tri,
                                                          Grid g, uint8_t* __restrict__ cls,
                                                          unsigned long long* __restrict__ dkey, int pass,
                                                          int* __restrict__ best) {
  const int t = blockIdx.x;
  const Tri T = load_tri(vert, tri, t);
  int r0[3], r1[3];
  for (int a = 0; a < 3; ++a) {
    const double lo = fmin(fmin(T.a[a], T.b[a]), T.c[a]), hi = fmax(fmax(T.a[a], T.b[a]), T.c[a]);
    cell_range(g, a, lo, hi, r0[a], r1[a]);
  }
  const int sx = r1[0] - r0[0] + 1, sy = r1[1] - r0[1] + 1, sz = r1[2] - r0[2] + 1;
  const int64_t cnt = int64_t(sx) * sy * sz;
  const double h = 0.5 * g.dx;
  for (int64_t q = threadIdx.x; q < cnt; q += kWave) {
    const int i = r0[0] + int(q % sx), j = r0[1] + int((q / sx) % sy), k = r0[2] + int(q / (int64_t(sx) * sy));
    const double c[3] = {centre(g, 0, i), centre(g, 1, j), centre(g, 2, k)};
    if (!tri_box(T, c, h)) continue;
    const int64_t cell = cell_index(g, i, j, k);
    double d, p[3];
    const bool in = project_inside(T, c, d, p);
    const unsigned long long key = __double_as_longlong(fabs(d));
    if (pass == 0) {
      cls[cell] = kSurface;
      if (in) atomicMin(&dkey[cell], key);
    } else if (in && key == dkey[cell]) {
      atomicMin(&best[cell], t);
    }
  }
}

__global__ __launch_bounds__(kWave) void k_ray_crossings(const double* __restrict__ vert, const int* __restrict__ tri,
                                                          Grid g, unsigned* __restrict__ toggle) {
  const Crossing X = crossing_of(load_tri(vert, tri, blockIdx.x), g);
  if (!X.valid) return;
  for (int q = threadIdx.x; q < X.sx * X.sy; q += kWave) {
    const int i = X.r0[0] + q % X.sx, j = X.r0[1] + q / X.sx;
    const int k = crossing_cell(X, g, i, j);
    if (k >= 0 && k < g.n[2]) {
      const int64_t cell = cell_index(g, i, j, k);
      atomicXor(&toggle[cell >> 5], 1u << (cell & 31));
    }
  }
}

__global__ __launch_bounds__(256) void k_column_parity(Grid g, const unsigned* __restrict__ toggle,
                                                        uint8_t* __restrict__ cls) {
  const int64_t col = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (col >= int64_t(g.n[0]) * g.n[1]) return;
  const int i = int(col % g.n[0]), j = int(col / g.n[0]);
  unsigned par = 0;
  for (int k = 0; k < g.n[2]; ++k) {
    const int64_t cell = cell_index(g, i, j, k);
    par ^= (toggle[cell >> 5] >> (cell & 31)) & 1u;
    if (par && cls[cell] != kSurface) cls[cell] = kInternal;
  }
}

__device__ __forceinline__ bool emits(const uint8_t* __restrict__ cls, const int* __restrict__ best, int64_t cell) {
  const uint8_t c = cls[cell];
  return c == kInternal || (c == kSurface && best[cell] != 0x7fffffff);
}

// per block of 256 cells: the number of particles it emits, and of them
// surface particles
__global__ __launch_bounds__(256) void k_emit_count(const uint8_t* __restrict__ cls, const int* __restrict__ best,
                                                     int64_t ncell, int* __restrict__ bcount,
                                                     int* __restrict__ scount) {
  const int64_t cell = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const bool e = cell < ncell && emits(cls, best, cell);
  const bool sf = e && cls[cell] == kSurface;
  __shared__ int w[4], ws[4];
  const uint64_t m = __ballot(e), ms = __ballot(sf);
  if ((threadIdx.x & 63) == 0) {
    w[threadIdx.x >> 6] = __popcll(m);
    ws[threadIdx.x >> 6] = __popcll(ms);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bcount[blockIdx.x] = w[0] + w[1] + w[2] + w[3];
    scount[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
  }
}

__global__ __launch_bounds__(256) void k_emit_write(const uint8_t* __restrict__ cls, const int* __restrict__ best,
                                                     const double* __restrict__ vert, const int* __restrict__ tri,
                                                     Grid g, int64_t ncell, const int* __restrict__ boff,
                                                     int64_t cap, float4* __restrict__ pos, int* __restrict__ owner) {
  const int64_t cell = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const bool e = cell < ncell && emits(cls, best, cell);
  __shared__ int w[4];
  const uint64_t m = __ballot(e);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) w[wid] = __popcll(m);
  __syncthreads();
  int before = 0;
  for (int k = 0; k < wid; ++k) before += w[k];
  if (!e) return;
  const int64_t slot = boff[blockIdx.x] + before + __popcll(m & ((1ull << lane) - 1));
  if (slot >= cap) return;
  const int i = int(cell % g.n[0]), j = int((cell / g.n[0]) % g.n[1]), k = int(cell / (int64_t(g.n[0]) * g.n[1]));
  const double c[3] = {centre(g, 0, i), centre(g, 1, j), centre(g, 2, k)};
  if (cls[cell] == kInternal) {
    pos[slot] = make_float4(float(c[0]), float(c[1]), float(c[2]), __int_as_float(FPPG_TAG_VOLUME));
    owner[slot] = -1;
  } else {
    const int t = best[cell];
    double d, p[3];
    project_inside(load_tri(vert, tri, t), c, d, p);
    pos[slot] = make_float4(float(p[0]), float(p[1]), float(p[2]), __int_as_float(FPPG_TAG_SURFACE));
    owner[slot] = t;
  }
}

__global__ void k_fill_u64(unsigned long long* __restrict__ a, int64_t n, unsigned long long v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_fill_i32b(int* __restrict__ a, int64_t n, int v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_fill_u8(uint8_t* __restrict__ a, int64_t n, uint8_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// Boolean combination of two classified solids on the same grid (section
// 3.2.3): set operations on the internal cells, surface cells kept where the
// combined surface can pass.
__global__ void k_cells_boolean(const uint8_t* __restrict__ a, const uint8_t* __restrict__ b, int64_t n, int op,
                                uint8_t* __restrict__ out) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const bool ai = a[q] == kInternal, as = a[q] == kSurface, bi = b[q] == kInternal, bs = b[q] == kSurface;
  bool i, s;
  if (op == 0) {          // union
    i = ai || bi;
    s = (as && !bi) || (bs && !ai);
  } else if (op == 1) {   // intersection
    i = ai && bi;
    s = (as && (bi || bs)) || (bs && (ai || as));
  } else {                // difference a - b
    i = ai && !(bi || bs);
    s = (as && !bi) || (bs && (ai || as));
  }
  out[q] = i ? kInternal : (s ? kSurface : kExternal);
}

inline int blocks(int64_t n, int b) { return int((n + b - 1) / b); }

}  // namespace gen
}  // namespace fppg

using namespace fppg;

extern "C" fppg_status fppg_generate(fppg_ctx* ctx, const double* vert, int32_t n_vert, const int32_t* tri,
                                     int32_t n_tri, double dx, const double* origin, const int32_t* dims,
                                     uint8_t* cell_class, float* pos, int32_t* owner, int64_t cap, int64_t* counts,
                                     void* stream) {
  if (!ctx) return fail(ctx, FPPG_E_ARG, "null ctx");
  if (!vert || !tri || n_vert < 3 || n_tri < 1 || !origin || !dims || !counts || !cell_class)
    return fail(ctx, FPPG_E_ARG, "null or empty mesh/grid/output");
  if (!(dx > 0.0) || !std::isfinite(dx)) return fail(ctx, FPPG_E_ARG, "dx must be finite and > 0");
  if (cap < 0 || (cap > 0 && (!pos || !owner))) return fail(ctx, FPPG_E_ARG, "bad particle capacity/outputs");
  if (!aligned(pos, 16)) return fail(ctx, FPPG_E_ARG, "pos must be 16-byte aligned");
  for (int a = 0; a < 3; ++a)
    if (dims[a] < 1 || !std::isfinite(origin[a])) return fail(ctx, FPPG_E_ARG, "bad grid");
  for (int64_t q = 0; q < 3 * int64_t(n_tri); ++q)
    if (tri[q] < 0 || tri[q] >= n_vert) return fail(ctx, FPPG_E_ARG, "facet vertex index out of range");
  const int64_t ncell = int64_t(dims[0]) * dims[1] * dims[2];
  if (ncell >= (int64_t(1) << 31)) return fail(ctx, FPPG_E_CAPACITY, "background grid exceeds 2^31 cells");
  counts[0] = counts[1] = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  gen::Grid g;
  for (int a = 0; a < 3; ++a) {
    g.o[a] = origin[a];
    g.n[a] = dims[a];
  }
  g.dx = dx;
  const int nb = gen::blocks(ncell, 256);
  double* d_vert = nullptr;
  int* d_tri = nullptr;
  unsigned long long* d_key = nullptr;
  int* d_best = nullptr;
  unsigned* d_tog = nullptr;
  int* d_bcount = nullptr;
  int* d_scount = nullptr;
  int* d_boff = nullptr;
  int* d_soff = nullptr;
  int* d_bsum = nullptr;
  fppg_status st = FPPG_OK;
  auto cleanup = [&]() {
    hipStreamSynchronize(s);
    hipFree(d_vert);
    hipFree(d_tri);
    hipFree(d_key);
    hipFree(d_best);
    hipFree(d_tog);
    hipFree(d_bcount);
    hipFree(d_scount);
    hipFree(d_boff);
    hipFree(d_soff);
    hipFree(d_bsum);
  };
#define GEN_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) {                             \
      st = fail(ctx, FPPG_E_HIP, hipGetErrorString(e_)); \
      cleanup();                                        \
      return st;                                        \
    }                                                   \
  } while (0)
  GEN_HIP(hipMalloc(&d_vert, sizeof(double) * 3 * n_vert));
  GEN_HIP(hipMalloc(&d_tri, sizeof(int) * 3 * n_tri));
  GEN_HIP(hipMalloc(&d_key, sizeof(unsigned long long) * ncell));
  GEN_HIP(hipMalloc(&d_best, sizeof(int) * ncell));
  GEN_HIP(hipMalloc(&d_tog, sizeof(unsigned) * ((ncell + 31) / 32)));
  GEN_HIP(hipMalloc(&d_bcount, sizeof(int) * nb));
  GEN_HIP(hipMalloc(&d_scount, sizeof(int) * nb));
  GEN_HIP(hipMalloc(&d_boff, sizeof(int) * (nb + 1)));
  GEN_HIP(hipMalloc(&d_soff, sizeof(int) * (nb + 1)));
  GEN_HIP(hipMalloc(&d_bsum, sizeof(int) * scan_blocksum_len(nb)));
  GEN_HIP(hipMemcpyAsync(d_vert, vert, sizeof(double) * 3 * n_vert, hipMemcpyHostToDevice, s));
  GEN_HIP(hipMemcpyAsync(d_tri, tri, sizeof(int) * 3 * n_tri, hipMemcpyHostToDevice, s));
  gen::k_fill_u8<<<gen::blocks(ncell, 256), 256, 0, s>>>(cell_class, ncell, gen::kExternal);
  gen::k_fill_u64<<<gen::blocks(ncell, 256), 256, 0, s>>>(d_key, ncell, ~0ull);
  gen::k_fill_i32b<<<gen::blocks(ncell, 256), 256, 0, s>>>(d_best, ncell, 0x7fffffff);
  gen::k_fill_i32b<<<gen::blocks((ncell + 31) / 32, 256), 256, 0, s>>>(reinterpret_cast<int*>(d_tog),
                                                                         (ncell + 31) / 32, 0);
  gen::k_surface_cells<<<n_tri, gen::kWave, 0, s>>>(d_vert, d_tri, g, cell_class, d_key, 0, d_best);
  gen::k_surface_cells<<<n_tri, gen::kWave, 0, s>>>(d_vert, d_tri, g, cell_class, d_key, 1, d_best);
  gen::k_ray_crossings<<<n_tri, gen::kWave, 0, s>>>(d_vert, d_tri, g, d_tog);
  gen::k_column_parity<<<gen::blocks(int64_t(dims[0]) * dims[1], 256), 256, 0, s>>>(g, d_tog, cell_class);
  gen::k_emit_count<<<nb, 256, 0, s>>>(cell_class, d_best, ncell, d_bcount, d_scount);
  // block offsets (the total below 2^31 cells fits) and the surface total
  if ((st = exclusive_scan(ctx, d_bcount, nb, d_boff, d_bsum, s)) != FPPG_OK ||
      (st = exclusive_scan(ctx, d_scount, nb, d_soff, d_bsum, s)) != FPPG_OK) {
    cleanup();
    return st;
  }
  gen::k_emit_write<<<nb, 256, 0, s>>>(cell_class, d_best, d_vert, d_tri, g, ncell, d_boff, cap,
                                       reinterpret_cast<float4*>(pos), owner);
  GEN_HIP(hipGetLastError());
  int total = 0, nsurf = 0;
  GEN_HIP(hipMemcpyAsync(&total, d_boff + nb, sizeof(int), hipMemcpyDeviceToHost, s));
  GEN_HIP(hipMemcpyAsync(&nsurf, d_soff + nb, sizeof(int), hipMemcpyDeviceToHost, s));
  GEN_HIP(hipStreamSynchronize(s));
#undef GEN_HIP
  cleanup();
  counts[0] = int64_t(total) - nsurf;
  counts[1] = nsurf;
  if (total > cap) {
    counts[0] = -1;
    counts[1] = total;
    return fail(ctx, FPPG_E_CAPACITY, "more particles than cap (counts[1] holds the total)");
  }
  return FPPG_OK;
}

extern "C" fppg_status fppg_cells_boolean(fppg_ctx* ctx, const uint8_t* a, const uint8_t* b, int64_t n, int32_t op,
                                          uint8_t* out, void* stream) {
  if (!ctx) return fail(ctx, FPPG_E_ARG, "null ctx");
  if (n < 0 || (n > 0 && (!a || !b || !out))) return fail(ctx, FPPG_E_ARG, "null class array");
  if (op < 0 || op > 2) return fail(ctx, FPPG_E_ARG, "op must be 0 (union), 1 (intersection) or 2 (difference)");
  if (n == 0) return FPPG_OK;
  gen::k_cells_boolean<<<gen::blocks(n, 256), 256, 0, static_cast<hipStream_t>(stream)>>>(a, b, n, op, out);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

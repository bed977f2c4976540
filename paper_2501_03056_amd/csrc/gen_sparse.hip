// Particle generation through the sparse storage of section 3.1.3: the same
// particles as fppg_generate (classes and mapping of the dense path, output
// in cell order) with memory proportional to the grid's columns, the surface
// and the output instead of one byte per background cell.
//
//   surface cells   the registered cells of the mesh's sparse grid (facet
//                   subdivision, separating-axis test with a pad of 1e-6 dx,
//                   C_compact in Morton order: register.hip); one lane per
//                   cell decodes its Morton code, keeps the facets that meet
//                   the cell under the whole-facet test of the dense path and
//                   maps the centre onto the nearest of them whose foot lies
//                   inside (smallest |plane distance|, ties: lowest facet)
//   crossings       one wavefront per facet emits the (column, height) events
//                   of the vertical ray casting; the events are radix-sorted
//                   and an event of even multiplicity cancels (parity)
//   column lists    toggles and surface cells as int32 heights, sorted, with
//                   per-column offsets (counts + exclusive scan)
//   emission        one lane per background cell in cell order reads its
//                   column's lists: a surface cell emits iff it maps onto a
//                   facet, another cell iff an odd number of toggles lie at or
//                   below it; per block count, scan, write (as the dense path)
#include "gen_common.h"

#include <algorithm>
#include <vector>

namespace fppg {
namespace gen {

constexpr int kT = 256;
constexpr int kTotalSlots = 512;

__device__ __forceinline__ uint32_t compact_bits(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v | (v >> 2)) & 0x10c30c30c30c30c3ull;
  v = (v | (v >> 4)) & 0x100f00f00f00f00full;
  v = (v | (v >> 8)) & 0x1f0000ff0000ffull;
  v = (v | (v >> 16)) & 0x1f00000000ffffull;
  v = (v | (v >> 32)) & 0x1fffffull;
  return uint32_t(v);
}

// One lane per registered cell: the facets registered to it (ascending) are
// re-tested against the cell with the whole-facet separating-axis test of the
// dense classification; a cell that none passes is not a surface cell
// (column key = the sentinel ncol * (nz + 1), sorted last). A surface cell
// gets its column key (column, height) and the facet its centre maps onto
// (-1: none).
__global__ __launch_bounds__(kT) void k_map_cells(const uint64_t* __restrict__ code, const int* __restrict__ begin,
                                                   const int* __restrict__ length, const int* __restrict__ facets,
                                                   int nc, const double* __restrict__ vert,
                                                   const int* __restrict__ tri, Grid g,
                                                   int* __restrict__ best,
                                                   uint64_t* __restrict__ col_key) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const uint64_t m = code[c];
  const int i = int(compact_bits(m)), j = int(compact_bits(m >> 1)), k = int(compact_bits(m >> 2));
  const double ce[3] = {centre(g, 0, i), centre(g, 1, j), centre(g, 2, k)};
  const double h = 0.5 * g.dx;
  unsigned long long bkey = ~0ull;
  int bt = -1;
  bool surface = false;
  for (int q = begin[c], e = begin[c] + length[c]; q < e; ++q) {
    const int t = facets[q];
    const Tri T = load_tri(vert, tri, t);
    if (!tri_box(T, ce, h)) continue;
    surface = true;
    double d, p[3];
    if (!project_inside(T, ce, d, p)) continue;
    const unsigned long long key = __double_as_longlong(fabs(d));
    if (key < bkey) {   // strict: the lowest facet on ties
      bkey = key;
      bt = t;
    }
  }
  const uint64_t per = uint64_t(g.n[2] + 1), ncol = uint64_t(g.n[0]) * uint64_t(g.n[1]);
  best[c] = surface ? bt : -2;
  col_key[c] = surface ? (uint64_t(j) * uint64_t(g.n[0]) + uint64_t(i)) * per + uint64_t(k) : ncol * per;
}

// Per facet (one wavefront): the number of crossing events, then the events.
__global__ __launch_bounds__(kWave) void k_cross_events(const double* __restrict__ vert, const int* __restrict__ tri,
                                                         Grid g, int* __restrict__ count,
                                                         const int* __restrict__ offs, uint64_t* __restrict__ ev) {
  const Crossing X = crossing_of(load_tri(vert, tri, blockIdx.x), g);
  int c = 0;
  const int base = offs ? offs[blockIdx.x] : 0;
  if (X.valid) {
    for (int q0 = 0; q0 < X.sx * X.sy; q0 += kWave) {
      const int q = q0 + int(threadIdx.x);
      int k = -1, i = 0, j = 0;
      if (q < X.sx * X.sy) {
        i = X.r0[0] + q % X.sx;
        j = X.r0[1] + q / X.sx;
        k = crossing_cell(X, g, i, j);
      }
      const bool hit = k >= 0 && k < g.n[2];
      const uint64_t m = __ballot(hit);
      if (hit && offs)
        ev[base + c + __popcll(m & ((1ull << threadIdx.x) - 1ull))] =
            (uint64_t(j) * uint64_t(g.n[0]) + uint64_t(i)) * uint64_t(g.n[2] + 1) + uint64_t(k);
      c += __popcll(m);
    }
  }
  if (!offs && threadIdx.x == 0) count[blockIdx.x] = c;
}

// Events of odd multiplicity (sorted keys): flag at the head of each run.
__global__ __launch_bounds__(kT) void k_odd_runs(const uint64_t* __restrict__ ev, int n, int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int f = 0;
  if (i == 0 || ev[i] != ev[i - 1]) {
    int e = i + 1;
    while (e < n && ev[e] == ev[i]) ++e;
    f = (e - i) & 1;
  }
  flag[i] = f;
}

__global__ __launch_bounds__(kT) void k_compact_u64(const uint64_t* __restrict__ in, int n,
                                                     const int* __restrict__ flag, const int* __restrict__ pos,
                                                     uint64_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = in[i];
}

// Entries per column; keys at or past ncol * per_col (the sentinel) are skipped.
__global__ __launch_bounds__(kT) void k_count_columns(const uint64_t* __restrict__ key, int n, uint64_t per_col,
                                                       uint64_t ncol, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && key[i] < ncol * per_col) atomicAdd(&cnt[key[i] / per_col], 1);
}

__global__ __launch_bounds__(kT) void k_zero(int* __restrict__ a, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    a[i] = 0;
}

// Per-column lists as int32 cell heights: the surviving toggles, and the
// surface cells with the facet each maps onto (-1: none).
__global__ __launch_bounds__(kT) void k_heights(const uint64_t* __restrict__ key, int n, uint64_t per,
                                                 int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = int(key[i] % per);
}

__global__ __launch_bounds__(kT) void k_surface_heights(const uint64_t* __restrict__ col_key,
                                                         const uint32_t* __restrict__ idx, const int* __restrict__ best,
                                                         const int* __restrict__ n_surf, uint64_t per,
                                                         int* __restrict__ sk, int* __restrict__ sb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *n_surf) return;
  sk[i] = int(col_key[i] % per);
  sb[i] = best[idx[i]];
}

__global__ __launch_bounds__(kT) void k_iota(uint32_t* __restrict__ a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = uint32_t(i);
}

// The class of cell (i, j, k) from its column's lists: a surface cell emits
// iff it maps onto a facet (*facet = that facet), any other cell iff an odd
// number of toggles lie at or below k (internal; *facet = -1).
__device__ __forceinline__ bool emits_cell(const int* __restrict__ toff, const int* __restrict__ tk,
                                           const int* __restrict__ soff, const int* __restrict__ sk,
                                           const int* __restrict__ sb, int64_t col, int k, int* facet) {
  for (int s = soff[col], e = soff[col + 1]; s < e; ++s) {
    const int h = sk[s];
    if (h == k) {
      *facet = sb[s];
      return sb[s] >= 0;
    }
    if (h > k) break;
  }
  int par = 0;
  for (int t = toff[col], e = toff[col + 1]; t < e && tk[t] <= k; ++t) par ^= 1;
  *facet = -1;
  return par != 0;
}

// Blocks of 256 cells in cell order (chunk of cells starting at base): pass 0
// counts each block's particles (and the totals), pass 1 writes them at the
// block's scanned offset, in cell order within the block.
template <bool WRITE>
__global__ __launch_bounds__(kT) void k_emit(const int* __restrict__ toff, const int* __restrict__ tk,
                                              const int* __restrict__ soff, const int* __restrict__ sk,
                                              const int* __restrict__ sb, Grid g, int64_t ncell, int64_t base,
                                              int* __restrict__ bcount, unsigned long long* __restrict__ totals,
                                              const int* __restrict__ boff, const double* __restrict__ vert,
                                              const int* __restrict__ tri, float4* __restrict__ pos,
                                              int* __restrict__ owner) {
  const int64_t blk = base / kT + blockIdx.x;
  const int64_t cell = blk * kT + threadIdx.x;
  int facet = -1;
  bool e = false;
  int i = 0, j = 0, k = 0;
  if (cell < ncell) {
    const int64_t plane = int64_t(g.n[0]) * g.n[1];
    k = int(cell / plane);
    const int64_t col = cell - int64_t(k) * plane;
    i = int(col % g.n[0]);
    j = int(col / g.n[0]);
    e = emits_cell(toff, tk, soff, sk, sb, col, k, &facet);
  }
  __shared__ int w[kT / kWave], ws[kT / kWave];
  const uint64_t m = __ballot(e), ms = __ballot(e && facet >= 0);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) {
    w[wid] = __popcll(m);
    ws[wid] = __popcll(ms);
  }
  __syncthreads();
  if (!WRITE) {
    if (threadIdx.x == 0) {
      int c = 0, cs = 0;
      for (int q = 0; q < kT / kWave; ++q) {
        c += w[q];
        cs += ws[q];
      }
      bcount[blk] = c;   // the totals over kTotalSlots addresses (one would serialise the blocks' atomics)
      if (c) atomicAdd(&totals[2 * (blk % kTotalSlots)], (unsigned long long)c);
      if (cs) atomicAdd(&totals[2 * (blk % kTotalSlots) + 1], (unsigned long long)cs);
    }
    return;
  }
  if (!e) return;
  int before = 0;
  for (int q = 0; q < wid; ++q) before += w[q];
  const int64_t slot = int64_t(boff[blk]) + before + __popcll(m & ((1ull << lane) - 1ull));
  const double c[3] = {centre(g, 0, i), centre(g, 1, j), centre(g, 2, k)};
  if (facet < 0) {
    pos[slot] = make_float4(float(c[0]), float(c[1]), float(c[2]), __int_as_float(FPPG_TAG_VOLUME));
    owner[slot] = -1;
  } else {
    double d, p[3];
    project_inside(load_tri(vert, tri, facet), c, d, p);
    pos[slot] = make_float4(float(p[0]), float(p[1]), float(p[2]), __int_as_float(FPPG_TAG_SURFACE));
    owner[slot] = facet;
  }
}

inline int nblk(int64_t n) { return int(std::max<int64_t>((n + kT - 1) / kT, 1)); }

static int bits_of(uint64_t v) {
  int b = 0;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

}  // namespace gen
}  // namespace fppg

using namespace fppg;

extern "C" fppg_status fppg_generate_sparse(fppg_ctx* ctx, const double* vert, int32_t n_vert, const int32_t* tri,
                                            int32_t n_tri, double dx, const double* origin, const int32_t* dims,
                                            float* pos, int32_t* owner, int64_t cap, int64_t* counts,
                                            int64_t* stats, void* stream) {
  using namespace fppg::gen;
  if (!ctx) return fail(ctx, FPPG_E_ARG, "null ctx");
  if (!vert || !tri || n_vert < 3 || n_tri < 1 || !origin || !dims || !counts)
    return fail(ctx, FPPG_E_ARG, "null or empty mesh/grid/output");
  if (!(dx > 0.0) || !std::isfinite(dx)) return fail(ctx, FPPG_E_ARG, "dx must be finite and > 0");
  if (cap < 0 || (cap > 0 && (!pos || !owner))) return fail(ctx, FPPG_E_ARG, "bad particle capacity/outputs");
  if (!aligned(pos, 16)) return fail(ctx, FPPG_E_ARG, "pos must be 16-byte aligned");
  for (int a = 0; a < 3; ++a)
    if (dims[a] < 1 || dims[a] > (1 << 21) || !std::isfinite(origin[a])) return fail(ctx, FPPG_E_ARG, "bad grid");
  const int64_t ncol64 = int64_t(dims[0]) * dims[1];
  if (ncol64 >= (int64_t(1) << 31)) return fail(ctx, FPPG_E_CAPACITY, "more than 2^31 grid columns");
  const int64_t ncell = ncol64 * dims[2];
  if (ncell >= (int64_t(1) << 38)) return fail(ctx, FPPG_E_CAPACITY, "background grid exceeds 2^38 cells");
  counts[0] = counts[1] = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the sparse grid (fppg_sparse_grid_create is synchronous)
  fppg_sparse_grid* sg = nullptr;
  fppg_status st = fppg_sparse_grid_create(ctx, vert, n_vert, tri, n_tri, origin, dx, dims, 1e-6 * dx, 0, &sg);
  if (st != FPPG_OK) return st;
  fppg_sparse_grid_view v{};
  fppg_sparse_grid_info(sg, &v);
  const int nc = int(v.n_cell);
  Grid g;
  for (int a = 0; a < 3; ++a) {
    g.o[a] = origin[a];
    g.n[a] = dims[a];
  }
  g.dx = dx;
  const int ncol = int(ncol64);
  const uint64_t per = uint64_t(dims[2] + 1);
  const int colkey_bits = bits_of(uint64_t(ncol) * per);
  std::vector<void*> owned;
  auto dalloc = [&](void** p, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
    if (e == hipSuccess) owned.push_back(*p);
    return e;
  };
  auto cleanup = [&]() {
    hipStreamSynchronize(s);
    for (void* p : owned) hipFree(p);
    fppg_sparse_grid_destroy(sg);
  };
#define GS_HIP(call)                                     \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) {                              \
      st = fail(ctx, FPPG_E_HIP, hipGetErrorString(e_)); \
      cleanup();                                         \
      return st;                                         \
    }                                                    \
  } while (0)
#define GS_ST(call)      \
  do {                   \
    st = (call);         \
    if (st != FPPG_OK) { \
      cleanup();         \
      return st;         \
    }                    \
  } while (0)
  double* d_vert = nullptr;
  int* d_tri = nullptr;
  GS_HIP(dalloc(reinterpret_cast<void**>(&d_vert), sizeof(double) * 3 * n_vert));
  GS_HIP(dalloc(reinterpret_cast<void**>(&d_tri), sizeof(int) * 3 * n_tri));
  GS_HIP(hipMemcpyAsync(d_vert, vert, sizeof(double) * 3 * n_vert, hipMemcpyHostToDevice, s));
  GS_HIP(hipMemcpyAsync(d_tri, tri, sizeof(int) * 3 * n_tri, hipMemcpyHostToDevice, s));
  // surface cells, their mapping, and their (column, height) order
  uint64_t *col_key, *col_tmp;
  int* best;
  uint32_t *idx, *idx_tmp;
  GS_HIP(dalloc(reinterpret_cast<void**>(&col_key), 8 * size_t(nc)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&col_tmp), 8 * size_t(nc)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&best), 4 * size_t(nc)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&idx), 4 * size_t(nc)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&idx_tmp), 4 * size_t(nc)));
  if (nc > 0) {
    k_map_cells<<<nblk(nc), kT, 0, s>>>(v.morton, v.begin, v.length, v.facets, nc, d_vert, d_tri, g, best, col_key);
    k_iota<<<nblk(nc), kT, 0, s>>>(idx, nc);
  }
  GS_HIP(hipGetLastError());
  GS_ST(radix_sort_pairs(ctx, col_key, idx, col_tmp, idx_tmp, nc, 0, colkey_bits, s));
  // crossing events: count, scan, write, sort
  int *fcnt, *foff, *bsum;
  GS_HIP(dalloc(reinterpret_cast<void**>(&fcnt), 4 * size_t(n_tri)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&foff), 4 * (size_t(n_tri) + 1)));
  const int64_t nblocks = (ncell + kT - 1) / kT;
  const int64_t bs_len = std::max<int64_t>({scan_blocksum_len(n_tri), scan_blocksum_len(ncol), scan_blocksum_len(nc),
                                            scan_blocksum_len(nblocks)});
  GS_HIP(dalloc(reinterpret_cast<void**>(&bsum), 4 * size_t(bs_len)));
  k_cross_events<<<n_tri, kWave, 0, s>>>(d_vert, d_tri, g, fcnt, nullptr, nullptr);
  GS_ST(exclusive_scan(ctx, fcnt, n_tri, foff, bsum, s));
  int nev = 0;
  GS_HIP(hipMemcpyAsync(&nev, foff + n_tri, 4, hipMemcpyDeviceToHost, s));
  GS_HIP(hipStreamSynchronize(s));
  uint64_t *ev, *ev_tmp;
  uint32_t *evv, *evv_tmp;
  GS_HIP(dalloc(reinterpret_cast<void**>(&ev), 8 * size_t(nev)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&ev_tmp), 8 * size_t(nev)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&evv), 4 * size_t(nev)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&evv_tmp), 4 * size_t(nev)));
  k_cross_events<<<n_tri, kWave, 0, s>>>(d_vert, d_tri, g, fcnt, foff, ev);
  GS_HIP(hipGetLastError());
  GS_ST(radix_sort_pairs(ctx, ev, evv, ev_tmp, evv_tmp, nev, 0, colkey_bits, s));
  // parity: the events of odd multiplicity survive, once
  int *eflag, *epos, *ebs;
  GS_HIP(dalloc(reinterpret_cast<void**>(&eflag), 4 * size_t(nev)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&epos), 4 * (size_t(nev) + 1)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&ebs), 4 * size_t(scan_blocksum_len(nev))));
  if (nev > 0) k_odd_runs<<<nblk(nev), kT, 0, s>>>(ev, nev, eflag);
  GS_ST(exclusive_scan(ctx, eflag, nev, epos, ebs, s));
  int ntog = 0;
  GS_HIP(hipMemcpyAsync(&ntog, epos + nev, 4, hipMemcpyDeviceToHost, s));
  GS_HIP(hipStreamSynchronize(s));
  uint64_t* tog;
  int* tk;
  GS_HIP(dalloc(reinterpret_cast<void**>(&tog), 8 * size_t(ntog)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&tk), 4 * size_t(ntog)));
  if (nev > 0) k_compact_u64<<<nblk(nev), kT, 0, s>>>(ev, nev, eflag, epos, tog);
  if (ntog > 0) k_heights<<<nblk(ntog), kT, 0, s>>>(tog, ntog, per, tk);
  // per-column offsets of the toggles and of the surface cells
  int *tcnt, *toff, *scnt, *soff, *sk, *sb;
  GS_HIP(dalloc(reinterpret_cast<void**>(&tcnt), 4 * size_t(ncol)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&toff), 4 * (size_t(ncol) + 1)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&scnt), 4 * size_t(ncol)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&soff), 4 * (size_t(ncol) + 1)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&sk), 4 * size_t(nc)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&sb), 4 * size_t(nc)));
  const int gz = std::min(nblk(ncol), 4096);
  k_zero<<<gz, kT, 0, s>>>(tcnt, ncol);
  k_zero<<<gz, kT, 0, s>>>(scnt, ncol);
  if (ntog > 0) k_count_columns<<<nblk(ntog), kT, 0, s>>>(tog, ntog, per, uint64_t(ncol), tcnt);
  if (nc > 0) k_count_columns<<<nblk(nc), kT, 0, s>>>(col_key, nc, per, uint64_t(ncol), scnt);
  GS_ST(exclusive_scan(ctx, tcnt, ncol, toff, bsum, s));
  GS_ST(exclusive_scan(ctx, scnt, ncol, soff, bsum, s));
  if (nc > 0) k_surface_heights<<<nblk(nc), kT, 0, s>>>(col_key, idx, best, soff + ncol, per, sk, sb);
  GS_HIP(hipGetLastError());
  // emission, pass 0: particles per block of cells and the totals
  int *bcount, *boff;
  unsigned long long* totals;
  GS_HIP(dalloc(reinterpret_cast<void**>(&bcount), 4 * size_t(nblocks)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&boff), 4 * (size_t(nblocks) + 1)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&totals), 16 * kTotalSlots));
  k_zero<<<4, kT, 0, s>>>(reinterpret_cast<int*>(totals), 4 * kTotalSlots);
  constexpr int64_t kChunkBlocks = int64_t(1) << 22;   // cells per launch: 2^30
  for (int64_t b0 = 0; b0 < nblocks; b0 += kChunkBlocks) {
    const int nb = int(std::min(kChunkBlocks, nblocks - b0));
    k_emit<false><<<nb, kT, 0, s>>>(toff, tk, soff, sk, sb, g, ncell, b0 * kT, bcount, totals, nullptr, nullptr,
                                    nullptr, nullptr, nullptr);
  }
  GS_HIP(hipGetLastError());
  std::vector<unsigned long long> slots(2 * kTotalSlots);
  GS_HIP(hipMemcpyAsync(slots.data(), totals, 16 * kTotalSlots, hipMemcpyDeviceToHost, s));
  GS_HIP(hipStreamSynchronize(s));
  unsigned long long tot[2] = {0, 0};
  for (int q = 0; q < kTotalSlots; ++q) {
    tot[0] += slots[2 * q];
    tot[1] += slots[2 * q + 1];
  }
  if (stats) {
    stats[0] = nc;
    stats[1] = nev;
    stats[2] = ntog;
    stats[3] = v.levels;
  }
  const int64_t total = int64_t(tot[0]), nsurf = int64_t(tot[1]);
  if (total > cap) {
    cleanup();
    counts[0] = -1;
    counts[1] = total;
    return fail(ctx, FPPG_E_CAPACITY, "more particles than cap (counts[1] holds the total)");
  }
  if (total >= (int64_t(1) << 31)) {
    cleanup();
    return fail(ctx, FPPG_E_CAPACITY, "more than 2^31 particles");
  }
  // pass 1: block offsets, then the particles in cell order
  GS_ST(exclusive_scan(ctx, bcount, nblocks, boff, bsum, s));
  for (int64_t b0 = 0; b0 < nblocks && total > 0; b0 += kChunkBlocks) {
    const int nb = int(std::min(kChunkBlocks, nblocks - b0));
    k_emit<true><<<nb, kT, 0, s>>>(toff, tk, soff, sk, sb, g, ncell, b0 * kT, nullptr, nullptr, boff, d_vert, d_tri,
                                   reinterpret_cast<float4*>(pos), owner);
  }
  GS_HIP(hipGetLastError());
  cleanup();
#undef GS_HIP
#undef GS_ST
  counts[0] = total - nsurf;
  counts[1] = nsurf;
  return FPPG_OK;
}

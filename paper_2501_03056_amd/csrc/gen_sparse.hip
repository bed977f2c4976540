// Particle generation through the sparse storage of section 3.1.3: the same
// particles as fppg_generate (classes and mapping of the dense path, output
// in cell order) with memory proportional to the surface, the output and the
// grid's columns instead of one byte per background cell.
//
//   surface cells   the registered cells of the mesh's sparse grid (facet
//                   subdivision, separating-axis test with a pad of 1e-6 dx,
//                   C_compact in Morton order: register.hip); one lane per
//                   cell decodes its Morton code, keeps the facets that meet
//                   the cell under the whole-facet test of the dense path and
//                   maps the centre onto the nearest of them whose foot lies
//                   inside (smallest |plane distance|, ties: lowest facet)
//   crossings       one wavefront per facet emits the (column, height) events
//                   of the vertical ray casting; sorted, an event of even
//                   multiplicity cancels (parity)
//   sweep           the columns are dealt to wavefronts in groups of 2048:
//                   lane l of group g owns the 32 columns 2048 g + 64 b + l
//                   (b = 0..31), its parity as the bits of one word. Events
//                   are keyed (owner, height, b), so one sort leaves every
//                   lane's events in height order. A wavefront takes a group
//                   and 8 planes, starts from the parity of the toggles below
//                   them and sweeps upwards: toggles at the height flip parity bits, a
//                   surface cell emits iff it maps onto a facet, another cell
//                   iff its parity bit is set. Pass 0 counts per (plane,
//                   group), an exclusive scan gives the offsets in cell order,
//                   pass 1 writes: for b = 0..31 the 64 lanes hold 64
//                   consecutive columns, so a ballot places them and the
//                   stores are contiguous.
#include "gen_common.h"

#include <algorithm>
#include <vector>

namespace fppg {
namespace gen {

constexpr int kT = 256;
constexpr int kGroupCols = 2048;   // columns per sweeping wavefront: 64 lanes x 32 bits
constexpr int kChunkPlanes = 8;    // planes per sweeping wavefront
constexpr int kTotalSlots = 256;   // the count pass's totals, spread over this many address pairs

__device__ __forceinline__ uint32_t compact_bits(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v | (v >> 2)) & 0x10c30c30c30c30c3ull;
  v = (v | (v >> 4)) & 0x100f00f00f00f00full;
  v = (v | (v >> 8)) & 0x1f0000ff0000ffull;
  v = (v | (v >> 16)) & 0x1f00000000ffffull;
  v = (v | (v >> 32)) & 0x1fffffull;
  return uint32_t(v);
}

// Sweep key of cell (column col, height k): ((owner * nz + k) * 32 + b) with
// owner = 64 * group + lane.
__device__ __forceinline__ uint64_t sweep_key(int64_t col, int k, int nz) {
  const uint64_t owner = (uint64_t(col) / kGroupCols) * kWave + uint64_t(col % kWave);
  const uint64_t b = uint64_t((col / kWave) % 32);
  return ((owner * uint64_t(nz) + uint64_t(k)) << 5) | b;
}

// One lane per registered cell: the facets registered to it (ascending) are
// re-tested against the cell with the whole-facet separating-axis test of the
// dense classification; a cell that none passes is not a surface cell (key =
// the sentinel, sorted last). A surface cell gets its sweep key and the facet
// its centre maps onto (-1: none).
__global__ __launch_bounds__(kT) void k_map_cells(const uint64_t* __restrict__ code, const int* __restrict__ begin,
                                                   const int* __restrict__ length, const int* __restrict__ facets,
                                                   int nc, const double* __restrict__ vert,
                                                   const int* __restrict__ tri, Grid g, uint64_t sentinel,
                                                   int* __restrict__ best, uint64_t* __restrict__ key) {
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
    const unsigned long long dk = __double_as_longlong(fabs(d));
    if (dk < bkey) {   // strict: the lowest facet on ties
      bkey = dk;
      bt = t;
    }
  }
  best[c] = surface ? bt : -2;
  key[c] = surface ? sweep_key(int64_t(j) * g.n[0] + i, k, g.n[2]) : sentinel;
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
        ev[base + c + __popcll(m & ((1ull << threadIdx.x) - 1ull))] = sweep_key(int64_t(j) * g.n[0] + i, k, g.n[2]);
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

// Surviving toggles: owner counts and (height << 5 | b) words, compacted.
__global__ __launch_bounds__(kT) void k_compact_toggles(const uint64_t* __restrict__ ev, int n,
                                                         const int* __restrict__ flag, const int* __restrict__ pos,
                                                         int nz, int* __restrict__ tkb, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  const uint64_t r = ev[i] >> 5;
  tkb[pos[i]] = int(((r % uint64_t(nz)) << 5) | (ev[i] & 31u));
  atomicAdd(&cnt[r / uint64_t(nz)], 1);
}

// Surface cells (sorted keys; the sentinels last): owner counts, the
// (height << 5 | b) words and the facets.
__global__ __launch_bounds__(kT) void k_surface_lists(const uint64_t* __restrict__ key,
                                                       const uint32_t* __restrict__ idx, const int* __restrict__ best,
                                                       int n, uint64_t sentinel, int nz, int* __restrict__ skb,
                                                       int* __restrict__ sb, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || key[i] >= sentinel) return;
  const uint64_t r = key[i] >> 5;
  skb[i] = int(((r % uint64_t(nz)) << 5) | (key[i] & 31u));
  sb[i] = best[idx[i]];
  atomicAdd(&cnt[r / uint64_t(nz)], 1);
}

__global__ __launch_bounds__(kT) void k_zero(int* __restrict__ a, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    a[i] = 0;
}

__global__ __launch_bounds__(kT) void k_iota(uint32_t* __restrict__ a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = uint32_t(i);
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// One wavefront per group of 2048 columns and chunk of kChunkPlanes planes
// (w = chunk * ngroups + group), sweeping its planes upwards from the parity
// of the toggles below them. Pass 0 (WRITE false): cnt[k * ngroups + group] =
// the particles of the group in plane k; totals (over kTotalSlots slots) +=
// (particles, surface particles). Pass 1: the particles at
// off[k * ngroups + group] onwards, in column order.
template <bool WRITE>
__global__ __launch_bounds__(kWave) void k_sweep(const int* __restrict__ toff, const int* __restrict__ tkb,
                                                  const int* __restrict__ soff, const int* __restrict__ skb,
                                                  const int* __restrict__ sb, Grid g, int ngroups,
                                                  int* __restrict__ cnt, unsigned long long* __restrict__ totals,
                                                  const int* __restrict__ off, const double* __restrict__ vert,
                                                  const int* __restrict__ tri, float4* __restrict__ pos,
                                                  int* __restrict__ owner) {
  const int group = int(blockIdx.x % unsigned(ngroups)), chunk = int(blockIdx.x / unsigned(ngroups));
  const int lane = threadIdx.x;
  const int o = group * kWave + lane;
  int t = toff[o];
  const int te = toff[o + 1];
  int sp = soff[o];
  const int se = soff[o + 1];
  const int k0 = chunk * kChunkPlanes, k1 = min(g.n[2], k0 + kChunkPlanes);
  uint32_t par = 0;
  for (; t < te && (tkb[t] >> 5) < k0; ++t) par ^= 1u << (tkb[t] & 31);
  while (sp < se && (skb[sp] >> 5) < k0) ++sp;
  long long all = 0, surf = 0;
  for (int k = k0; k < k1; ++k) {
    while (t < te && (tkb[t] >> 5) == k) {
      par ^= 1u << (tkb[t] & 31);
      ++t;
    }
    uint32_t S = 0, M = 0;
    const int s0 = sp;
    while (sp < se && (skb[sp] >> 5) == k) {
      const uint32_t bit = 1u << (skb[sp] & 31);
      S |= bit;
      if (sb[sp] >= 0) M |= bit;
      ++sp;
    }
    const uint32_t E = (par & ~S) | M;
    if (!WRITE) {
      const int c = wave_sum(__popc(E));
      if (lane == 0) cnt[int64_t(k) * ngroups + group] = c;
      all += __popc(E);
      surf += __popc(M);
      continue;
    }
    if (__ballot(E != 0u) == 0ull) continue;
    int64_t base = off[int64_t(k) * ngroups + group];
    int q = s0;
    for (int b = 0; b < 32; ++b) {
      const bool e = (E >> b) & 1u;
      const uint64_t m = __ballot(e);
      if (e) {
        const int64_t col = int64_t(group) * kGroupCols + b * kWave + lane;
        const int64_t slot = base + __popcll(m & ((1ull << lane) - 1ull));
        const int i = int(col % g.n[0]), j = int(col / g.n[0]);
        const double c[3] = {centre(g, 0, i), centre(g, 1, j), centre(g, 2, k)};
        if ((M >> b) & 1u) {
          while ((skb[q] & 31) < b) ++q;   // this plane's surface cells, by b
          const int f = sb[q];
          double d, p[3];
          project_inside(load_tri(vert, tri, f), c, d, p);
          pos[slot] = make_float4(float(p[0]), float(p[1]), float(p[2]), __int_as_float(FPPG_TAG_SURFACE));
          owner[slot] = f;
        } else {
          pos[slot] = make_float4(float(c[0]), float(c[1]), float(c[2]), __int_as_float(FPPG_TAG_VOLUME));
          owner[slot] = -1;
        }
      }
      base += __popcll(m);
    }
  }
  if (!WRITE) {
    all = wave_sum(all);
    surf = wave_sum(surf);
    if (lane == 0) {
      const unsigned slot = 2u * (blockIdx.x % unsigned(kTotalSlots));
      atomicAdd(&totals[slot], (unsigned long long)all);
      atomicAdd(&totals[slot + 1], (unsigned long long)surf);
    }
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
  const int nz = dims[2];
  const int ngroups = int((ncol64 + kGroupCols - 1) / kGroupCols);
  const int n_owner = ngroups * kWave;
  const uint64_t sentinel = (uint64_t(n_owner) * uint64_t(nz)) << 5;
  const int key_bits = bits_of(sentinel);
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
  // surface cells, their mapping, and their sweep order
  uint64_t *skey, *skey_tmp;
  int* best;
  uint32_t *idx, *idx_tmp;
  GS_HIP(dalloc(reinterpret_cast<void**>(&skey), 8 * size_t(nc)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&skey_tmp), 8 * size_t(nc)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&best), 4 * size_t(nc)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&idx), 4 * size_t(nc)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&idx_tmp), 4 * size_t(nc)));
  if (nc > 0) {
    k_map_cells<<<nblk(nc), kT, 0, s>>>(v.morton, v.begin, v.length, v.facets, nc, d_vert, d_tri, g, sentinel, best,
                                        skey);
    k_iota<<<nblk(nc), kT, 0, s>>>(idx, nc);
  }
  GS_HIP(hipGetLastError());
  GS_ST(radix_sort_pairs(ctx, skey, idx, skey_tmp, idx_tmp, nc, 0, key_bits, s));
  // crossing events: count, scan, write, sort
  int *fcnt, *foff, *bsum;
  GS_HIP(dalloc(reinterpret_cast<void**>(&fcnt), 4 * size_t(n_tri)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&foff), 4 * (size_t(n_tri) + 1)));
  const int64_t n_plane_group = int64_t(nz) * ngroups;
  const int64_t bs_len = std::max<int64_t>({scan_blocksum_len(n_tri), scan_blocksum_len(n_owner),
                                            scan_blocksum_len(n_plane_group)});
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
  GS_ST(radix_sort_pairs(ctx, ev, evv, ev_tmp, evv_tmp, nev, 0, key_bits, s));
  // parity: the events of odd multiplicity survive, once; per-owner lists of
  // toggles and of surface cells
  int *eflag, *epos, *ebs, *tkb, *tcnt, *toff, *skb, *sb, *scnt, *soff;
  GS_HIP(dalloc(reinterpret_cast<void**>(&eflag), 4 * size_t(nev)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&epos), 4 * (size_t(nev) + 1)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&ebs), 4 * size_t(scan_blocksum_len(nev))));
  GS_HIP(dalloc(reinterpret_cast<void**>(&tkb), 4 * size_t(nev)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&tcnt), 4 * size_t(n_owner)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&toff), 4 * (size_t(n_owner) + 1)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&skb), 4 * size_t(nc)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&sb), 4 * size_t(nc)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&scnt), 4 * size_t(n_owner)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&soff), 4 * (size_t(n_owner) + 1)));
  const int gz = std::min(nblk(n_owner), 4096);
  k_zero<<<gz, kT, 0, s>>>(tcnt, n_owner);
  k_zero<<<gz, kT, 0, s>>>(scnt, n_owner);
  if (nev > 0) k_odd_runs<<<nblk(nev), kT, 0, s>>>(ev, nev, eflag);
  GS_ST(exclusive_scan(ctx, eflag, nev, epos, ebs, s));
  if (nev > 0) k_compact_toggles<<<nblk(nev), kT, 0, s>>>(ev, nev, eflag, epos, nz, tkb, tcnt);
  if (nc > 0) k_surface_lists<<<nblk(nc), kT, 0, s>>>(skey, idx, best, nc, sentinel, nz, skb, sb, scnt);
  GS_HIP(hipGetLastError());
  GS_ST(exclusive_scan(ctx, tcnt, n_owner, toff, bsum, s));
  GS_ST(exclusive_scan(ctx, scnt, n_owner, soff, bsum, s));
  int ntog = 0;
  GS_HIP(hipMemcpyAsync(&ntog, epos + nev, 4, hipMemcpyDeviceToHost, s));
  // the sweep, pass 0: particles per (plane, group) and the totals
  int *pcnt, *poff;
  unsigned long long* totals;
  GS_HIP(dalloc(reinterpret_cast<void**>(&pcnt), 4 * size_t(n_plane_group)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&poff), 4 * (size_t(n_plane_group) + 1)));
  GS_HIP(dalloc(reinterpret_cast<void**>(&totals), 16 * kTotalSlots));
  k_zero<<<4, kT, 0, s>>>(reinterpret_cast<int*>(totals), 4 * kTotalSlots);
  const int64_t nwaves = int64_t(ngroups) * ((nz + kChunkPlanes - 1) / kChunkPlanes);
  if (nwaves >= (int64_t(1) << 31)) {
    cleanup();
    return fail(ctx, FPPG_E_CAPACITY, "background grid too large for the sweep");
  }
  k_sweep<false><<<int(nwaves), kWave, 0, s>>>(toff, tkb, soff, skb, sb, g, ngroups, pcnt, totals, nullptr,
                                           nullptr, nullptr, nullptr, nullptr);
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
  // pass 1: offsets in cell order, then the particles
  GS_ST(exclusive_scan(ctx, pcnt, n_plane_group, poff, bsum, s));
  if (total > 0)
    k_sweep<true><<<int(nwaves), kWave, 0, s>>>(toff, tkb, soff, skb, sb, g, ngroups, nullptr, nullptr, poff,
                                            d_vert, d_tri, reinterpret_cast<float4*>(pos), owner);
  GS_HIP(hipGetLastError());
  cleanup();
#undef GS_HIP
#undef GS_ST
  counts[0] = total - nsurf;
  counts[1] = nsurf;
  return FPPG_OK;
}

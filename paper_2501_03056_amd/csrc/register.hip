// Facet registration on a uniform grid (section 3.1.1) and the sparse storage
// of the registered cells (section 3.1.3, Eq. 9-10).
//
//   subdivision  level by level: a triangle of a level is a leaf when its box
//                fits one cell along every axis; otherwise its edges whose
//                extent along some axis exceeds the cell edge are split at
//                their midpoints (the others' midpoints are virtual) and its
//                2, 3 or 4 children go to the next level. Per level: a count
//                pass, two prefix sums, a write pass (children in item order).
//   registration a leaf's box widened by pad reaches at most two cells per
//                axis; those passing the closed separating-axis test against
//                the cell box widened by pad give (key, facet) pairs. An item
//                whose widened box spans at most 4 cells per axis is finished
//                inside its lane (depth-first over its subtree, the cells its
//                leaves meet gathered in a 64-bit mask: one pair per cell and
//                item), so the last, largest levels are never stored. The
//                work per lane stays bounded however large or thin the facet
//                (the reason for the subdivision on a GPU).
//   sort         rocPRIM's stable device radix sort of the packed (key,
//                facet) words, so the pairs end in (key, facet) order;
//                duplicates (a facet met by several of its leaves in one cell)
//                dropped by a flag and a prefix sum.
//   dense CSR    the facet search grid of the projection: per-cell counts,
//                a prefix sum, the non-empty flags.
//   sparse       key = Morton code of the cell (Eq. 9); C_compact = the runs
//                of equal codes (begin, length); the hash of Eq. 10 of every
//                C_compact cell, entries sorted by it (stable: (hash, morton)),
//                H_begin / H_length from per-value counts and a prefix sum.
//
// All geometry is FP64 in the order the oracle evaluates it (the file is
// compiled without contraction).
#include "internal.h"
#include "sat.h"

#include <rocprim/device/device_radix_sort.hpp>

#include <vector>

namespace fppg {

namespace reg {

constexpr int kThreads = 256;
constexpr int kMaxLevels = 48;

__device__ __forceinline__ bool needs_split(const double p[3], const double q[3], double cell) {
  return fmax(fmax(fabs(q[0] - p[0]), fabs(q[1] - p[1])), fabs(q[2] - p[2])) > cell;
}

__device__ __forceinline__ void midpoint(const double p[3], const double q[3], double m[3]) {
  for (int k = 0; k < 3; ++k) m[k] = (p[k] + q[k]) * 0.5;
}

__device__ __forceinline__ void set_item(RegItem& o, const double a[3], const double b[3], const double c[3], int facet,
                                         int grid) {
  for (int k = 0; k < 3; ++k) {
    o.a[k] = a[k];
    o.b[k] = b[k];
    o.c[k] = c[k];
  }
  o.facet = facet;
  o.grid = grid;
}

// Eq. 9: bits of x, y, z interleaved (x lowest), 21 bits per axis.
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__device__ __forceinline__ uint64_t morton3(int x, int y, int z) {
  return spread3(uint64_t(x)) | (spread3(uint64_t(y)) << 1) | (spread3(uint64_t(z)) << 2);
}

__device__ __forceinline__ uint32_t compact3(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v | (v >> 2)) & 0x10c30c30c30c30c3ull;
  v = (v | (v >> 4)) & 0x100f00f00f00f00full;
  v = (v | (v >> 8)) & 0x1f0000ff0000ffull;
  v = (v | (v >> 16)) & 0x1f00000000ffffull;
  v = (v | (v >> 32)) & 0x1fffffull;
  return uint32_t(v);
}

// Eq. 10 in 64-bit unsigned arithmetic.
__device__ __forceinline__ uint32_t hash3(uint32_t x, uint32_t y, uint32_t z, uint64_t size) {
  return uint32_t((738560931ull * x + 19349663ull * y + 83492791ull * z) % size);
}

// The cell range [lo, hi] per axis of T's box widened by pad.
__device__ __forceinline__ void cell_box(const RegItem& T, const RegGrid& g, int lo[3], int hi[3]) {
  const double* v[3] = {T.a, T.b, T.c};
  for (int q = 0; q < 3; ++q) {
    const double mn = fmin(fmin(v[0][q], v[1][q]), v[2][q]);
    const double mx = fmax(fmax(v[0][q], v[1][q]), v[2][q]);
    // clamped in FP64 first, so that a far-off leaf converts without overflow
    lo[q] = max(0, int(fmax(floor((mn - g.pad - g.o[q]) * g.inv), -1.0)));
    hi[q] = min(g.dims[q] - 1, int(fmin(floor((mx + g.pad - g.o[q]) * g.inv), double(g.dims[q]))));
  }
}

// Visit the cells met by leaf T: f(x, y, z).
template <class F>
__device__ void leaf_cells(const RegItem& T, const RegGrid& g, F&& f) {
  int lo[3], hi[3];
  cell_box(T, g, lo, hi);
  const Tri tri{{T.a[0], T.a[1], T.a[2]}, {T.b[0], T.b[1], T.b[2]}, {T.c[0], T.c[1], T.c[2]}};
  const double h = 0.5 * g.cell + g.pad;
  for (int z = lo[2]; z <= hi[2]; ++z)
    for (int y = lo[1]; y <= hi[1]; ++y)
      for (int x = lo[0]; x <= hi[0]; ++x) {
        const double c[3] = {g.o[0] + (double(x) + 0.5) * g.cell, g.o[1] + (double(y) + 0.5) * g.cell,
                             g.o[2] + (double(z) + 0.5) * g.cell};
        if (tri_box(tri, c, h)) f(x, y, z);
      }
}

// The number of children of T (0: a leaf).
__device__ __forceinline__ int child_count(const RegItem& T, double cell) {
  const int n = int(needs_split(T.a, T.b, cell)) + int(needs_split(T.b, T.c, cell)) + int(needs_split(T.c, T.a, cell));
  return n == 0 ? 0 : n + 1;
}

__device__ __forceinline__ void pick3(int r, const double a[3], const double b[3], const double c[3], double o[3]) {
  for (int k = 0; k < 3; ++k) o[k] = r == 0 ? a[k] : (r == 1 ? b[k] : c[k]);
}

// Child `which` of T (vertex order as the oracle's). Three split edges: the
// corner triangles at a, b, c and the centre one; two: the corner where the
// split edges meet, then the rest cut along the diagonal from the far end of
// the unsplit edge (u, v); one: the two halves through the opposite vertex.
// The vertices are chosen by selects (no array of children or of vertex
// pointers), so a lane keeps everything in registers.
__device__ void make_child(const RegItem& T, double cell, int which, RegItem& out) {
  const bool s0 = needs_split(T.a, T.b, cell), s1 = needs_split(T.b, T.c, cell), s2 = needs_split(T.c, T.a, cell);
  const int n = int(s0) + int(s1) + int(s2);
  double p[3], q[3], r[3];
  if (n == 3) {
    double mab[3], mbc[3], mca[3];
    midpoint(T.a, T.b, mab);
    midpoint(T.b, T.c, mbc);
    midpoint(T.c, T.a, mca);
    // (a, mab, mca), (mab, b, mbc), (mca, mbc, c), (mab, mbc, mca)
    for (int k = 0; k < 3; ++k) {
      p[k] = which == 0 ? T.a[k] : (which == 2 ? mca[k] : mab[k]);
      q[k] = which == 0 ? mab[k] : (which == 1 ? T.b[k] : mbc[k]);
      r[k] = which == 0 ? mca[k] : (which == 1 ? mbc[k] : (which == 2 ? T.c[k] : mca[k]));
    }
  } else if (n == 2) {
    const int e = !s0 ? 0 : (!s1 ? 1 : 2);   // the unsplit edge (u, v)
    double u[3], v[3], w[3], mvw[3], mwu[3];
    pick3(e, T.a, T.b, T.c, u);
    pick3((e + 1) % 3, T.a, T.b, T.c, v);
    pick3((e + 2) % 3, T.a, T.b, T.c, w);
    midpoint(v, w, mvw);
    midpoint(w, u, mwu);
    // (mvw, w, mwu), (u, v, mvw), (u, mvw, mwu)
    for (int k = 0; k < 3; ++k) {
      p[k] = which == 0 ? mvw[k] : u[k];
      q[k] = which == 0 ? w[k] : (which == 1 ? v[k] : mvw[k]);
      r[k] = which == 0 ? mwu[k] : (which == 1 ? mvw[k] : mwu[k]);
    }
  } else {
    const int e = s0 ? 0 : (s1 ? 1 : 2);      // the split edge (u, v)
    double u[3], v[3], w[3], muv[3];
    pick3(e, T.a, T.b, T.c, u);
    pick3((e + 1) % 3, T.a, T.b, T.c, v);
    pick3((e + 2) % 3, T.a, T.b, T.c, w);
    midpoint(u, v, muv);
    // (u, muv, w), (muv, v, w)
    for (int k = 0; k < 3; ++k) {
      p[k] = which == 0 ? u[k] : muv[k];
      q[k] = which == 0 ? muv[k] : v[k];
      r[k] = w[k];
    }
  }
  set_item(out, p, q, r, T.facet, T.grid);
}

// A small item (its widened box within 4 x 4 x 4 cells) is subdivided inside
// one lane, depth first, down to its leaves; the cells its leaves meet are
// gathered as bits of a 4 x 4 x 4 mask relative to lo, so that a cell met by
// several leaves of one item gives one pair. Returns false (the item then
// goes on level by level) if the subtree is deeper than kLocalDepth.
constexpr int kLocalDepth = 8;

__device__ bool small_box(const RegItem& T, const RegGrid& g, int lo[3]) {
  int hi[3];
  cell_box(T, g, lo, hi);
  return hi[0] - lo[0] < 4 && hi[1] - lo[1] < 4 && hi[2] - lo[2] < 4;
}

__device__ bool subtree_mask(const RegItem& T, const RegGrid& g, const int lo[3], uint64_t& mask) {
  // the path as 3-bit fields: the child taken (d) and the siblings (nn) per depth
  uint32_t d = 0, nn = 0;
  int depth = 0;
  RegItem node = T;
  mask = 0;
  bool inside = true;
  for (;;) {
    const int c = child_count(node, g.cell);
    if (c > 0) {
      if (depth == kLocalDepth) return false;
      d &= ~(7u << (3 * depth));
      nn = (nn & ~(7u << (3 * depth))) | (uint32_t(c) << (3 * depth));
      ++depth;
      RegItem ch;
      make_child(node, g.cell, 0, ch);
      node = ch;
      continue;
    }
    leaf_cells(node, g, [&](int x, int y, int z) {
      const int bx = x - lo[0], by = y - lo[1], bz = z - lo[2];
      if (bx < 0 || by < 0 || bz < 0 || bx > 3 || by > 3 || bz > 3) inside = false;
      else mask |= uint64_t(1) << ((bz * 4 + by) * 4 + bx);
    });
    if (!inside) return false;
    while (depth > 0 && ((d >> (3 * (depth - 1))) & 7u) + 1 >= ((nn >> (3 * (depth - 1))) & 7u)) --depth;
    if (depth == 0) return true;
    d += 1u << (3 * (depth - 1));
    node = T;   // down the path again to the next sibling
    for (int k = 0; k < depth; ++k) {
      RegItem ch;
      make_child(node, g.cell, int((d >> (3 * k)) & 7u), ch);
      node = ch;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_level_count(const RegItem* __restrict__ items, int n,
                                                          const RegGrid* __restrict__ grids, int* __restrict__ nch,
                                                          int* __restrict__ npair) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const RegItem T = items[i];
  const RegGrid g = grids[T.grid];
  int c = child_count(T, g.cell);
  int p = 0;
  int lo[3];
  uint64_t mask;
  if (c == 0) {
    leaf_cells(T, g, [&](int, int, int) { ++p; });
  } else if (small_box(T, g, lo) && subtree_mask(T, g, lo, mask)) {
    c = 0;
    p = __popcll(mask);
  }
  nch[i] = c;
  npair[i] = p;
}

__global__ __launch_bounds__(kThreads) void k_level_write(const RegItem* __restrict__ items, int n,
                                                          const RegGrid* __restrict__ grids,
                                                          const int* __restrict__ choff, const int* __restrict__ poff,
                                                          RegItem* __restrict__ next, uint64_t* __restrict__ keys,
                                                          uint32_t* __restrict__ facets, int morton) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const RegItem T = items[i];
  const RegGrid g = grids[T.grid];
  const int c = child_count(T, g.cell);
  int o = poff[i];
  auto emit = [&](int x, int y, int z) {
    keys[o] = morton ? morton3(x, y, z)
                     : uint64_t(g.key_begin + (int64_t(z) * g.dims[1] + y) * g.dims[0] + x);
    facets[o] = uint32_t(T.facet);
    ++o;
  };
  if (c == 0) {
    leaf_cells(T, g, emit);
    return;
  }
  int lo[3];
  uint64_t mask;
  if (small_box(T, g, lo) && subtree_mask(T, g, lo, mask)) {
    for (; mask; mask &= mask - 1) {
      const int b = __ffsll((unsigned long long)mask) - 1;
      emit(lo[0] + (b & 3), lo[1] + ((b >> 2) & 3), lo[2] + (b >> 4));
    }
    return;
  }
  for (int k = 0; k < c; ++k) {
    RegItem ch;
    make_child(T, g.cell, k, ch);
    next[choff[i] + k] = ch;
  }
}

// (key << val_bits) | val, and back: one 64-bit sort key when both fit.
__global__ __launch_bounds__(kThreads) void k_pack_pairs(const uint64_t* __restrict__ keys,
                                                         const uint32_t* __restrict__ vals, int n, int val_bits,
                                                         uint64_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (keys[i] << val_bits) | uint64_t(vals[i]);
}

__global__ __launch_bounds__(kThreads) void k_unpack_pairs(uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                           int n, int val_bits) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t c = keys[i];
  keys[i] = c >> val_bits;
  vals[i] = uint32_t(c & ((uint64_t(1) << val_bits) - 1u));
}

__global__ __launch_bounds__(kThreads) void k_head_flags(const uint64_t* __restrict__ keys,
                                                         const uint32_t* __restrict__ vals, int n, int with_vals,
                                                         int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || keys[i] != keys[i - 1] || (with_vals && vals[i] != vals[i - 1])) ? 1 : 0;
}

__global__ __launch_bounds__(kThreads) void k_compact_pairs(const uint64_t* __restrict__ keys,
                                                            const uint32_t* __restrict__ vals, int n,
                                                            const int* __restrict__ flag, const int* __restrict__ pos,
                                                            uint64_t* __restrict__ kout, uint32_t* __restrict__ vout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  kout[pos[i]] = keys[i];
  vout[pos[i]] = vals[i];
}

__global__ __launch_bounds__(kThreads) void k_count_keys(const uint64_t* __restrict__ keys, int n,
                                                         int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[keys[i]], 1);
}

__global__ __launch_bounds__(kThreads) void k_zero_i32(int* __restrict__ a, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    a[i] = 0;
}

__global__ __launch_bounds__(kThreads) void k_nonempty(const int* __restrict__ start, int64_t n,
                                                       uint8_t* __restrict__ flag) {
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < n; c += int64_t(gridDim.x) * blockDim.x)
    flag[c] = start[c + 1] > start[c] ? kCellHasFacet : 0;
}

__global__ __launch_bounds__(kThreads) void k_u32_to_i32(const uint32_t* __restrict__ in, int n,
                                                         int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = int(in[i]);
}

// C_compact from the heads of equal Morton codes: code, begin, and per entry
// the hash of its cell (the sort key of the hash table) and its index.
__global__ __launch_bounds__(kThreads) void k_compact_cells(const uint64_t* __restrict__ keys, int m,
                                                            const int* __restrict__ flag, const int* __restrict__ pos,
                                                            uint64_t* __restrict__ code, int* __restrict__ begin,
                                                            uint64_t* __restrict__ hkey, uint32_t* __restrict__ idx,
                                                            uint64_t hsize) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m || !flag[i]) return;
  const int c = pos[i];
  const uint64_t k = keys[i];
  code[c] = k;
  begin[c] = i;
  hkey[c] = hash3(compact3(k), compact3(k >> 1), compact3(k >> 2), hsize);
  idx[c] = uint32_t(c);
}

__global__ __launch_bounds__(kThreads) void k_compact_lengths(const int* __restrict__ begin, int nc, int m,
                                                              int* __restrict__ length) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nc) length[c] = (c + 1 < nc ? begin[c + 1] : m) - begin[c];
}

__global__ __launch_bounds__(kThreads) void k_lookup(const double* __restrict__ pts, int n, RegGrid g,
                                                     const uint64_t* __restrict__ code, const int* __restrict__ begin,
                                                     const int* __restrict__ length, const int* __restrict__ order,
                                                     const int* __restrict__ h_begin, const int* __restrict__ h_length,
                                                     uint64_t hsize, int* __restrict__ out_begin,
                                                     int* __restrict__ out_length) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int b = -1, l = 0;
  int64_t c[3];
  bool inside = true;
  for (int q = 0; q < 3; ++q) {
    const double t = floor((pts[3 * i + q] - g.o[q]) * g.inv);
    inside = inside && t >= 0.0 && t < double(g.dims[q]);   // false for NaN
    c[q] = inside ? int64_t(t) : 0;
  }
  if (inside) {
    const uint64_t k = morton3(int(c[0]), int(c[1]), int(c[2]));
    const uint32_t h = hash3(uint32_t(c[0]), uint32_t(c[1]), uint32_t(c[2]), hsize);
    for (int q = h_begin[h], e = h_begin[h] + h_length[h]; q < e; ++q) {
      const int e2 = order[q];
      if (code[e2] == k) {
        b = begin[e2];
        l = length[e2];
        break;
      }
    }
  }
  out_begin[i] = b;
  out_length[i] = l;
}

inline int blocks(int64_t n) { return int((n + kThreads - 1) / kThreads); }

// Device buffer released at scope exit unless released.
template <class T>
struct DevBuf {
  T* p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { hipFree(p); }
  hipError_t alloc(int64_t n) {
    hipFree(p);
    p = nullptr;
    return hipMalloc(reinterpret_cast<void**>(&p), size_t(std::max<int64_t>(n, 1)) * sizeof(T));
  }
  T* release() {
    T* q = p;
    p = nullptr;
    return q;
  }
};

static int bits_for(uint64_t v) {
  int b = 0;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

// Stable sort of (keys, vals) by (key bits [0, key_bits), val bits [0,
// val_bits)), on rocPRIM's device radix sort (stable, LSD): one sort of the
// packed 64-bit (key, val) when both fit, else by val and then by key.
static fppg_status radix_sort(fppg_ctx* ctx, uint64_t*& keys, uint32_t*& vals, uint64_t*& ktmp, uint32_t*& vtmp,
                              int n, int val_bits, int key_bits, hipStream_t s) {
  if (n <= 1 || key_bits + val_bits == 0) return FPPG_OK;
  const size_t m = size_t(n);
  DevBuf<char> tmp;
  size_t bytes = 0;
  if (val_bits == 0) {
    FPPG_HIP(ctx, rocprim::radix_sort_pairs(nullptr, bytes, keys, ktmp, vals, vtmp, m, 0u, unsigned(key_bits), s));
    FPPG_HIP(ctx, tmp.alloc(int64_t(bytes)));
    FPPG_HIP(ctx, rocprim::radix_sort_pairs(tmp.p, bytes, keys, ktmp, vals, vtmp, m, 0u, unsigned(key_bits), s));
    std::swap(keys, ktmp);
    std::swap(vals, vtmp);
  } else if (key_bits + val_bits <= 64) {
    k_pack_pairs<<<blocks(n), kThreads, 0, s>>>(keys, vals, n, val_bits, ktmp);
    FPPG_HIP(ctx, hipGetLastError());
    const unsigned end = unsigned(key_bits + val_bits);
    FPPG_HIP(ctx, rocprim::radix_sort_keys(nullptr, bytes, ktmp, keys, m, 0u, end, s));
    FPPG_HIP(ctx, tmp.alloc(int64_t(bytes)));
    FPPG_HIP(ctx, rocprim::radix_sort_keys(tmp.p, bytes, ktmp, keys, m, 0u, end, s));
    k_unpack_pairs<<<blocks(n), kThreads, 0, s>>>(keys, vals, n, val_bits);
    FPPG_HIP(ctx, hipGetLastError());
  } else {
    size_t b2 = 0;
    FPPG_HIP(ctx, rocprim::radix_sort_pairs(nullptr, bytes, vals, vtmp, keys, ktmp, m, 0u, unsigned(val_bits), s));
    FPPG_HIP(ctx, rocprim::radix_sort_pairs(nullptr, b2, ktmp, keys, vtmp, vals, m, 0u, unsigned(key_bits), s));
    bytes = std::max(bytes, b2);
    FPPG_HIP(ctx, tmp.alloc(int64_t(bytes)));
    b2 = bytes;
    FPPG_HIP(ctx, rocprim::radix_sort_pairs(tmp.p, b2, vals, vtmp, keys, ktmp, m, 0u, unsigned(val_bits), s));
    b2 = bytes;
    FPPG_HIP(ctx, rocprim::radix_sort_pairs(tmp.p, b2, ktmp, keys, vtmp, vals, m, 0u, unsigned(key_bits), s));
  }
  FPPG_HIP(ctx, hipStreamSynchronize(s));   // the scratch above is freed on return
  return FPPG_OK;
}

// Drop repeated (key[, val]) entries of a sorted list: keys/vals replaced by the unique list.
static fppg_status unique_pairs(fppg_ctx* ctx, uint64_t*& keys, uint32_t*& vals, int n, int* m_out, hipStream_t s) {
  DevBuf<int> flag, pos, bsum;
  DevBuf<uint64_t> ku;
  DevBuf<uint32_t> vu;
  FPPG_HIP(ctx, flag.alloc(n));
  FPPG_HIP(ctx, pos.alloc(int64_t(n) + 1));
  FPPG_HIP(ctx, bsum.alloc(scan_blocksum_len(n)));
  if (n > 0) k_head_flags<<<blocks(n), kThreads, 0, s>>>(keys, vals, n, 1, flag.p);
  fppg_status st = exclusive_scan(ctx, flag.p, n, pos.p, bsum.p, s);
  if (st != FPPG_OK) return st;
  int m = 0;
  FPPG_HIP(ctx, hipMemcpyAsync(&m, pos.p + n, sizeof(int), hipMemcpyDeviceToHost, s));
  FPPG_HIP(ctx, hipStreamSynchronize(s));
  FPPG_HIP(ctx, ku.alloc(m));
  FPPG_HIP(ctx, vu.alloc(m));
  if (n > 0) k_compact_pairs<<<blocks(n), kThreads, 0, s>>>(keys, vals, n, flag.p, pos.p, ku.p, vu.p);
  FPPG_HIP(ctx, hipGetLastError());
  FPPG_HIP(ctx, hipStreamSynchronize(s));
  hipFree(keys);
  hipFree(vals);
  keys = ku.release();
  vals = vu.release();
  *m_out = m;
  return FPPG_OK;
}

}  // namespace reg

using namespace reg;

fppg_status radix_sort_pairs(fppg_ctx* ctx, uint64_t*& keys, uint32_t*& vals, uint64_t*& ktmp, uint32_t*& vtmp,
                             int n, int val_bits, int key_bits, hipStream_t s) {
  return radix_sort(ctx, keys, vals, ktmp, vtmp, n, val_bits, key_bits, s);
}

fppg_status register_facets(fppg_ctx* ctx, const std::vector<RegItem>& items, const std::vector<RegGrid>& grids,
                            bool morton, int key_bits, int facet_bits, RegPairs* out, hipStream_t s) {
  *out = RegPairs{};
  DevBuf<RegGrid> dg;
  FPPG_HIP(ctx, dg.alloc(int64_t(grids.size())));
  if (!grids.empty())
    FPPG_HIP(ctx, hipMemcpy(dg.p, grids.data(), grids.size() * sizeof(RegGrid), hipMemcpyHostToDevice));
  DevBuf<RegItem> cur;
  int64_t n = int64_t(items.size());
  FPPG_HIP(ctx, cur.alloc(n));
  if (n > 0) FPPG_HIP(ctx, hipMemcpy(cur.p, items.data(), size_t(n) * sizeof(RegItem), hipMemcpyHostToDevice));
  std::vector<std::pair<uint64_t*, uint32_t*>> level_pairs;
  std::vector<int64_t> level_count;
  auto free_levels = [&]() {
    for (auto& lp : level_pairs) {
      hipFree(lp.first);
      hipFree(lp.second);
    }
  };
  int64_t total = 0;
  int level = 0;
  fppg_status st = FPPG_OK;
  while (n > 0) {
    if (level >= kMaxLevels) {
      free_levels();
      return fail(ctx, FPPG_E_CAPACITY, "facet subdivision deeper than 48 levels (cell too small for the mesh)");
    }
    if (n >= (int64_t(1) << 31) - 1) {
      free_levels();
      return fail(ctx, FPPG_E_CAPACITY, "facet subdivision exceeds 2^31 triangles per level");
    }
    DevBuf<int> nch, npair, choff, poff, bsum;
    hipError_t e;
    if ((e = nch.alloc(n)) != hipSuccess || (e = npair.alloc(n)) != hipSuccess || (e = choff.alloc(n + 1)) != hipSuccess ||
        (e = poff.alloc(n + 1)) != hipSuccess || (e = bsum.alloc(scan_blocksum_len(n))) != hipSuccess) {
      free_levels();
      FPPG_HIP(ctx, e);
    }
    k_level_count<<<blocks(n), kThreads, 0, s>>>(cur.p, int(n), dg.p, nch.p, npair.p);
    if ((st = exclusive_scan(ctx, nch.p, n, choff.p, bsum.p, s)) != FPPG_OK ||
        (st = exclusive_scan(ctx, npair.p, n, poff.p, bsum.p, s)) != FPPG_OK) {
      free_levels();
      return st;
    }
    int nc = 0, np = 0;
    if ((e = hipMemcpyAsync(&nc, choff.p + n, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&np, poff.p + n, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
      free_levels();
      FPPG_HIP(ctx, e);
    }
    DevBuf<RegItem> next;
    DevBuf<uint64_t> pk;
    DevBuf<uint32_t> pf;
    if ((e = next.alloc(nc)) != hipSuccess || (e = pk.alloc(np)) != hipSuccess || (e = pf.alloc(np)) != hipSuccess) {
      free_levels();
      FPPG_HIP(ctx, e);
    }
    k_level_write<<<blocks(n), kThreads, 0, s>>>(cur.p, int(n), dg.p, choff.p, poff.p, next.p, pk.p, pf.p,
                                                 morton ? 1 : 0);
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess) {
      free_levels();
      FPPG_HIP(ctx, e);
    }
    level_pairs.emplace_back(pk.release(), pf.release());
    level_count.push_back(np);
    total += np;
    if (total >= (int64_t(1) << 31) - 1) {
      free_levels();
      return fail(ctx, FPPG_E_CAPACITY, "facet registration exceeds 2^31 entries");
    }
    std::swap(cur.p, next.p);
    n = nc;
    ++level;
  }
  // all levels' pairs in one list
  DevBuf<uint64_t> keys, ktmp;
  DevBuf<uint32_t> vals, vtmp;
  hipError_t e;
  if ((e = keys.alloc(total)) != hipSuccess || (e = vals.alloc(total)) != hipSuccess ||
      (e = ktmp.alloc(total)) != hipSuccess || (e = vtmp.alloc(total)) != hipSuccess) {
    free_levels();
    FPPG_HIP(ctx, e);
  }
  int64_t off = 0;
  for (size_t l = 0; l < level_pairs.size(); ++l) {
    const int64_t c = level_count[l];
    if (c > 0 &&
        ((e = hipMemcpyAsync(keys.p + off, level_pairs[l].first, size_t(c) * 8, hipMemcpyDeviceToDevice, s)) !=
             hipSuccess ||
         (e = hipMemcpyAsync(vals.p + off, level_pairs[l].second, size_t(c) * 4, hipMemcpyDeviceToDevice, s)) !=
             hipSuccess)) {
      free_levels();
      FPPG_HIP(ctx, e);
    }
    off += c;
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) {
    free_levels();
    FPPG_HIP(ctx, e);
  }
  free_levels();
  st = radix_sort(ctx, keys.p, vals.p, ktmp.p, vtmp.p, int(total), facet_bits, key_bits, s);
  if (st != FPPG_OK) return st;
  int m = 0;
  st = unique_pairs(ctx, keys.p, vals.p, int(total), &m, s);
  if (st != FPPG_OK) return st;
  out->keys = keys.release();
  out->facets = vals.release();
  out->n = m;
  out->levels = level;
  return FPPG_OK;
}

fppg_status registration_csr(fppg_ctx* ctx, const RegPairs& pairs, int64_t n_cells, int** start, int** tri,
                             uint8_t** flag, hipStream_t s) {
  DevBuf<int> cnt, st_, tr, bsum;
  DevBuf<uint8_t> fl;
  FPPG_HIP(ctx, cnt.alloc(n_cells));
  FPPG_HIP(ctx, st_.alloc(n_cells + 1));
  FPPG_HIP(ctx, tr.alloc(pairs.n));
  FPPG_HIP(ctx, fl.alloc(n_cells));
  FPPG_HIP(ctx, bsum.alloc(scan_blocksum_len(n_cells)));
  const int g = int(std::min<int64_t>(blocks(n_cells), 4096));
  k_zero_i32<<<std::max(g, 1), kThreads, 0, s>>>(cnt.p, n_cells);
  if (pairs.n > 0) {
    k_count_keys<<<blocks(pairs.n), kThreads, 0, s>>>(pairs.keys, int(pairs.n), cnt.p);
    k_u32_to_i32<<<blocks(pairs.n), kThreads, 0, s>>>(pairs.facets, int(pairs.n), tr.p);
  }
  fppg_status r = exclusive_scan(ctx, cnt.p, n_cells, st_.p, bsum.p, s);
  if (r != FPPG_OK) return r;
  k_nonempty<<<std::max(g, 1), kThreads, 0, s>>>(st_.p, n_cells, fl.p);
  FPPG_HIP(ctx, hipGetLastError());
  FPPG_HIP(ctx, hipStreamSynchronize(s));
  *start = st_.release();
  *tri = tr.release();
  *flag = fl.release();
  return FPPG_OK;
}

}  // namespace fppg

using namespace fppg;

struct fppg_sparse_grid {
  int device;
  RegGrid grid;
  int64_t n_leaf_levels;
  int64_t m;        // facet list length
  int64_t nc;       // C_compact length
  uint64_t hsize;   // H_size
  int* facets;      // [m]
  uint64_t* code;   // [nc]
  int* begin;       // [nc]
  int* length;      // [nc]
  int* order;       // [nc]
  int* h_begin;     // [hsize]
  int* h_length;    // [hsize]
};

static void free_sparse(fppg_sparse_grid* g) {
  if (!g) return;
  hipFree(g->facets);
  hipFree(g->code);
  hipFree(g->begin);
  hipFree(g->length);
  hipFree(g->order);
  hipFree(g->h_begin);
  hipFree(g->h_length);
  delete g;
}

extern "C" fppg_status fppg_sparse_grid_create(fppg_ctx* ctx, const double* vert, int32_t n_vert, const int32_t* tri,
                                               int32_t n_tri, const double origin[3], double cell,
                                               const int32_t dims[3], double pad, int64_t hash_size,
                                               fppg_sparse_grid** out) {
  if (!ctx || !out) return fail(ctx, FPPG_E_ARG, "null ctx/out");
  *out = nullptr;
  if (n_vert < 0 || n_tri < 0 || (n_vert > 0 && !vert) || (n_tri > 0 && !tri) || !origin || !dims)
    return fail(ctx, FPPG_E_ARG, "null or negative mesh argument");
  if (!(cell > 0.0) || !std::isfinite(cell) || !(pad >= 0.0) || !std::isfinite(pad))
    return fail(ctx, FPPG_E_ARG, "cell must be finite and > 0, pad finite and >= 0");
  for (int q = 0; q < 3; ++q) {
    if (!std::isfinite(origin[q])) return fail(ctx, FPPG_E_ARG, "origin must be finite");
    if (dims[q] < 1 || dims[q] > (1 << 21)) return fail(ctx, FPPG_E_ARG, "dims must lie in [1, 2^21]");
  }
  if (hash_size < 0 || hash_size >= (int64_t(1) << 31)) return fail(ctx, FPPG_E_ARG, "hash_size out of range");
  for (int32_t t = 0; t < 3 * n_tri; ++t)
    if (tri[t] < 0 || tri[t] >= n_vert) return fail(ctx, FPPG_E_ARG, "vertex index out of range");
  for (int32_t v = 0; v < 3 * n_vert; ++v)
    if (!std::isfinite(vert[v])) return fail(ctx, FPPG_E_ARG, "non-finite vertex");
  RegGrid g{};
  for (int q = 0; q < 3; ++q) {
    g.o[q] = origin[q];
    g.dims[q] = dims[q];
  }
  g.cell = cell;
  g.inv = 1.0 / cell;
  g.pad = pad;
  g.key_begin = 0;
  std::vector<RegItem> items(static_cast<size_t>(n_tri));
  for (int32_t t = 0; t < n_tri; ++t) {
    RegItem& it = items[size_t(t)];
    for (int q = 0; q < 3; ++q) {
      it.a[q] = vert[3 * tri[3 * t] + q];
      it.b[q] = vert[3 * tri[3 * t + 1] + q];
      it.c[q] = vert[3 * tri[3 * t + 2] + q];
    }
    it.facet = t;
    it.grid = 0;
  }
  hipStream_t s = nullptr;
  RegPairs p{};
  int max_dim = std::max(dims[0], std::max(dims[1], dims[2]));
  fppg_status st = register_facets(ctx, items, std::vector<RegGrid>{g}, true, 3 * bits_for(uint64_t(max_dim - 1)),
                                   bits_for(uint64_t(std::max(n_tri - 1, 0))), &p, s);
  if (st != FPPG_OK) return st;
  fppg_sparse_grid* sg = new (std::nothrow) fppg_sparse_grid{};
  if (!sg) {
    hipFree(p.keys);
    hipFree(p.facets);
    return fail(ctx, FPPG_E_CAPACITY, "out of host memory");
  }
  sg->device = ctx->device;
  sg->grid = g;
  sg->n_leaf_levels = p.levels;
  sg->m = p.n;
  const int m = int(p.n);
  // facets as int32 (the pair list's own values)
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&sg->facets), size_t(std::max(m, 1)) * 4);
  if (e == hipSuccess && m > 0) k_u32_to_i32<<<blocks(m), kThreads, 0, s>>>(p.facets, m, sg->facets);
  // C_compact: heads of equal codes
  DevBuf<int> flag, pos, bsum;
  DevBuf<uint64_t> hkey, hk2;
  DevBuf<uint32_t> idx, idx2;
  if (e == hipSuccess) e = flag.alloc(m);
  if (e == hipSuccess) e = pos.alloc(int64_t(m) + 1);
  if (e == hipSuccess) e = bsum.alloc(scan_blocksum_len(m));
  if (e != hipSuccess) {
    hipFree(p.keys);
    hipFree(p.facets);
    free_sparse(sg);
    FPPG_HIP(ctx, e);
  }
  if (m > 0) k_head_flags<<<blocks(m), kThreads, 0, s>>>(p.keys, p.facets, m, 0, flag.p);
  st = exclusive_scan(ctx, flag.p, m, pos.p, bsum.p, s);
  int nc = 0;
  if (st == FPPG_OK) {
    e = hipMemcpy(&nc, pos.p + m, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) st = fail(ctx, FPPG_E_HIP, hipGetErrorString(e));
  }
  const uint64_t H = hash_size > 0 ? uint64_t(hash_size) : uint64_t(std::max(nc, 1));
  sg->nc = nc;
  sg->hsize = H;
  if (st == FPPG_OK) {
    if ((e = hipMalloc(reinterpret_cast<void**>(&sg->code), size_t(std::max(nc, 1)) * 8)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&sg->begin), size_t(std::max(nc, 1)) * 4)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&sg->length), size_t(std::max(nc, 1)) * 4)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&sg->order), size_t(std::max(nc, 1)) * 4)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&sg->h_begin), size_t(H) * 4 + 4)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&sg->h_length), size_t(H) * 4)) != hipSuccess ||
        (e = hkey.alloc(nc)) != hipSuccess || (e = hk2.alloc(nc)) != hipSuccess || (e = idx.alloc(nc)) != hipSuccess ||
        (e = idx2.alloc(nc)) != hipSuccess)
      st = fail(ctx, FPPG_E_HIP, hipGetErrorString(e));
  }
  if (st == FPPG_OK) {
    if (m > 0) {
      k_compact_cells<<<blocks(m), kThreads, 0, s>>>(p.keys, m, flag.p, pos.p, sg->code, sg->begin, hkey.p, idx.p, H);
      k_compact_lengths<<<blocks(nc), kThreads, 0, s>>>(sg->begin, nc, m, sg->length);
    }
    // the hash table: entries by (hash, morton), counts per value, their prefix
    uint64_t* hk = hkey.p;
    uint32_t* ix = idx.p;
    uint64_t* hk_t = hk2.p;
    uint32_t* ix_t = idx2.p;
    st = radix_sort(ctx, hk, ix, hk_t, ix_t, nc, 0, bits_for(H - 1), s);
    if (st == FPPG_OK) {
      DevBuf<int> hcnt, hb;
      if ((e = hcnt.alloc(int64_t(H))) != hipSuccess || (e = hb.alloc(scan_blocksum_len(int64_t(H)))) != hipSuccess) {
        st = fail(ctx, FPPG_E_HIP, hipGetErrorString(e));
      } else {
        const int gz = int(std::min<int64_t>(blocks(int64_t(H)), 4096));
        k_zero_i32<<<std::max(gz, 1), kThreads, 0, s>>>(hcnt.p, int64_t(H));
        if (nc > 0) {
          k_count_keys<<<blocks(nc), kThreads, 0, s>>>(hk, nc, hcnt.p);
          k_u32_to_i32<<<blocks(nc), kThreads, 0, s>>>(ix, nc, sg->order);
        }
        st = exclusive_scan(ctx, hcnt.p, int64_t(H), sg->h_begin, hb.p, s);
        if (st == FPPG_OK &&
            (e = hipMemcpyAsync(sg->h_length, hcnt.p, size_t(H) * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess)
          st = fail(ctx, FPPG_E_HIP, hipGetErrorString(e));
        if (st == FPPG_OK && (e = hipStreamSynchronize(s)) != hipSuccess) st = fail(ctx, FPPG_E_HIP, hipGetErrorString(e));
      }
    }
    // radix_sort swapped the pointers: free whichever buffers the DevBufs no longer own
    hkey.p = hk;
    hk2.p = hk_t;
    idx.p = ix;
    idx2.p = ix_t;
  }
  hipFree(p.keys);
  hipFree(p.facets);
  if (st != FPPG_OK) {
    free_sparse(sg);
    return st;
  }
  *out = sg;
  return FPPG_OK;
}

extern "C" fppg_status fppg_sparse_grid_info(const fppg_sparse_grid* sg, fppg_sparse_grid_view* v) {
  if (!sg || !v) return FPPG_E_ARG;
  v->n_entry = sg->m;
  v->n_cell = sg->nc;
  v->hash_size = int64_t(sg->hsize);
  v->levels = sg->n_leaf_levels;
  v->facets = sg->facets;
  v->morton = sg->code;
  v->begin = sg->begin;
  v->length = sg->length;
  v->order = sg->order;
  v->h_begin = sg->h_begin;
  v->h_length = sg->h_length;
  return FPPG_OK;
}

extern "C" fppg_status fppg_sparse_grid_copy(fppg_ctx* ctx, const fppg_sparse_grid* sg, int32_t* facets,
                                             uint64_t* morton, int32_t* begin, int32_t* length, int32_t* order,
                                             int32_t* h_begin, int32_t* h_length, void* stream) {
  if (!ctx || !sg) return fail(ctx, FPPG_E_ARG, "null ctx/grid");
  if (sg->device != ctx->device) return fail(ctx, FPPG_E_ARG, "grid and context on different devices");
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    return (dst && bytes) ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s) : hipSuccess;
  };
  FPPG_HIP(ctx, cp(facets, sg->facets, size_t(sg->m) * 4));
  FPPG_HIP(ctx, cp(morton, sg->code, size_t(sg->nc) * 8));
  FPPG_HIP(ctx, cp(begin, sg->begin, size_t(sg->nc) * 4));
  FPPG_HIP(ctx, cp(length, sg->length, size_t(sg->nc) * 4));
  FPPG_HIP(ctx, cp(order, sg->order, size_t(sg->nc) * 4));
  FPPG_HIP(ctx, cp(h_begin, sg->h_begin, size_t(sg->hsize) * 4 + 4));
  FPPG_HIP(ctx, cp(h_length, sg->h_length, size_t(sg->hsize) * 4));
  return FPPG_OK;
}

extern "C" fppg_status fppg_sparse_grid_lookup(fppg_ctx* ctx, const fppg_sparse_grid* sg, int64_t n,
                                               const double* points, int32_t* begin, int32_t* length, void* stream) {
  if (!ctx || !sg) return fail(ctx, FPPG_E_ARG, "null ctx/grid");
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(ctx, FPPG_E_ARG, "n out of range");
  if (n > 0 && (!points || !begin || !length)) return fail(ctx, FPPG_E_ARG, "null argument");
  if (sg->device != ctx->device) return fail(ctx, FPPG_E_ARG, "grid and context on different devices");
  if (n == 0) return FPPG_OK;
  k_lookup<<<blocks(n), kThreads, 0, static_cast<hipStream_t>(stream)>>>(
      points, int(n), sg->grid, sg->code, sg->begin, sg->length, sg->order, sg->h_begin, sg->h_length, sg->hsize,
      begin, length);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

extern "C" fppg_status fppg_sparse_grid_destroy(fppg_sparse_grid* sg) {
  free_sparse(sg);
  return FPPG_OK;
}

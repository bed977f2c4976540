// Feature extraction and feature-line particles (section 3.2.2) on the GPU.
//
//   edges        the 3 edges of every facet as 64-bit keys (smaller vertex in
//                the high word) with their facet, radix-sorted (rocPRIM):
//                the runs of equal keys are the mesh edges with their facets.
//                (Compactions: exclusive scans in one block, in index order.)
//   feature      a run of other than two facets, or two facets whose FP64 unit
//                normals satisfy n1 . n2 < cos_threshold (sums of three
//                products left to right); compacted in key order.
//   singular     vertices on one feature edge or on more than two.
//   lines        one thread per (singular vertex, feature neighbour) walks
//                the chain to the next singular vertex and keeps it if its
//                (start, second) pair is the smaller of the two ends; then
//                one thread per unvisited vertex of degree two walks its
//                loop and keeps it if it is the loop's smallest vertex
//                (oriented towards the smaller neighbour). Lines in (start,
//                second) order, loops after them.
//   particles    one thread per line: n = max(1, ceil(L / dx)) equal steps
//                of arc length; interior points of open lines, all n points
//                of loops.
// Compactions use exclusive scans in index order, so every output is
// deterministic.
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

#include "internal.h"

namespace fppg {
namespace feat {

__device__ __forceinline__ double dot3(const double* u, const double* v) { return (u[0] * v[0] + u[1] * v[1]) + u[2] * v[2]; }

__global__ void k_edge_keys(const int* __restrict__ tri, int n_tri, unsigned long long* __restrict__ key,
                            int* __restrict__ fac) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 3 * n_tri) return;
  const int t = q / 3, k = q % 3;
  const int u = tri[3 * t + k], v = tri[3 * t + (k + 1) % 3];
  const unsigned a = unsigned(min(u, v)), b = unsigned(max(u, v));
  key[q] = (static_cast<unsigned long long>(a) << 32) | b;
  fac[q] = t;
}

__global__ void k_normals(const double* __restrict__ vert, const int* __restrict__ tri, int n_tri,
                          double* __restrict__ nrm) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tri) return;
  const double* A = vert + 3 * tri[3 * t];
  const double* B = vert + 3 * tri[3 * t + 1];
  const double* C = vert + 3 * tri[3 * t + 2];
  const double e0[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
  const double e1[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
  const double n[3] = {e0[1] * e1[2] - e0[2] * e1[1], e0[2] * e1[0] - e0[0] * e1[2], e0[0] * e1[1] - e0[1] * e1[0]};
  const double len = sqrt(dot3(n, n));
  for (int q = 0; q < 3; ++q) nrm[3 * t + q] = n[q] / len;
}

// flag[i] = 1 at the start of every run of equal keys that is a feature edge
__global__ void k_edge_flags(const unsigned long long* __restrict__ key, const int* __restrict__ fac, int m,
                             const double* __restrict__ nrm, double cos_threshold, int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int f = 0;
  if (i == 0 || key[i] != key[i - 1]) {
    int e = i + 1;
    while (e < m && key[e] == key[i]) ++e;
    if (e - i != 2) f = 1;
    else f = dot3(nrm + 3 * fac[i], nrm + 3 * fac[i + 1]) < cos_threshold ? 1 : 0;
  }
  flag[i] = f;
}

__global__ void k_edge_write(const unsigned long long* __restrict__ key, const int* __restrict__ flag,
                             const int* __restrict__ off, int m, int* __restrict__ edges, int* __restrict__ deg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m || !flag[i]) return;
  const int u = int(key[i] >> 32), v = int(key[i] & 0xffffffffu);
  edges[2 * off[i]] = u;
  edges[2 * off[i] + 1] = v;
  atomicAdd(&deg[u], 1);
  atomicAdd(&deg[v], 1);
}

__global__ void k_flag_singular(const int* __restrict__ deg, int n, int* __restrict__ flag) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) flag[v] = (deg[v] != 0 && deg[v] != 2) ? 1 : 0;
}

__global__ void k_write_index(const int* __restrict__ flag, const int* __restrict__ off, int n, int* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && flag[v]) out[off[v]] = v;
}

// adjacency lists: fill, then sort each (short) list ascending
__global__ void k_adj_fill(const int* __restrict__ edges, int ne, const int* __restrict__ aoff, int* __restrict__ cur,
                           int* __restrict__ adj) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int u = edges[2 * e], v = edges[2 * e + 1];
  adj[aoff[u] + atomicAdd(&cur[u], 1)] = v;
  adj[aoff[v] + atomicAdd(&cur[v], 1)] = u;
}

__global__ void k_adj_sort(const int* __restrict__ aoff, const int* __restrict__ deg, int n, int* __restrict__ adj) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int* a = adj + aoff[v];
  for (int i = 1; i < deg[v]; ++i) {
    const int x = a[i];
    int j = i - 1;
    while (j >= 0 && a[j] > x) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = x;
  }
}

__device__ __forceinline__ int other(const int* __restrict__ adj, const int* __restrict__ aoff, int cur, int prev) {
  const int a = adj[aoff[cur]], b = adj[aoff[cur] + 1];
  return a == prev ? b : a;
}

// One thread per adjacency slot p of a singular vertex s: walk to the next
// singular vertex. pass 0: len[p] = vertex count if the line is kept, else 0;
// pass 1: write it at line_off[p] and mark its interior vertices.
__global__ void k_trace_lines(const int* __restrict__ adj, const int* __restrict__ aoff, const int* __restrict__ deg,
                              const int* __restrict__ owner_of_slot, int nslot, int pass, int* __restrict__ len,
                              const int* __restrict__ line_off, int* __restrict__ line_vert, int* __restrict__ vis) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nslot) return;
  const int s = owner_of_slot[p];
  if (deg[s] == 2) {
    if (pass == 0) len[p] = 0;
    return;
  }
  const int w = adj[p];
  int prev = s, cur = w, cnt = 2;
  while (deg[cur] == 2) {
    const int nx = other(adj, aoff, cur, prev);
    prev = cur;
    cur = nx;
    ++cnt;
  }
  const bool keep = s < cur || (s == cur && w < prev);
  if (pass == 0) {
    len[p] = keep ? cnt : 0;
    return;
  }
  if (!keep) return;
  int o = line_off[p];
  line_vert[o++] = s;
  prev = s;
  cur = w;
  while (deg[cur] == 2) {
    line_vert[o++] = cur;
    vis[cur] = 1;
    const int nx = other(adj, aoff, cur, prev);
    prev = cur;
    cur = nx;
  }
  line_vert[o] = cur;
}

// One thread per vertex of degree two not on a line: if it is the smallest
// vertex of its loop, pass 0 stores the loop's vertex count, pass 1 writes the
// loop from it towards its smaller neighbour.
__global__ void k_trace_loops(const int* __restrict__ adj, const int* __restrict__ aoff, const int* __restrict__ deg,
                              const int* __restrict__ vis, int n, int pass, int* __restrict__ len,
                              const int* __restrict__ loop_off, int* __restrict__ line_vert) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  bool keep = deg[v] == 2 && !vis[v];
  int cnt = 0;
  if (keep) {
    int prev = v, cur = adj[aoff[v]];
    cnt = 1;
    while (cur != v) {
      if (cur < v) {
        keep = false;
        break;
      }
      const int nx = other(adj, aoff, cur, prev);
      prev = cur;
      cur = nx;
      ++cnt;
    }
  }
  if (pass == 0) {
    len[v] = keep ? cnt : 0;
    return;
  }
  if (!keep) return;
  int o = loop_off[v];
  const int first = adj[aoff[v]];   // the smaller neighbour (lists are ascending)
  line_vert[o++] = v;
  int prev = v, cur = first;
  while (cur != v) {
    line_vert[o++] = cur;
    const int nx = other(adj, aoff, cur, prev);
    prev = cur;
    cur = nx;
  }
}

__device__ __forceinline__ double seg_len(const double* __restrict__ vert, int a, int b) {
  const double d[3] = {vert[3 * b] - vert[3 * a], vert[3 * b + 1] - vert[3 * a + 1], vert[3 * b + 2] - vert[3 * a + 2]};
  return sqrt(dot3(d, d));
}

// vertex k of line l, with a loop closed by its first vertex
__device__ __forceinline__ int lv(const int* __restrict__ line_vert, int b, int nv, bool closed, int k) {
  return (closed && k == nv) ? line_vert[b] : line_vert[b + k];
}

__global__ void k_line_particles(const double* __restrict__ vert, const int* __restrict__ line_begin,
                                 const int* __restrict__ line_vert, const uint8_t* __restrict__ closed, int n_lines,
                                 double dx, int pass, int* __restrict__ cnt, const int* __restrict__ poff,
                                 float4* __restrict__ pos, int* __restrict__ line_of, double* __restrict__ arc,
                                 int* __restrict__ seg_of, double* __restrict__ u_in) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_lines) return;
  const int b = line_begin[l], nv = line_begin[l + 1] - b;
  const bool cl = closed[l] != 0;
  const int nseg = cl ? nv : nv - 1;
  double L = 0.0;
  for (int i = 0; i < nseg; ++i) L += seg_len(vert, lv(line_vert, b, nv, cl, i), lv(line_vert, b, nv, cl, i + 1));
  const int n = max(1, int(ceil(L / dx)));
  const int k0 = cl ? 0 : 1;
  if (pass == 0) {
    cnt[l] = n - k0;
    return;
  }
  int o = poff[l];
  // the targets grow with k, so the segment walk resumes where the previous
  // particle's stopped (acc is the same left-to-right sum of the lengths)
  double acc = 0.0;
  int i = 0;
  for (int k = k0; k < n; ++k) {
    const double target = k * (L / n);
    while (i < nseg - 1) {
      const double len = seg_len(vert, lv(line_vert, b, nv, cl, i), lv(line_vert, b, nv, cl, i + 1));
      if (!(acc + len < target)) break;
      acc += len;
      ++i;
    }
    const int pa = lv(line_vert, b, nv, cl, i), pb = lv(line_vert, b, nv, cl, i + 1);
    const double t = (target - acc) / seg_len(vert, pa, pb);
    float p[3];
    for (int q = 0; q < 3; ++q) p[q] = float(vert[3 * pa + q] + t * (vert[3 * pb + q] - vert[3 * pa + q]));
    pos[o] = make_float4(p[0], p[1], p[2], __int_as_float(FPPG_TAG_FEATURE));
    line_of[o] = l;
    arc[o] = target;
    seg_of[o] = i;
    u_in[o] = target - acc;
    ++o;
  }
}

__global__ void k_slot_owner(const int* __restrict__ aoff, const int* __restrict__ deg, int n, int* __restrict__ own) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  for (int k = 0; k < deg[v]; ++k) own[aoff[v] + k] = v;
}

__global__ void k_line_begin(const int* __restrict__ lens, const int* __restrict__ off, int nslot,
                             const int* __restrict__ loop_len, const int* __restrict__ loop_off, int nvert,
                             int base_vert, int base_line_loops, const int* __restrict__ line_index,
                             const int* __restrict__ loop_index, int* __restrict__ line_begin,
                             uint8_t* __restrict__ closed) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nslot && lens[q] > 0) {
    line_begin[line_index[q]] = off[q];
    closed[line_index[q]] = 0;
  }
  if (q < nvert && loop_len[q] > 0) {
    line_begin[base_line_loops + loop_index[q]] = base_vert + loop_off[q];
    closed[base_line_loops + loop_index[q]] = 1;
  }
}

__global__ void k_nonzero(const int* __restrict__ a, int n, int* __restrict__ f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = a[i] > 0 ? 1 : 0;
}

__global__ void k_set_last(int* __restrict__ a, int idx, int v) { a[idx] = v; }

constexpr int kScanThreads = 1024;

// exclusive scan of in [n] into out [n], the total into *total; one block:
// each thread sums a contiguous run, the run totals are scanned once
// (Hillis-Steele), then each thread writes its run's prefix sums
__global__ __launch_bounds__(kScanThreads) void k_scan1(const int* __restrict__ in, int* __restrict__ out, int n,
                                                        int* __restrict__ total) {
  __shared__ int sh[kScanThreads];
  const int per = (n + kScanThreads - 1) / kScanThreads;
  const int i0 = min(n, int(threadIdx.x) * per), i1 = min(n, i0 + per);
  int v = 0;
  for (int i = i0; i < i1; ++i) v += in[i];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const int add = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - v;
  for (int i = i0; i < i1; ++i) {
    const int x = in[i];
    out[i] = run;
    run += x;
  }
  if (threadIdx.x == kScanThreads - 1) *total = sh[kScanThreads - 1];
}

// Multi-block exclusive scan for long arrays: tiles of kTile = 256 threads x 8
// consecutive items; the tile sums, their one-block scan (k_scan1), then each
// tile rescanned with its offset.
constexpr int kTileThreads = 256, kTileItems = 8, kTile = kTileThreads * kTileItems;

// exclusive scan of one value per thread over a 256-thread block; returns the prefix, *total the sum
__device__ __forceinline__ int tile_block_scan(int v, int* total) {
  __shared__ int wsum[kTileThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kTileThreads / 64; ++k) {
    before += k < w ? wsum[k] : 0;
    tot += wsum[k];
  }
  *total = tot;
  return before + inc - v;
}

__global__ __launch_bounds__(kTileThreads) void k_tile_sums(const int* __restrict__ in, int n, int* __restrict__ sums) {
  const int i0 = blockIdx.x * kTile + threadIdx.x * kTileItems;
  int v = 0;
#pragma unroll
  for (int q = 0; q < kTileItems; ++q) v += i0 + q < n ? in[i0 + q] : 0;
  int total;
  tile_block_scan(v, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kTileThreads) void k_tile_apply(const int* __restrict__ in, int n,
                                                             const int* __restrict__ offs, int* __restrict__ out) {
  const int i0 = blockIdx.x * kTile + threadIdx.x * kTileItems;
  int x[kTileItems];
  int v = 0;
#pragma unroll
  for (int q = 0; q < kTileItems; ++q) {
    x[q] = i0 + q < n ? in[i0 + q] : 0;
    v += x[q];
  }
  int total;
  int run = offs[blockIdx.x] + tile_block_scan(v, &total);
#pragma unroll
  for (int q = 0; q < kTileItems; ++q) {
    if (i0 + q < n) out[i0 + q] = run;
    run += x[q];
  }
}

inline int nb(int64_t n) { return int(std::max<int64_t>(1, (n + 255) / 256)); }   // kernels check bounds

}  // namespace feat
}  // namespace fppg

using namespace fppg;

namespace {

struct Dev {
  std::vector<void*> p;
  hipStream_t s = nullptr;   // work that may still use the buffers (an early return) ends first
  ~Dev() {
    hipStreamSynchronize(s);
    for (void* q : p) hipFree(q);
  }
  template <class T>
  T* alloc(size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(1, n) * sizeof(T)) != hipSuccess) return nullptr;
    p.push_back(q);
    return static_cast<T*>(q);
  }
};

// exclusive scan of n ints into out in one block (a set-up call: the sizes
// are the mesh's); returns the total
bool scan(Dev& d, const int* in, int* out, int n, hipStream_t s, int* total) {
  if (n == 0) {
    *total = 0;
    return true;
  }
  int* tot = d.alloc<int>(1);
  if (!tot) return false;
  if (n <= feat::kTile) {
    feat::k_scan1<<<1, feat::kScanThreads, 0, s>>>(in, out, n, tot);
  } else {
    const int nt = (n + feat::kTile - 1) / feat::kTile;
    int* sums = d.alloc<int>(nt);
    int* offs = d.alloc<int>(nt);
    if (!sums || !offs) return false;
    feat::k_tile_sums<<<nt, feat::kTileThreads, 0, s>>>(in, n, sums);
    feat::k_scan1<<<1, feat::kScanThreads, 0, s>>>(sums, offs, nt, tot);
    feat::k_tile_apply<<<nt, feat::kTileThreads, 0, s>>>(in, n, offs, out);
  }
  if (hipGetLastError() != hipSuccess) return false;
  if (hipMemcpyAsync(total, tot, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
  return hipStreamSynchronize(s) == hipSuccess;
}

}  // namespace

extern "C" fppg_status fppg_features(fppg_ctx* ctx, const double* vert, int32_t n_vert, const int32_t* tri,
                                     int32_t n_tri, double cos_threshold, double dx, fppg_features_out* out,
                                     void* stream) {
  if (!ctx) return fail(ctx, FPPG_E_ARG, "null ctx");
  if (!vert || !tri || !out || n_vert < 3 || n_tri < 1) return fail(ctx, FPPG_E_ARG, "null or empty mesh/output");
  if (!(dx > 0.0) || !std::isfinite(dx) || !std::isfinite(cos_threshold))
    return fail(ctx, FPPG_E_ARG, "dx must be finite and > 0, cos_threshold finite");
  if (int64_t(n_tri) * 3 >= (int64_t(1) << 31)) return fail(ctx, FPPG_E_CAPACITY, "too many facets");
  for (int64_t q = 0; q < 3 * int64_t(n_tri); ++q)
    if (tri[q] < 0 || tri[q] >= n_vert) return fail(ctx, FPPG_E_ARG, "facet vertex index out of range");
  if (!aligned(out->pos, 16)) return fail(ctx, FPPG_E_ARG, "pos must be 16-byte aligned");
  out->n_edges = out->n_singular = out->n_lines = out->n_line_vert = out->n_particles = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Dev d;
  d.s = s;
  const int m = 3 * n_tri;
  double* d_vert = d.alloc<double>(3 * size_t(n_vert));
  int* d_tri = d.alloc<int>(3 * size_t(n_tri));
  unsigned long long* k0 = d.alloc<unsigned long long>(m);
  unsigned long long* k1 = d.alloc<unsigned long long>(m);
  int* f0 = d.alloc<int>(m);
  int* f1 = d.alloc<int>(m);
  double* nrm = d.alloc<double>(3 * size_t(n_tri));
  int* flag = d.alloc<int>(std::max(m, n_vert) + 1);
  int* off = d.alloc<int>(std::max(m, n_vert) + 1);
  int* deg = d.alloc<int>(n_vert);
  if (!d_vert || !d_tri || !k0 || !k1 || !f0 || !f1 || !nrm || !flag || !off || !deg)
    return fail(ctx, FPPG_E_HIP, "device allocation failed");
  FPPG_HIP(ctx, hipMemcpyAsync(d_vert, vert, sizeof(double) * 3 * n_vert, hipMemcpyHostToDevice, s));
  FPPG_HIP(ctx, hipMemcpyAsync(d_tri, tri, sizeof(int) * 3 * n_tri, hipMemcpyHostToDevice, s));
  FPPG_HIP(ctx, hipMemsetAsync(deg, 0, sizeof(int) * n_vert, s));
  feat::k_edge_keys<<<feat::nb(m), 256, 0, s>>>(d_tri, n_tri, k0, f0);
  feat::k_normals<<<feat::nb(n_tri), 256, 0, s>>>(d_vert, d_tri, n_tri, nrm);
  size_t tb = 0;
  FPPG_HIP(ctx, rocprim::radix_sort_pairs(nullptr, tb, k0, k1, f0, f1, m, 0, 64, s));
  void* tmp = d.alloc<char>(tb);
  if (!tmp) return fail(ctx, FPPG_E_HIP, "device allocation failed");
  FPPG_HIP(ctx, rocprim::radix_sort_pairs(tmp, tb, k0, k1, f0, f1, m, 0, 64, s));
  feat::k_edge_flags<<<feat::nb(m), 256, 0, s>>>(k1, f1, m, nrm, cos_threshold, flag);
  int ne = 0;
  if (!scan(d, flag, off, m, s, &ne)) return fail(ctx, FPPG_E_HIP, "scan failed");
  int* edges = d.alloc<int>(2 * size_t(ne));
  if (!edges) return fail(ctx, FPPG_E_HIP, "device allocation failed");
  feat::k_edge_write<<<feat::nb(m), 256, 0, s>>>(k1, flag, off, m, edges, deg);
  // singular vertices
  feat::k_flag_singular<<<feat::nb(n_vert), 256, 0, s>>>(deg, n_vert, flag);
  int nsing = 0;
  if (!scan(d, flag, off, n_vert, s, &nsing)) return fail(ctx, FPPG_E_HIP, "scan failed");
  int* sing = d.alloc<int>(nsing);
  if (!sing) return fail(ctx, FPPG_E_HIP, "device allocation failed");
  feat::k_write_index<<<feat::nb(n_vert), 256, 0, s>>>(flag, off, n_vert, sing);
  // adjacency
  int* aoff = d.alloc<int>(n_vert + 1);
  int nslot = 0;
  if (!aoff || !scan(d, deg, aoff, n_vert, s, &nslot)) return fail(ctx, FPPG_E_HIP, "scan failed");
  int* adj = d.alloc<int>(nslot);
  int* cur = d.alloc<int>(n_vert);
  int* own = d.alloc<int>(nslot);
  int* vis = d.alloc<int>(n_vert);
  int* lens = d.alloc<int>(nslot + 1);
  int* loff = d.alloc<int>(nslot + 1);
  int* looplen = d.alloc<int>(n_vert + 1);
  int* loopoff = d.alloc<int>(n_vert + 1);
  int* lidx = d.alloc<int>(nslot + 1);
  int* pidx = d.alloc<int>(n_vert + 1);
  if (!adj || !cur || !own || !vis || !lens || !loff || !looplen || !loopoff || !lidx || !pidx)
    return fail(ctx, FPPG_E_HIP, "device allocation failed");
  FPPG_HIP(ctx, hipMemsetAsync(cur, 0, sizeof(int) * n_vert, s));
  FPPG_HIP(ctx, hipMemsetAsync(vis, 0, sizeof(int) * n_vert, s));
  feat::k_adj_fill<<<feat::nb(ne), 256, 0, s>>>(edges, ne, aoff, cur, adj);
  feat::k_adj_sort<<<feat::nb(n_vert), 256, 0, s>>>(aoff, deg, n_vert, adj);
  feat::k_slot_owner<<<feat::nb(n_vert), 256, 0, s>>>(aoff, deg, n_vert, own);
  // open lines
  feat::k_trace_lines<<<feat::nb(nslot), 256, 0, s>>>(adj, aoff, deg, own, nslot, 0, lens, nullptr, nullptr, nullptr);
  int nlv_open = 0, nl_open = 0;
  if (!scan(d, lens, loff, nslot, s, &nlv_open)) return fail(ctx, FPPG_E_HIP, "scan failed");
  feat::k_nonzero<<<feat::nb(nslot), 256, 0, s>>>(lens, nslot, flag);
  if (!scan(d, flag, lidx, nslot, s, &nl_open)) return fail(ctx, FPPG_E_HIP, "scan failed");
  // line vertices: open lines then loops (the loop pass needs the visited marks)
  const int64_t cap_lv = out->cap_line_vert;
  int* lvert = d.alloc<int>(size_t(nlv_open) + n_vert + 1);
  if (!lvert) return fail(ctx, FPPG_E_HIP, "device allocation failed");
  feat::k_trace_lines<<<feat::nb(nslot), 256, 0, s>>>(adj, aoff, deg, own, nslot, 1, lens, loff, lvert, vis);
  feat::k_trace_loops<<<feat::nb(n_vert), 256, 0, s>>>(adj, aoff, deg, vis, n_vert, 0, looplen, nullptr, nullptr);
  int nlv_loop = 0, nl_loop = 0;
  if (!scan(d, looplen, loopoff, n_vert, s, &nlv_loop)) return fail(ctx, FPPG_E_HIP, "scan failed");
  feat::k_nonzero<<<feat::nb(n_vert), 256, 0, s>>>(looplen, n_vert, flag);
  if (!scan(d, flag, pidx, n_vert, s, &nl_loop)) return fail(ctx, FPPG_E_HIP, "scan failed");
  feat::k_trace_loops<<<feat::nb(n_vert), 256, 0, s>>>(adj, aoff, deg, vis, n_vert, 1, looplen, loopoff,
                                                        lvert + nlv_open);
  const int n_lines = nl_open + nl_loop, n_lv = nlv_open + nlv_loop;
  int* lbegin = d.alloc<int>(n_lines + 1);
  uint8_t* lclosed = d.alloc<uint8_t>(n_lines + 1);
  if (!lbegin || !lclosed) return fail(ctx, FPPG_E_HIP, "device allocation failed");
  feat::k_line_begin<<<feat::nb(std::max(nslot, n_vert)), 256, 0, s>>>(lens, loff, nslot, looplen, loopoff, n_vert,
                                                                       nlv_open, nl_open, lidx, pidx, lbegin, lclosed);
  feat::k_set_last<<<1, 1, 0, s>>>(lbegin, n_lines, n_lv);
  // particles
  int* pcnt = d.alloc<int>(n_lines + 1);
  int* poff = d.alloc<int>(n_lines + 1);
  if (!pcnt || !poff) return fail(ctx, FPPG_E_HIP, "device allocation failed");
  feat::k_line_particles<<<feat::nb(n_lines), 256, 0, s>>>(d_vert, lbegin, lvert, lclosed, n_lines, dx, 0, pcnt,
                                                           nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  int np = 0;
  if (!scan(d, pcnt, poff, n_lines, s, &np)) return fail(ctx, FPPG_E_HIP, "scan failed");
  out->n_edges = ne;
  out->n_singular = nsing;
  out->n_lines = n_lines;
  out->n_line_vert = n_lv;
  out->n_particles = np;
  if (!out->line_begin) {   // a size query
    FPPG_HIP(ctx, hipStreamSynchronize(s));
    return FPPG_OK;
  }
  if (ne > out->cap_edges || nsing > out->cap_singular || n_lines > out->cap_lines || n_lv > cap_lv ||
      np > out->cap_particles) {
    FPPG_HIP(ctx, hipStreamSynchronize(s));
    return fail(ctx, FPPG_E_CAPACITY, "an output exceeds its capacity (the counts hold the sizes needed)");
  }
  if ((ne && !out->edges) || (nsing && !out->singular) || (n_lines && !out->line_closed) ||
      (n_lv && !out->line_vert) || (np && (!out->pos || !out->line_of || !out->arc || !out->seg || !out->u))) {
    FPPG_HIP(ctx, hipStreamSynchronize(s));
    return fail(ctx, FPPG_E_ARG, "null output array");
  }
  feat::k_line_particles<<<feat::nb(n_lines), 256, 0, s>>>(d_vert, lbegin, lvert, lclosed, n_lines, dx, 1, pcnt,
                                                           poff, reinterpret_cast<float4*>(out->pos), out->line_of,
                                                           out->arc, out->seg, out->u);
  FPPG_HIP(ctx, hipGetLastError());
  if (ne) FPPG_HIP(ctx, hipMemcpyAsync(out->edges, edges, sizeof(int) * 2 * ne, hipMemcpyDeviceToDevice, s));
  if (nsing) FPPG_HIP(ctx, hipMemcpyAsync(out->singular, sing, sizeof(int) * nsing, hipMemcpyDeviceToDevice, s));
  FPPG_HIP(ctx, hipMemcpyAsync(out->line_begin, lbegin, sizeof(int) * (n_lines + 1), hipMemcpyDeviceToDevice, s));
  if (n_lines)
    FPPG_HIP(ctx, hipMemcpyAsync(out->line_closed, lclosed, n_lines, hipMemcpyDeviceToDevice, s));
  if (n_lv) FPPG_HIP(ctx, hipMemcpyAsync(out->line_vert, lvert, sizeof(int) * n_lv, hipMemcpyDeviceToDevice, s));
  FPPG_HIP(ctx, hipStreamSynchronize(s));
  return FPPG_OK;
}

// Cell-list rebuild by counting sort (the "updating data structures" step of
// Algorithm 1). The final order is (cell key, particle id): deterministic,
// whatever order the atomics of the counting pass complete in.
//
//   fill      count[c] = 0
//   key       key_i of every particle (non-finite positions: the quarantine
//             key ncell, after every geometry), rank_i = arrival index in its cell
//             (one atomic per run of equal keys in a wavefront: the input is
//             the previous iteration's sorted order, so runs are long)
//   scan      cell_start = exclusive prefix sum of count (reduce / top / down)
//   scatter   slot = cell_start[key] + rank: id, source index and key to slot
//   final     inside each cell, the rank of the particle's id among the cell's
//             ids gives its final slot; gather pos/id/owner there. A lane counts
//             the smaller ids of its cell, which bounds the work at
//             kRankDirect^2 per cell; a fuller cell (a clump, or the quarantine
//             cell of many non-finite particles) is listed instead, and
//             k_final_big sorts it: ids sorted in LDS chunks, then merged in
//             passes of doubling width (O(m log m) per cell of m particles)
#include "internal.h"

namespace fppg {

__device__ __forceinline__ int cell_key(const float4 p, const GeomDev& G) {
  // binary32, one rounding per operation (file compiled without FP contraction)
  float tx = (p.x - G.origin[0]) * G.inv_cell_x;
  float ty = (p.y - G.origin[1]) * G.inv_cell;
  float tz = (p.z - G.origin[2]) * G.inv_cell;
  tx = fminf(fmaxf(tx, 0.0f), float(G.dims[0] - 1));   // fmaxf(NaN, 0) = 0
  ty = fminf(fmaxf(ty, 0.0f), float(G.dims[1] - 1));
  tz = fminf(fmaxf(tz, 0.0f), float(G.dims[2] - 1));
  const int cx = int(floorf(tx)), cy = int(floorf(ty)), cz = int(floorf(tz));
  return row_key(G, cy, cz) + cx;
}

__global__ void k_fill_i32(int* __restrict__ a, int64_t n, int v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    a[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_key_count(const float4* __restrict__ pos, int n,
                                                      const GeomDev* __restrict__ geoms, int n_geom,
                                                      int quarantine, int* __restrict__ key,
                                                      int* __restrict__ rank, int* __restrict__ count,
                                                      uint32_t* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int k = -1;
  if (i < n) {
    const float4 p = pos[i];
    int g = geom_of(p.w);
    if (g >= n_geom) {
      atomicOr(status, FPPG_S_BAD_INDEX);
      g = n_geom - 1;
    }
    if (isfinite(p.x) && isfinite(p.y) && isfinite(p.z)) {
      k = cell_key(p, geoms[g]);
    } else {
      atomicOr(status, FPPG_S_NONFINITE_POS);
      k = quarantine;   // after every geometry's cells: no stencil reaches it
    }
  }
  // runs of equal keys among consecutive lanes share one atomic
  const int kprev = __shfl_up(k, 1);
  const bool head = (lane == 0) || (kprev != k);
  const uint64_t heads = __ballot(head);
  const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1);
  const int start = 63 - __clzll(heads & upto);
  const uint64_t above = heads & ~upto;
  const int end = above ? (__ffsll((long long)above) - 1) : 64;
  int base = 0;
  if (head && k >= 0) base = atomicAdd(&count[k], end - lane);
  base = __shfl(base, start);
  if (i < n) {
    key[i] = k;
    rank[i] = base + (lane - start);
  }
}

// Block-wide exclusive scan of 8 items per thread (1024 threads); a thread's
// items are read (and written) as two 16-byte vectors where the array is
// 16-byte aligned and the items are all in range.
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// The kScanItems items of a thread starting at base (0 past the end).
__device__ __forceinline__ void load_items(const int* __restrict__ a, int64_t base, int64_t n, int v[kScanItems]) {
  if (base + kScanItems <= n && aligned16(a)) {
    const int4 x = *reinterpret_cast<const int4*>(a + base);
    const int4 y = *reinterpret_cast<const int4*>(a + base + 4);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
    return;
  }
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) v[q] = (base + q < n) ? a[base + q] : 0;
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

// returns the exclusive prefix of `v` over the block and the block total
__device__ __forceinline__ int block_excl_scan(int v, int* total) {
  __shared__ int wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int inc = wave_incl_scan(v, lane);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    int s = lane < kScanThreads / 64 ? wsum[lane] : 0;
    s = wave_incl_scan(s, lane);
    if (lane < kScanThreads / 64) wsum[lane] = s;
  }
  __syncthreads();
  const int before = wid > 0 ? wsum[wid - 1] : 0;
  *total = wsum[kScanThreads / 64 - 1];
  __syncthreads();
  return before + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int* __restrict__ count, int64_t ncell,
                                                              int* __restrict__ blocksum) {
  const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  int v[kScanItems];
  load_items(count, base, ncell, v);
  int s = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) s += v[q];
  int total;
  block_excl_scan(s, &total);
  if (threadIdx.x == 0) blocksum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(int* __restrict__ blocksum, int nb) {
  int carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kScanThreads) {
    const int b = b0 + threadIdx.x;
    const int v = b < nb ? blocksum[b] : 0;
    int total;
    const int ex = block_excl_scan(v, &total);
    if (b < nb) blocksum[b] = carry + ex;
    carry += total;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const int* __restrict__ count, int64_t ncell,
                                                            const int* __restrict__ blocksum,
                                                            int* __restrict__ cell_start, int n) {
  const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  int v[kScanItems];
  load_items(count, base, ncell, v);
  int s = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) s += v[q];
  int total;
  int ex = block_excl_scan(s, &total) + blocksum[blockIdx.x];
  int o[kScanItems];
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    o[q] = ex;
    ex += v[q];
  }
  if (base + kScanItems <= ncell && aligned16(cell_start)) {
    *reinterpret_cast<int4*>(cell_start + base) = make_int4(o[0], o[1], o[2], o[3]);
    *reinterpret_cast<int4*>(cell_start + base + 4) = make_int4(o[4], o[5], o[6], o[7]);
  } else {
#pragma unroll
    for (int q = 0; q < kScanItems; ++q)
      if (base + q < ncell) cell_start[base + q] = o[q];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) cell_start[ncell] = n;   // ncell here counts the quarantine cell
}

__global__ __launch_bounds__(kBlock) void k_scatter(const int* __restrict__ key, const int* __restrict__ rank,
                                                    const int* __restrict__ id, const int* __restrict__ cell_start,
                                                    int n, int* __restrict__ tmp_id, int* __restrict__ tmp_src,
                                                    int* __restrict__ tmp_key) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = key[i];
  const int slot = cell_start[k] + rank[i];
  tmp_id[slot] = id[i];
  tmp_src[slot] = i;
  tmp_key[slot] = k;
}

// Cells of more particles than this are ranked by k_final_big.
constexpr int kRankDirect = 64;

__global__ __launch_bounds__(kBlock) void k_final(const int* __restrict__ tmp_id, const int* __restrict__ tmp_src,
                                                  const int* __restrict__ tmp_key, const int* __restrict__ cell_start,
                                                  int n, const float4* __restrict__ pos_in,
                                                  const int* __restrict__ owner_in, float4* __restrict__ pos_out,
                                                  int* __restrict__ id_out, int* __restrict__ owner_out,
                                                  int* __restrict__ big, int* __restrict__ big_count) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int k = tmp_key[s];
  const int my = tmp_id[s];
  const int src = tmp_src[s];
  const int b = cell_start[k], e = cell_start[k + 1];
  const float4 p = pos_in[src];
  const int o = owner_in[src];
  // Three rounds of dependent loads instead of five: the entry, then the cell
  // bounds beside the gathers, then the rank loop. The empty statement takes
  // the values so that the compiler keeps the loads here rather than sinking
  // them past the loop to their only use (it contains no instruction).
  asm volatile("" ::"v"(p.x), "v"(p.y), "v"(p.z), "v"(p.w), "v"(o), "v"(my));
  if (e - b > kRankDirect) {
    if (s == b) big[atomicAdd(big_count, 1)] = k;   // one entry per cell; the list's order does not matter
    return;
  }
  int r = 0;
  for (int t = b; t < e; ++t) r += tmp_id[t] < my;
  const int dst = b + r;
  pos_out[dst] = p;
  id_out[dst] = my;
  owner_out[dst] = o;
}

constexpr int kBigThreads = 1024;
constexpr int kBigChunk = 4096;   // (id, source) pairs sorted together in LDS
constexpr int kBigBlocks = 64;

// (id, source slot) as one unsigned key ordered as (signed id, slot)
__device__ __forceinline__ uint64_t id_slot_key(int id, int slot) {
  return (uint64_t(uint32_t(id) ^ 0x80000000u) << 32) | uint32_t(slot);
}

// Ascending bitonic sort of kBigChunk keys in LDS by the whole block.
__device__ void lds_bitonic_sort(uint64_t* sh) {
  for (int size = 2; size <= kBigChunk; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < kBigChunk / 2; t += kBigThreads) {
        const int lo = 2 * t - (t & (stride - 1));   // the partner index with the stride bit clear
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t a = sh[lo], c = sh[hi];
        if ((a > c) == up) {
          sh[lo] = c;
          sh[hi] = a;
        }
      }
      __syncthreads();
    }
}

// Number of entries of the sorted run [lo, hi) of (id, src) below (x, xs), or
// at or below it with `upto` (a stable merge: left-run entries count the right
// run's smaller keys, right-run entries the left run's smaller or equal ones).
__device__ __forceinline__ int run_rank(const int* __restrict__ rid, const int* __restrict__ rsrc, int lo, int hi,
                                        int x, int xs, bool upto) {
  const int base = lo;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int y = rid[mid], ys = rsrc[mid];
    const bool before = (y < x) || (y == x && (upto ? ys <= xs : ys < xs));
    if (before)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo - base;
}

// One block per listed cell (blocks stride over the list): the cell's slots
// [b, e) of tmp_id / tmp_src are sorted by (id, source) — chunks of kBigChunk
// in LDS, written back in place, then merge passes ping-ponging with the same
// slots of two scratch arrays (the key and rank arrays of the counting pass,
// free by now) — and gathered to the output.
__global__ __launch_bounds__(kBigThreads) void k_final_big(int* __restrict__ tmp_id, int* __restrict__ tmp_src,
                                                           const int* __restrict__ cell_start,
                                                           const int* __restrict__ big,
                                                           const int* __restrict__ big_count,
                                                           int* __restrict__ scratch_id, int* __restrict__ scratch_src,
                                                           const float4* __restrict__ pos_in,
                                                           const int* __restrict__ owner_in,
                                                           float4* __restrict__ pos_out, int* __restrict__ id_out,
                                                           int* __restrict__ owner_out) {
  __shared__ uint64_t sh[kBigChunk];
  const int nbig = *big_count;
  for (int c = blockIdx.x; c < nbig; c += gridDim.x) {
    const int k = big[c];
    const int b = cell_start[k], m = cell_start[k + 1] - b;
    for (int c0 = 0; c0 < m; c0 += kBigChunk) {
      const int len = min(kBigChunk, m - c0);
      for (int t = threadIdx.x; t < kBigChunk; t += kBigThreads)
        sh[t] = t < len ? id_slot_key(tmp_id[b + c0 + t], tmp_src[b + c0 + t]) : ~0ull;
      __syncthreads();
      lds_bitonic_sort(sh);
      for (int t = threadIdx.x; t < len; t += kBigThreads) {
        tmp_id[b + c0 + t] = int(uint32_t(sh[t] >> 32) ^ 0x80000000u);
        tmp_src[b + c0 + t] = int(uint32_t(sh[t]));
      }
      __syncthreads();
    }
    int *aid = tmp_id + b, *asrc = tmp_src + b, *bid = scratch_id + b, *bsrc = scratch_src + b;
    for (int64_t w = kBigChunk; w < m; w *= 2) {
      for (int p = threadIdx.x; p < m; p += kBigThreads) {
        const int pair = int(p / (2 * w) * (2 * w));
        const bool left = p < pair + w;
        const int os = int(left ? pair + w : pair);              // the other run of the pair
        const int oe = int(left ? std::min<int64_t>(pair + 2 * w, m) : pair + w);
        const int x = aid[p], xs = asrc[p];
        const int own = int(p - (left ? pair : pair + w));
        const int other = os < oe ? run_rank(aid, asrc, os, oe, x, xs, !left) : 0;
        bid[pair + own + other] = x;
        bsrc[pair + own + other] = xs;
      }
      __syncthreads();
      int* t = aid; aid = bid; bid = t;
      t = asrc; asrc = bsrc; bsrc = t;
    }
    for (int r = threadIdx.x; r < m; r += kBigThreads) {
      const int src = asrc[r];
      pos_out[b + r] = pos_in[src];
      id_out[b + r] = aid[r];
      owner_out[b + r] = owner_in[src];
    }
    __syncthreads();
  }
}

// ---- list of the moving particles (sorted indices, ascending) -----------------------------

__device__ __forceinline__ bool moving_at(const float4* __restrict__ pos, int i, int n, uint32_t move_mask) {
  return i < n && is_moving(tag_of(pos[i].w), move_mask);
}

// moving lanes below this one in the block, and the block's total
__device__ __forceinline__ int block_rank(bool m, int* total) {
  __shared__ int wcnt[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint64_t b = __ballot(m);
  if (lane == 0) wcnt[wid] = __popcll(b);
  __syncthreads();
  int before = 0, t = 0;
  for (int w = 0; w < kBlock / 64; ++w) {
    if (w < wid) before += wcnt[w];
    t += wcnt[w];
  }
  *total = t;
  __syncthreads();
  return before + __popcll(b & ((1ull << lane) - 1ull));
}

__global__ __launch_bounds__(kBlock) void k_list_count(const float4* __restrict__ pos, int n, uint32_t move_mask,
                                                       int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int total;
  block_rank(moving_at(pos, i, n, move_mask), &total);
  if (threadIdx.x == 0) cnt[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_list_write(const float4* __restrict__ pos, int n, uint32_t move_mask,
                                                       const int* __restrict__ offs, int nb,
                                                       int* __restrict__ list, int* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool m = moving_at(pos, i, n, move_mask);
  int total;
  const int r = block_rank(m, &total);
  if (m) list[offs[blockIdx.x] + r] = i;
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) count[0] = offs[blockIdx.x] + total;
}

// ---- tier partition: the particles a tier reaches first -----------------------------------
// A particle is reached when its class rank is at most R, the highest rank of
// the moving classes: the movers and every class they take as a source.

__device__ __forceinline__ bool reached_at(const float4* __restrict__ pos, int i, int n, int R) {
  return i < n && rank_of(tag_of(pos[i].w)) <= R;
}

__global__ __launch_bounds__(kBlock) void k_part_count(const float4* __restrict__ pos, int n, int R,
                                                       int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int total;
  block_rank(reached_at(pos, i, n, R), &total);
  if (threadIdx.x == 0) cnt[blockIdx.x] = total;
}

// offs = exclusive prefix of cnt over the blocks: reached particles go to
// offs[b] + (reached lanes below), the others after all reached ones in the
// same relative order
__global__ __launch_bounds__(kBlock) void k_part_write(const float4* __restrict__ pos_in,
                                                       const int* __restrict__ id_in,
                                                       const int* __restrict__ owner_in, int n, int R,
                                                       const int* __restrict__ cnt, const int* __restrict__ offs,
                                                       int nb, float4* __restrict__ pos_out,
                                                       int* __restrict__ id_out, int* __restrict__ owner_out,
                                                       int* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool m = reached_at(pos_in, i, n, R);
  int total;
  const int r = block_rank(m, &total);
  const int reached = offs[nb - 1] + cnt[nb - 1];
  if (i < n) {
    const int dst = m ? offs[blockIdx.x] + r
                      : reached + (blockIdx.x * kBlock - offs[blockIdx.x]) + (int(threadIdx.x) - r);
    pos_out[dst] = pos_in[i];
    id_out[dst] = id_in[i];
    owner_out[dst] = owner_in[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) count[0] = reached;
}

static inline int grid_for(int64_t n, int block) { return int((n + block - 1) / block); }

__global__ void k_scan_total(const int* __restrict__ in, int64_t n, int* __restrict__ out) {
  if (threadIdx.x == 0) out[n] = n > 0 ? out[n - 1] + in[n - 1] : 0;
}

fppg_status exclusive_scan(fppg_ctx* ctx, const int* in, int64_t n, int* out, int* blocksum, hipStream_t s) {
  const int nb = int((n + kScanTile - 1) / kScanTile);
  if (n > 0) {
    k_scan_reduce<<<nb, kScanThreads, 0, s>>>(in, n, blocksum);
    k_scan_top<<<1, kScanThreads, 0, s>>>(blocksum, nb);
    k_scan_down<<<nb, kScanThreads, 0, s>>>(in, n, blocksum, out, 0);
  }
  k_scan_total<<<1, 64, 0, s>>>(in, n, out);   // after k_scan_down, which writes out[n] = 0
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

int64_t scan_blocksum_len(int64_t n) { return (n + kScanTile - 1) / kScanTile + 2; }

}  // namespace fppg

using namespace fppg;

extern "C" fppg_status fppg_build_cells(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos_in,
                                        const int32_t* id_in, const int32_t* owner_in, float* pos_out,
                                        int32_t* id_out, int32_t* owner_out, int32_t* cell_start, void* ws,
                                        size_t ws_bytes, void* stream) {
  if (!ctx || !geom) return fail(ctx, FPPG_E_ARG, "null ctx/geom");
  if (n != geom->n_active) return fail(ctx, FPPG_E_ARG, "n differs from the active particle count of the geometry");
  if (n > 0 && (!pos_in || !id_in || !owner_in || !pos_out || !id_out || !owner_out))
    return fail(ctx, FPPG_E_ARG, "null particle array");
  if (!cell_start || !ws) return fail(ctx, FPPG_E_ARG, "null cell_start/ws");
  if (!aligned(pos_in, 16) || !aligned(pos_out, 16) || !aligned(ws, 256))
    return fail(ctx, FPPG_E_ARG, "pos must be 16-byte and ws 256-byte aligned");
  if (n > 0 && (pos_in == pos_out || id_in == id_out || owner_in == owner_out))
    return fail(ctx, FPPG_E_ARG, "build_cells output must not alias its input");
  const WsLayout L = ws_layout(geom, n);
  if (ws_bytes < L.build_end) return fail(ctx, FPPG_E_WORKSPACE, "workspace too small for build_cells");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  int* key = reinterpret_cast<int*>(w + L.key);
  int* rank = reinterpret_cast<int*>(w + L.rank);
  int* tmp_id = reinterpret_cast<int*>(w + L.tmp_id);
  int* tmp_src = reinterpret_cast<int*>(w + L.tmp_src);
  int* tmp_key = reinterpret_cast<int*>(w + L.tmp_key);
  int* count = reinterpret_cast<int*>(w + L.count);
  int* blocksum = reinterpret_cast<int*>(w + L.blocksum);
  int* big = reinterpret_cast<int*>(w + L.big);
  const int64_t nc = geom->ncell + 1;   // the geometries' cells and the quarantine cell
  int* big_count = count + nc;          // the slot after the scanned counts
  const int nb = int((nc + kScanTile - 1) / kScanTile);
  const int ni = int(n);
  PhaseTimer timer(ctx, 0, s);
  k_fill_i32<<<std::min(grid_for(nc + 1, kBlock), 4096), kBlock, 0, s>>>(count, nc + 1, 0);
  if (ni > 0)
    k_key_count<<<grid_for(ni, kBlock), kBlock, 0, s>>>(reinterpret_cast<const float4*>(pos_in), ni, geom->d_geom,
                                                        geom->n_geom, int(geom->ncell), key, rank, count,
                                                        ctx->d_status);
  k_scan_reduce<<<nb, kScanThreads, 0, s>>>(count, nc, blocksum);
  k_scan_top<<<1, kScanThreads, 0, s>>>(blocksum, nb);
  k_scan_down<<<nb, kScanThreads, 0, s>>>(count, nc, blocksum, cell_start, ni);
  if (ni > 0) {
    k_scatter<<<grid_for(ni, kBlock), kBlock, 0, s>>>(key, rank, id_in, cell_start, ni, tmp_id, tmp_src, tmp_key);
    k_final<<<grid_for(ni, kBlock), kBlock, 0, s>>>(tmp_id, tmp_src, tmp_key, cell_start, ni,
                                                    reinterpret_cast<const float4*>(pos_in), owner_in,
                                                    reinterpret_cast<float4*>(pos_out), id_out, owner_out,
                                                    big, big_count);
    k_final_big<<<kBigBlocks, kBigThreads, 0, s>>>(tmp_id, tmp_src, cell_start, big, big_count, key, rank,
                                                   reinterpret_cast<const float4*>(pos_in), owner_in,
                                                   reinterpret_cast<float4*>(pos_out), id_out, owner_out);
  }
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

extern "C" fppg_status fppg_moving_list(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                        uint32_t move_mask, int32_t* list, int32_t* count, void* ws,
                                        size_t ws_bytes, void* stream) {
  if (!ctx || !geom) return fail(ctx, FPPG_E_ARG, "null ctx/geom");
  if (n != geom->n_active) return fail(ctx, FPPG_E_ARG, "n differs from the active particle count of the geometry");
  if (!count || !ws || (n > 0 && (!pos || !list))) return fail(ctx, FPPG_E_ARG, "null argument");
  if (!aligned(pos, 16) || !aligned(ws, 256)) return fail(ctx, FPPG_E_ARG, "pos must be 16-byte and ws 256-byte aligned");
  const WsLayout L = ws_layout(geom, n);
  if (ws_bytes < L.list_end) return fail(ctx, FPPG_E_WORKSPACE, "workspace too small for moving_list");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n == 0) {
    k_fill_i32<<<1, kBlock, 0, s>>>(count, 1, 0);
    FPPG_HIP(ctx, hipGetLastError());
    return FPPG_OK;
  }
  char* w = static_cast<char*>(ws);
  int* cnt = reinterpret_cast<int*>(w + L.list_cnt);
  int* offs = reinterpret_cast<int*>(w + L.list_offs);
  int* bsum = reinterpret_cast<int*>(w + L.list_bsum);
  const int ni = int(n);
  const int nb = grid_for(ni, kBlock);
  const int nt = int((int64_t(nb) + kScanTile - 1) / kScanTile);
  const float4* p4 = reinterpret_cast<const float4*>(pos);
  k_list_count<<<nb, kBlock, 0, s>>>(p4, ni, move_mask, cnt);
  k_scan_reduce<<<nt, kScanThreads, 0, s>>>(cnt, nb, bsum);
  k_scan_top<<<1, kScanThreads, 0, s>>>(bsum, nt);
  k_scan_down<<<nt, kScanThreads, 0, s>>>(cnt, nb, bsum, offs, 0);
  k_list_write<<<nb, kBlock, 0, s>>>(p4, ni, move_mask, offs, nb, list, count);
  FPPG_HIP(ctx, hipGetLastError());
  return FPPG_OK;
}

extern "C" fppg_status fppg_tier_partition(fppg_ctx* ctx, fppg_geom* geom, int64_t n, float* pos_in, int32_t* id_in,
                                           int32_t* owner_in, float* pos_out, int32_t* id_out, int32_t* owner_out,
                                           uint32_t move_mask, int64_t* n_active, void* ws, size_t ws_bytes,
                                           void* stream) {
  if (!ctx || !geom || !n_active) return fail(ctx, FPPG_E_ARG, "null ctx/geom/n_active");
  if (n != geom->n_part) return fail(ctx, FPPG_E_ARG, "n differs from the particle count of the geometry descriptors");
  if (n > 0 && (!pos_in || !id_in || !owner_in || !pos_out || !id_out || !owner_out))
    return fail(ctx, FPPG_E_ARG, "null particle array");
  if (!ws || !aligned(pos_in, 16) || !aligned(pos_out, 16) || !aligned(ws, 256))
    return fail(ctx, FPPG_E_ARG, "null ws, or pos not 16-byte / ws not 256-byte aligned");
  if (n > 0 && (pos_in == pos_out || id_in == id_out || owner_in == owner_out))
    return fail(ctx, FPPG_E_ARG, "tier_partition output must not alias its input");
  const WsLayout L = ws_layout(geom, n);
  if (ws_bytes < L.list_end) return fail(ctx, FPPG_E_WORKSPACE, "workspace too small for tier_partition");
  int R = -1;
  for (int t = FPPG_TAG_FEATURE; t <= FPPG_TAG_VOLUME; ++t)
    if ((move_mask >> t) & 1u) R = t;   // rank_of(t) = t for these classes
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = int(n);
  int na = ni;
  if (ni > 0 && R >= 0 && R < FPPG_TAG_VOLUME) {
    char* w = static_cast<char*>(ws);
    int* cnt = reinterpret_cast<int*>(w + L.list_cnt);
    int* offs = reinterpret_cast<int*>(w + L.list_offs);
    int* bsum = reinterpret_cast<int*>(w + L.list_bsum);
    int* dcount = cnt + grid_for(ni, kBlock);   // list_cnt holds nb + 1 ints
    const int nb = grid_for(ni, kBlock);
    const int nt = int((int64_t(nb) + kScanTile - 1) / kScanTile);
    k_part_count<<<nb, kBlock, 0, s>>>(reinterpret_cast<const float4*>(pos_in), ni, R, cnt);
    k_scan_reduce<<<nt, kScanThreads, 0, s>>>(cnt, nb, bsum);
    k_scan_top<<<1, kScanThreads, 0, s>>>(bsum, nt);
    k_scan_down<<<nt, kScanThreads, 0, s>>>(cnt, nb, bsum, offs, 0);
    k_part_write<<<nb, kBlock, 0, s>>>(reinterpret_cast<const float4*>(pos_in), id_in, owner_in, ni, R, cnt, offs,
                                       nb, reinterpret_cast<float4*>(pos_out), id_out, owner_out, dcount);
    FPPG_HIP(ctx, hipGetLastError());
    FPPG_HIP(ctx, hipMemcpyAsync(&na, dcount, sizeof(int), hipMemcpyDeviceToHost, s));
    FPPG_HIP(ctx, hipStreamSynchronize(s));
    if (na < ni) {   // the unreached tail into the input buffers too: both halves of a double buffer hold it
      const size_t t = size_t(ni - na);
      FPPG_HIP(ctx, hipMemcpyAsync(pos_in + 4 * size_t(na), pos_out + 4 * size_t(na), 16 * t,
                                   hipMemcpyDeviceToDevice, s));
      FPPG_HIP(ctx, hipMemcpyAsync(id_in + na, id_out + na, 4 * t, hipMemcpyDeviceToDevice, s));
      FPPG_HIP(ctx, hipMemcpyAsync(owner_in + na, owner_out + na, 4 * t, hipMemcpyDeviceToDevice, s));
    }
  } else if (ni > 0) {   // every particle is reached (or nothing moves): order unchanged
    FPPG_HIP(ctx, hipMemcpyAsync(pos_out, pos_in, 16 * size_t(ni), hipMemcpyDeviceToDevice, s));
    FPPG_HIP(ctx, hipMemcpyAsync(id_out, id_in, 4 * size_t(ni), hipMemcpyDeviceToDevice, s));
    FPPG_HIP(ctx, hipMemcpyAsync(owner_out, owner_in, 4 * size_t(ni), hipMemcpyDeviceToDevice, s));
  }
  FPPG_HIP(ctx, hipStreamSynchronize(s));
  geom->n_active = na;
  *n_active = na;
  return FPPG_OK;
}

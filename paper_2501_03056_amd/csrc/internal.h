// Internal definitions shared by the HIP translation units of libfppg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fppg.h"

namespace fppg {

constexpr int kBlock = 256;          // threads per block of the streaming kernels
// The particle cells are the cells of the caller's grid split in kXSplit along
// x: a receiver's stencil rows then end within half a cell of its support
// sphere instead of a whole cell (fewer candidates per row).
constexpr int kXSplit = 2;
constexpr int kMaxGeom = 1 << 16;    // geometry index lives in bits 8..23 of pos.w

// Per-geometry descriptor as the kernels read it (device array, one per geometry).
struct GeomDev {
  float origin[3];
  float inv_cell;   // 1 / cell edge along y and z
  float inv_cell_x; // kXSplit inv_cell (exact): 1 / cell edge along x
  int32_t dims[3];  // particle cells per axis (dims[0] = kXSplit times the caller's)
  int32_t k;
  float h;
  float rc2;        // fl32(fl32(2h)^2)
  float R;          // projection radius
  float kcoef;      // K = 5 alpha / h^2 (binary32)
  float inv_slab;   // fl32(1 / slab)
  int64_t cell_begin;
  int64_t part_begin, part_end;
  // facet search grid
  double tg_origin[3];
  double tg_inv;    // 1 / search-cell edge
  int32_t tg_dims[3];
  int32_t slab;     // rows of cells along y per slab of the cell key (1..dims[1])
  int64_t tg_begin; // offset of this geometry's cells in the global search-cell arrays
  int32_t tri_begin, tri_end, seg_begin, seg_end;
  int32_t csg_op;            // FPPG_CSG_*: the facets are those of convex parts combined by a Boolean operation
  int32_t part_begin_csg, part_end_csg;   // global part range of an assembly
  int32_t max_level;         // multi-resolution levels 0..max_level (0: one smoothing length)
};

// Boolean assemblies: per global facet its part where a point test is needed
// (-1: not in an assembly, or a facet wholly on the assembly's boundary; a
// facet never on it is not in the facet search grid), per part its plane
// range, planes (n, d) with n.x - d < 0 inside the part.
struct PartDev {
  int32_t plane_begin, plane_end;   // range in the plane array
  double lo[3], hi[3];              // bounding box of the part's vertices
};

struct CsgDev {
  const int* facet_part = nullptr;
  const uint8_t* facet_mask = nullptr;   // per facet: bit j = the facet crosses part (first part + j) of its assembly
  const PartDev* part = nullptr;
  const double4* plane = nullptr;
};

// FP64 facet frame for the projection and crossing tests.
struct FacetDev {
  double a[3];      // vertex A
  double n[3];      // unit outward normal
  double e0[3];     // B - A
  double e1[3];     // C - A
  double d00, d01, d11, inv_den;  // Gram matrix of (e0, e1) and 1/det
};

// FP64 feature segment: start point, unit tangent, length, its line's segment range.
struct SegDev {
  double p0[3];
  double t[3];
  double len;
  int32_t lo, hi;   // global segment range [lo, hi) of the segment's line
  int32_t closed;
  int32_t pad;
};

// Search-cell flag: the cell holds at least one facet.
constexpr uint8_t kCellHasFacet = 1;

struct Geom {
  int32_t n_geom = 0;
  int32_t k = 1;
  int64_t ncell = 0;
  int64_t n_tri = 0, n_seg = 0;
  int64_t tg_cells = 0, tg_entries = 0;
  int64_t n_part = 0;
  int64_t n_active = 0;             // particles the per-iteration calls take (a tier's reached prefix)
  int64_t n_vert = 0;               // mesh vertices over the batch
  std::vector<GeomDev> host;
  GeomDev* d_geom = nullptr;
  FacetDev* d_facet = nullptr;
  float4* d_n32 = nullptr;          // binary32 unit normals (tangential projection)
  int4* d_tri_vert = nullptr;       // global vertex ids of each facet (A, B, C, 0)
  SegDev* d_seg = nullptr;
  int2* d_seg_vert = nullptr;       // global vertex ids of each segment end (-1: none)
  int32_t* d_tg_start = nullptr;    // [tg_cells + 1]
  int32_t* d_tg_tri = nullptr;      // [tg_entries] global facet ids
  uint8_t* d_tg_flag = nullptr;     // [tg_cells]
  int32_t* d_facet_part = nullptr;  // [n_tri] part of each facet in an assembly, -1 otherwise
  PartDev* d_part = nullptr;        // [n_parts] plane range and bounding box of each part
  uint8_t* d_facet_mask = nullptr;  // [n_tri] the parts a facet's points must be tested against
  double4* d_plane = nullptr;       // [n_planes]
  bool has_csg = false;
  bool has_levels = false;   // some geometry is multi-resolution
  CsgDev csg() const { return CsgDev{d_facet_part, d_facet_mask, d_part, d_plane}; }
  int device = 0;
};

}  // namespace fppg

namespace fppg {
constexpr int kProfSlots = 4096;
struct PhaseProf {
  std::vector<hipEvent_t> start, stop;
  int used = 0;          // event pairs recorded since the last read
  double ms = 0.0;       // accumulated at read time
  int64_t launches = 0;
};
}  // namespace fppg

struct fppg_ctx {
  int device = 0;
  std::string err;
  uint32_t* d_status = nullptr;     // device status word
  uint32_t profiling = 0;   // bit p: time phase p
  fppg::PhaseProf prof[FPPG_NPHASES];
  int force_block = 256;    // launch shape of the force kernel (fppg_set_launch)
  int xcd_remap = 1;         // 0 round-robin, 1 contiguous per XCD, 2 runs (launch_chunk)
  double* dot_scratch = nullptr;   // device address of this device's static dot-product scratch
  bool persistent = false;  // force kernel schedule (fppg_set_schedule)
  int* d_tickets = nullptr; // [8] ticket counters of the persistent schedule
  int resident[2][3] = {};  // resident force blocks per CU by (k - 1, block 128/256/512); 0 = not queried
  int num_cu = 0;
};

struct fppg_geom : fppg::Geom {};

namespace fppg {

// Record an error message in the context and return the status.
fppg_status fail(fppg_ctx* ctx, fppg_status s, const std::string& msg);
fppg_status hip_fail(fppg_ctx* ctx, hipError_t e, const char* what);

#define FPPG_HIP(ctx, call)                                   \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return fppg::hip_fail(ctx, e_, #call); \
  } while (0)

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Event pair around one phase of a per-iteration call (no-op unless profiling).
struct PhaseTimer {
  PhaseProf* p = nullptr;
  hipStream_t s;
  PhaseTimer(fppg_ctx* ctx, int phase, hipStream_t stream) : s(stream) {
    if (ctx && ((ctx->profiling >> phase) & 1u) && ctx->prof[phase].used < kProfSlots) {
      p = &ctx->prof[phase];
      (void)hipEventRecord(p->start[p->used], s);   // a failed record is reported by fppg_profile_read
    }
  }
  ~PhaseTimer() {
    if (p) {
      (void)hipEventRecord(p->stop[p->used], s);
      p->used++;
    }
  }
};

constexpr int kHeavyGroupMax = 8;   // projection: volume-pass blocks served by one block of k_project_heavy (at most)

// Workspace layout (byte offsets from the workspace base, 256-aligned).
struct WsLayout {
  // build_cells
  size_t key, rank, tmp_id, tmp_src, tmp_key, count, blocksum, big, build_end;
  // relax_step
  size_t accel, step_end;
  // moving_list (block counts, their offsets, scan partials)
  size_t list_cnt, list_offs, list_bsum, list_end;
  // project (per volume-pass block: queue length; per k_project_heavy block:
  // revert counts; the queue of surface, feature and near-facet volume particles)
  size_t proj_count, proj_part, proj_queue, proj_hard, proj_end;
  // relax_energy / vec_dot partial sums
  size_t reduce_end;
  size_t total;
};
WsLayout ws_layout(const Geom* g, int64_t n);

// Facet registration on uniform grids (register.hip).
struct RegGrid {
  double o[3];         // origin of cell (0, 0, 0)
  double cell, inv;    // cell edge and its reciprocal
  double pad;          // boxes widened by pad on every side
  int dims[3];
  int unused;
  int64_t key_begin;   // dense keys: index of this grid's first cell
};
struct RegItem {       // a triangle to register: its vertices, facet and grid
  double a[3], b[3], c[3];
  int facet, grid;
};
struct RegPairs {      // unique (key, facet) pairs sorted by (key, facet), device
  uint64_t* keys = nullptr;
  uint32_t* facets = nullptr;
  int64_t n = 0;
  int levels = 0;      // subdivision levels
};
// Subdivide and register `items` (facets, by grid); key = Morton code of the
// cell (morton) or key_begin + its dense index. key_bits / facet_bits bound
// the keys and facet ids (the radix passes). Synchronous on s.
fppg_status register_facets(fppg_ctx* ctx, const std::vector<RegItem>& items, const std::vector<RegGrid>& grids,
                            bool morton, int key_bits, int facet_bits, RegPairs* out, hipStream_t s);
// Dense CSR of registered pairs with dense keys < n_cells: start [n_cells + 1],
// facets [pairs.n] (int32), non-empty flags [n_cells] (kCellHasFacet); device
// arrays the caller frees. Synchronous on s.
fppg_status registration_csr(fppg_ctx* ctx, const RegPairs& pairs, int64_t n_cells, int** start, int** tri,
                             uint8_t** flag, hipStream_t s);

// Exclusive prefix sum of in[0..n) into out[0..n), out[n] = the total
// (cells.hip). blocksum: scan_blocksum_len(n) ints of device scratch.
fppg_status exclusive_scan(fppg_ctx* ctx, const int* in, int64_t n, int* out, int* blocksum, hipStream_t s);
int64_t scan_blocksum_len(int64_t n);

// Deterministic FP64 reductions (linalg.hip): per-block partial sums in a
// fixed order, then one block sums the partials in index order.
constexpr int kDotPartials = 2048;   // partial sums of fppg_vec_dot (doubles of workspace)
fppg_status sum_partials(fppg_ctx* ctx, const double* partial, int nb, double* out, hipStream_t s);
// Resolve the device address of the static dot-product scratch array on the
// current device into ctx->dot_scratch (linalg.hip; called by fppg_create).
fppg_status init_dot_scratch(fppg_ctx* ctx);

// Device helpers ---------------------------------------------------------------------------

// FP64 sum over a block of 256 threads in a fixed tree order (thread 0 gets it).
__device__ __forceinline__ double block_sum256(double v) {
  __shared__ double s_part[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
  __syncthreads();
  return t;
}

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b to XCD b % 8),
// each XCD with its own L2. Map workgroup b to chunk c so that every XCD gets
// one contiguous range of chunks: neighbouring receivers then share the halo
// rows they read in the same L2. A bijection on [0, nb) for any nb.
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_chunk(int b, int nb) {
  const int q = nb / kNumXcd, r = nb % kNumXcd;
  const int x = b % kNumXcd, k = b / kNumXcd;
  return x * q + min(x, r) + k;
}

// Runs of kXcdRun consecutive chunks dealt to the XCDs in turn: run m goes to
// XCD m % 8, so the k-th workgroup of XCD x takes chunk (8 (k / R) + x) R +
// k % R. Each XCD then walks many shorter contiguous stretches spread over
// the whole domain: neighbouring receivers still share an L2, and the XCDs
// get equal shares of every region. Workgroups past the last whole round of
// 8 runs keep their own index (a bijection on [0, nb) for any nb).
constexpr int kXcdRun = 16;
__device__ __forceinline__ int xcd_run_chunk(int b, int nb) {
  const int full = nb / (kNumXcd * kXcdRun) * (kNumXcd * kXcdRun);
  if (b >= full) return b;
  const int x = b % kNumXcd, k = b / kNumXcd;
  return ((k / kXcdRun) * kNumXcd + x) * kXcdRun + k % kXcdRun;
}

// Chunk of workgroup b of nb by the launch's XCD mapping: 0 round-robin (the
// hardware's deal), 1 one contiguous range per XCD, 2 runs of kXcdRun chunks.
__device__ __forceinline__ int launch_chunk(int mode, int b, int nb) {
  return mode == 1 ? xcd_chunk(b, nb) : (mode == 2 ? xcd_run_chunk(b, nb) : b);
}

// Key of cell (0, y, z) of a geometry: the y range is cut into slabs of
// `slab` rows (the last one may be narrower); keys run over the slabs, within
// a slab over z, then over the slab's rows, then x. Cell (x, y, z) has key
// row_key(G, y, z) + x. floor((y + 1/2) / slab) in binary32 is exact here:
// the quotient stays at least 1/(2 slab) away from an integer and the grid
// has far fewer than 2^20 rows.
__device__ __forceinline__ int row_key(const GeomDev& G, int y, int z) {
  const int S = G.slab;
  const int s = int((float(y) + 0.5f) * G.inv_slab);
  const int y0 = s * S;
  const int w = min(S, G.dims[1] - y0);
  return int(G.cell_begin) + y0 * G.dims[0] * G.dims[2] + (z * w + (y - y0)) * G.dims[0];
}

__device__ __forceinline__ int tag_of(float w) { return __float_as_int(w) & 7; }
__device__ __forceinline__ int geom_of(float w) { return (__float_as_int(w) >> 8) & 0xFFFF; }
__device__ __forceinline__ int rank_of(int tag) { return tag < 3 ? tag : 3; }
__device__ __forceinline__ bool is_moving(int tag, uint32_t move_mask) {
  return tag >= 1 && tag <= 3 && ((move_mask >> tag) & 1u);
}

// x <- P x for particle i (the tangent spaces of Eq. 24-25): surface
// I - n n^T with n the binary32 normal of facet owner[i], feature t t^T with
// t the FP64 tangent of segment feat_seg[owner[i]], volume I, a particle
// that does not move 0. An out-of-range owner or segment gives 0 and sets
// FPPG_S_BAD_INDEX.
__device__ __forceinline__ float4 tangent_apply(float4 x, int tag, int i, uint32_t move_mask,
                                                const int* __restrict__ owner, const int* __restrict__ feat_seg,
                                                int n_feat, int n_tri, int n_seg, const float4* __restrict__ n32,
                                                const SegDev* __restrict__ segs, uint32_t* status) {
  const float4 zero = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (!is_moving(tag, move_mask)) return zero;
  if (tag == FPPG_TAG_SURFACE) {
    const int o = owner[i];
    if (o < 0 || o >= n_tri) {
      atomicOr(status, FPPG_S_BAD_INDEX);
      return zero;
    }
    const float4 nn = n32[o];
    const float s = x.x * nn.x + x.y * nn.y + x.z * nn.z;
    x.x -= s * nn.x;
    x.y -= s * nn.y;
    x.z -= s * nn.z;
  } else if (tag == FPPG_TAG_FEATURE) {
    const int o = owner[i];
    const int sg = (o >= 0 && o < n_feat) ? feat_seg[o] : -1;
    if (sg < 0 || sg >= n_seg) {
      atomicOr(status, FPPG_S_BAD_INDEX);
      return zero;
    }
    const SegDev S = segs[sg];
    const double s = double(x.x) * S.t[0] + double(x.y) * S.t[1] + double(x.z) * S.t[2];
    x.x = float(s * S.t[0]);
    x.y = float(s * S.t[1]);
    x.z = float(s * S.t[2]);
  }
  return x;
}

// Particle handled by launch slot r: r itself, or list[r] when a receiver
// list is given (slots past n_list get n: idle).
__device__ __forceinline__ int listed(int r, int n, const int* __restrict__ list, int n_list) {
  if (!list) return r;
  return r < n_list ? list[r] : n;
}

}  // namespace fppg

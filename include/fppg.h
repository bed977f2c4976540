/*
 * fppg.h - C ABI of the MI355X (gfx950) particle-relaxation library.
 *
 * The library implements the per-iteration hot path of the physics-based
 * particle relaxation of the feature-preserving particle generation method
 * (FPPG, arXiv 2501.03056, section 3.3, Algorithm 1):
 *
 *   fppg_build_cells  rebuild the cell-linked list of the particles by a
 *                     counting sort on the cell key ("updating data
 *                     structures", Algorithm 1; the paper's sorted compact
 *                     list of section 3.1.3 is the analogue)
 *   fppg_relax_step   Wendland C2 kernel-gradient repulsion (Eq. 15-17), the
 *                     bounded time step, velocity reset and displacement
 *                     (Eq. 22-23) restricted to the geometry (Eq. 24-25)
 *   fppg_project      surface reprojection onto the nearest facet with revert
 *                     (section 3.3.3), feature-line motion, volume particles
 *                     kept inside the closed mesh
 *   fppg_relax_hvp    Jacobian-vector product of the force field (Hessian-
 *                     vector product of the pair energy), for Newton-Krylov
 *                     relaxation and for differentiation
 *
 * Conventions
 *  - Every function returns an fppg_status (0 = OK, < 0 = error) and never
 *    throws. On error, fppg_last_error(ctx) describes it.
 *  - Array arguments of the per-iteration calls (build_cells, relax_step,
 *    project, relax_hvp, debug_neighbors) are DEVICE pointers owned by the
 *    caller; the library never frees them and allocates nothing in these
 *    calls: scratch memory is the caller's workspace `ws` of at least
 *    fppg_workspace_size bytes (256-byte aligned).
 *  - These calls only enqueue work on `stream` (a hipStream_t passed as
 *    void*; NULL = the default stream) and do not synchronise. Conditions
 *    found on the device (non-finite values) set bits of a device status word
 *    read by fppg_read_status, which synchronises the stream.
 *  - Positions are float4 arrays passed as float*, 16-byte aligned: x, y, z
 *    in binary32 and w holding int32 bits  tag | (level << 3) | (geometry << 8)
 *    where tag is the particle class 0 singular point, 1 feature-line
 *    particle, 2 surface particle, 3 volume particle, 4 fixed volume particle
 *    (innermost layer), level (0..3) the resolution level of a particle of a
 *    multi-resolution geometry (fppg_geom_desc.max_level; 0 otherwise), and
 *    geometry is the index of the particle's geometry in the batch.
 *  - Facets and feature segments are numbered globally over a batch: the
 *    facets of geometry g follow those of geometries 0..g-1 (same for
 *    segments). `owner` holds the global facet of a surface particle, the
 *    feature slot (index into feat_seg / feat_u) of a feature particle, the
 *    global mesh vertex of a singular particle (read only by the mesh-gradient
 *    calls), and -1 otherwise.
 *  - A context is used by one host thread at a time.
 */
#ifndef FPPG_H
#define FPPG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fppg_status;
#define FPPG_OK             0
#define FPPG_E_ARG         -1  /* invalid argument: null/misaligned pointer, bad size or descriptor */
#define FPPG_E_HIP         -2  /* a HIP runtime call failed */
#define FPPG_E_WORKSPACE   -3  /* workspace too small */
#define FPPG_E_CAPACITY    -4  /* a fixed-size limit of the library was exceeded */
#define FPPG_E_UNSUPPORTED -5  /* configuration not supported (e.g. stencil half-width) */
#define FPPG_E_NODEVICE    -6  /* no usable gfx950 device */

/* particle classes (low 3 bits of pos.w) */
#define FPPG_TAG_SINGULAR 0
#define FPPG_TAG_FEATURE  1
#define FPPG_TAG_SURFACE  2
#define FPPG_TAG_VOLUME   3
#define FPPG_TAG_FIXED    4

/* flags of fppg_relax_step */
#define FPPG_F_COUNT_PAIRS 1u  /* accel.w = number of sources of the receiver (as float) */
#define FPPG_F_FORCES_ONLY 2u  /* accel and amax only: no displacement (disp may be NULL; accel must not) */

/* device status bits (fppg_read_status) */
#define FPPG_S_NONFINITE_ACCEL 1u  /* a receiver's acceleration was not finite (it did not move) */
#define FPPG_S_NONFINITE_POS   2u  /* a moved position was not finite (the move was reverted) */
#define FPPG_S_BAD_INDEX       4u  /* a geometry, owner or feature index was out of range (particle held) */
#define FPPG_S_FIXED_RANGE     8u  /* a vertex-gradient contribution or running sum left the 64-bit
                                      fixed-point range |v| < 2^23 (step/fixed adjoint): that gradient is invalid */

/* counters accumulated by fppg_project (int64 each) */
#define FPPG_C_REVERT_SURFACE 0
#define FPPG_C_REVERT_FEATURE 1
#define FPPG_C_REVERT_VOLUME  2
#define FPPG_NCOUNTERS        8  /* slots 3..7 reserved */

typedef struct fppg_ctx fppg_ctx;
typedef struct fppg_geom fppg_geom;

/*
 * One geometry of a batch (host memory; fppg_geom_create copies it).
 *
 * Particle grid (cell list of section 3.1.1's uniform background grid,
 * rebuilt every iteration): the cells of the grid (origin, inv_cell, dims)
 * split in two along x, nx = 2 dims[0] of them per row. Cell (cx, cy, cz) of
 * a position p is
 *   cx = clamp(floor(fl32(fl32(p.x - origin[0]) * fl32(2 inv_cell))), 0, nx - 1)
 *   cy, cz = clamp(floor(fl32(fl32(p - origin) * inv_cell)), 0, dims - 1)
 * (binary32, one rounding per operation; 2 inv_cell is exact) and its key is
 *   cell_begin(g) + s S nx dims[2] + (cz w + cy - s S) nx + cx,
 *   s = cy div S,  w = min(S, dims[1] - s S),  S = slab
 * with cell_begin(g) the total cell count of geometries 0..g-1: the y range
 * is cut into slabs of S rows (slab <= 0 or > dims[1]: one slab, the plain
 * (cz dims[1] + cy) nx + cx), each slab numbered z-major with x fastest.
 * Any S gives the same cell list; narrow slabs keep the rows a stencil reads
 * close in memory; the half-width cells along x let a stencil row end within
 * half a cell of the support sphere. The cell edge
 * 1/inv_cell must be at least (2h/k)(1 + 2^-9) so that the (2k+1)^3 cell
 * stencil holds every pair with q < 2; k is 1 or 2 and equal across a batch.
 * fppg_geom_info reports the total cell count (2 dims[0] dims[1] dims[2]
 * summed over the geometries).
 *
 * Particles of geometry g occupy the index range [part_begin, part_end) of
 * the particle arrays, which the cell sort preserves.
 *
 * Mesh: closed triangle surface, facets counter-clockwise seen from outside
 * (outward normal (B-A)x(C-A)), FP64 vertices. Feature lines: line l has the
 * segments line_seg_begin[l] .. line_seg_begin[l+1]-1 (local numbering), each
 * segment s runs from seg_p[6s..6s+2] to seg_p[6s+3..6s+5], consecutive
 * segments of a line are joined, line_closed[l] != 0 for a loop.
 *
 * proj_radius R: a surface projection is accepted only if the particle is
 * within R of the facet plane (section 3.3.3). The facet search grid uses
 * cells of edge R(1 + 2^-6): R = dx makes them the background grid of the
 * generation, whose 27 cells around a particle the reprojection searches.
 * A particle moves at most h/16 per step, so any R of a few h/16 or more
 * accepts the same projections; a smaller R gives fewer facets per cell and
 * more cells (memory: 5 bytes per search cell).
 */
typedef struct {
  float   origin[3];
  float   inv_cell;
  int32_t dims[3];
  int32_t k;
  float   h;                 /* smoothing length; support radius 2h */
  float   proj_radius;       /* R */
  int64_t part_begin, part_end;
  const double*  vert;  int32_t n_vert;   /* [n_vert * 3] */
  const int32_t* tri;   int32_t n_tri;    /* [n_tri * 3] */
  const int32_t* line_seg_begin; int32_t n_line;  /* [n_line + 1], may be NULL if n_line = 0 */
  const double*  seg_p;                   /* [n_seg * 6], n_seg = line_seg_begin[n_line] */
  const uint8_t* line_closed;             /* [n_line] */
  const int32_t* seg_vert;                /* [n_seg * 2] mesh vertex (local index) at each segment
                                             end, -1 if none; may be NULL (mesh gradients only) */
  int32_t slab;                           /* cell rows per slab of the key (see above) */
  /* Boolean assembly (section 3.2.3): 0 = the mesh is the solid; otherwise the
     mesh is the facets of n_part closed convex parts, part k owning the facets
     part_tri_begin[k] .. part_tri_begin[k+1]-1 (part_tri_begin[0] = 0,
     part_tri_begin[n_part] = n_tri), and the solid is
       FPPG_CSG_UNION       the union of the parts
       FPPG_CSG_DIFFERENCE  part 0 minus the union of the others.
     Every part must be convex (each vertex of a part on the inner side of every
     plane of its facets; FPPG_E_ARG otherwise). See fppg_project for how the
     relaxation treats an assembly. */
  int32_t csg_op;
  int32_t n_part;
  const int32_t* part_tri_begin;          /* [n_part + 1], 1 <= n_part <= 8; may be NULL if csg_op = 0 */
  /* Multi-resolution (the paper's future work; the pair length of Eq. 6):
     0 = one smoothing length h. 1..3 = a particle of level l (pos.w bits 3-4,
     l <= max_level) has h_i = h 2^-l; a pair uses h_ij = (h_i + h_j) / 2:
     neighbours iff |r|^2 < fl32(fl32(h_i + h_j)^2), force term
     K(h_ij) (1 - r / 2h_ij)^3 r_ij, and the time step moves each particle at
     most h_i / 16 (amax is the largest |a_i| 2^l_i). The particle cells are
     sized by h, the coarsest length. The Jacobian, energy, density and
     neighbour-export calls refuse such a geometry (FPPG_E_UNSUPPORTED). */
  int32_t max_level;
} fppg_geom_desc;

#define FPPG_CSG_NONE       0
#define FPPG_CSG_UNION      1
#define FPPG_CSG_DIFFERENCE 2

/* ---- context ---------------------------------------------------------------------------- */

/* Select HIP device `device` (must be gfx950), allocate the device status word. */
fppg_status fppg_create(int32_t device, fppg_ctx** out);
void        fppg_destroy(fppg_ctx* ctx);
const char* fppg_status_str(fppg_status s);
const char* fppg_last_error(const fppg_ctx* ctx);   /* never NULL */

/* Hash of the sources and compiler flags the library was built from (32 hex
 * digits, a static string; "unknown" if the build did not define it). A
 * loader compares it with the sources it expects, to refuse a stale build. */
const char* fppg_source_hash(void);

/* Synchronise `stream`, return the device status bits (FPPG_S_*) and clear them. */
fppg_status fppg_read_status(fppg_ctx* ctx, void* stream, uint32_t* flags);

/*
 * Kernel timing with HIP events recorded on the launch stream. phases: bit p
 * set times phase p (FPPG_PROFILE_ALL: every phase; 0: off). A nonzero mask
 * creates the events (allocation happens here, not in the hot calls) and
 * resets the accumulators; while enabled, every per-iteration call records an
 * event pair around each selected phase (each pair adds a little time to the
 * stream). fppg_profile_read synchronises on the recorded events and returns,
 * per phase, the summed milliseconds and the number of launches:
 *   0 build_cells (all its kernels)  1 force + amax kernel
 *   2 displacement kernel            3 project (all its kernels)
 *   4 relax_hvp kernel
 * Phase times are accumulated when read; at most 4096 launches per phase are
 * kept between reads (further launches are not timed: count stops growing).
 */
#define FPPG_NPHASES 5
#define FPPG_PROFILE_ALL 0x1fu
fppg_status fppg_profile(fppg_ctx* ctx, uint32_t phases);
fppg_status fppg_profile_read(fppg_ctx* ctx, double* ms /*[FPPG_NPHASES]*/, int64_t* launches /*[FPPG_NPHASES]*/);

/*
 * Launch shape of the force kernel of fppg_relax_step (and of the Jacobian
 * products), chosen by the autotuner: force_block threads per block (128, 256
 * or 512) and the mapping of blocks to the 8 XCDs (each with its own L2):
 * xcd_remap 0 keeps the hardware's round-robin deal, 1 gives each XCD one
 * contiguous range of receivers, 2 deals runs of 16 consecutive chunks of
 * force_block receivers to the XCDs in turn (each XCD walks many short
 * contiguous stretches spread over the domain; chunks past the last whole
 * round of 8 runs keep the round-robin deal). No result depends on the choice
 * (per-receiver sums; amax is a maximum). Defaults 256 and 1.
 * Applies to later calls on the context (and to graphs captured after it).
 * Errors: FPPG_E_ARG for other values.
 */
fppg_status fppg_set_launch(fppg_ctx* ctx, int32_t force_block, int32_t xcd_remap);

/*
 * Schedule of the force kernel of fppg_relax_step, chosen by the autotuner:
 * persistent = 0 launches one block per chunk of force_block receivers;
 * persistent = 1 launches as many blocks as fit on the device at once, each
 * taking chunks by tickets: the blocks of XCD x (workgroup b runs on XCD b %
 * 8) first take the contiguous range of chunks that xcd_remap 1 would give x,
 * then the other XCDs' leftovers. The ticket counters are cleared by a small
 * kernel before every launch (stream-ordered; graph-capturable) and live in
 * the context, so calls on one context must not overlap. No result depends
 * on the schedule (each chunk is computed the same way). Errors: FPPG_E_ARG.
 */
fppg_status fppg_set_schedule(fppg_ctx* ctx, int32_t persistent);

/* ---- geometry ----------------------------------------------------------------------------- */

/*
 * Build the device-resident geometry of a batch of n_geom geometries: facet
 * frames (FP64), the facet search grid (facets registered conservatively in
 * every cell they touch, section 3.1.1-3.1.2; built on the host), feature
 * segments, and the per-geometry particle-grid descriptors. Synchronous;
 * allocates device memory owned by the returned object.
 * The per-iteration calls take n = the descriptors' particle count (the
 * active count, until fppg_tier_partition narrows it).
 * Errors: FPPG_E_ARG for inconsistent descriptors (particle ranges must tile
 * [0, n) in order, indices in range), FPPG_E_UNSUPPORTED for k not in {1, 2}
 * or differing across the batch, FPPG_E_CAPACITY beyond 2^31 cells/entries.
 */
fppg_status fppg_geom_create(fppg_ctx* ctx, const fppg_geom_desc* descs, int32_t n_geom,
                             fppg_geom** out);
void        fppg_geom_destroy(fppg_geom* geom);

/* Sizes of a built geometry: total particle cells (cell_start has ncell + 2
 * entries), facets, segments, facet-search cells and their facet entries. */
fppg_status fppg_geom_info(const fppg_geom* geom, int64_t* ncell, int64_t* n_tri, int64_t* n_seg,
                           int64_t* search_cells, int64_t* search_entries);

/* Copy the facet search grid (registered on the device at fppg_geom_create:
 * facets subdivided and tested against the cells as fppg_sparse_grid_create
 * does, with a pad of 1e-6 cell) into caller device buffers: start
 * [search_cells + 1] (facet-list offsets of every search cell, the
 * geometries' grids one after another), tri [search_entries] (global facet
 * ids, ascending within a cell), flag [search_cells] (1: the cell holds a
 * facet). A null destination is skipped. Stream-ordered. */
fppg_status fppg_geom_search_grid(fppg_ctx* ctx, const fppg_geom* geom, int32_t* start, int32_t* tri, uint8_t* flag,
                                  void* stream);

/* Workspace bytes needed by the per-iteration calls for n particles. */
fppg_status fppg_workspace_size(const fppg_geom* geom, int64_t n, size_t* bytes);

/*
 * Tier partition (the tiers of Algorithm 1: feature lines, then surfaces,
 * then the volume, section 3.3). A particle takes as sources only the classes
 * of rank at most its own (section 2.2), so in a tier whose highest moving
 * class has rank R the particles of rank > R are neither receivers nor
 * sources: a volume particle plays no part while the feature lines or the
 * surfaces relax. The call stably partitions the n = all particles of the
 * geometry (pos_in, id_in, owner_in, in their current order) into out: first
 * the *n_active particles of rank <= R, then the rest, each part in input
 * order. The rest [*n_active, n) is also copied back into the input arrays,
 * so both buffers of a double-buffered state hold it.
 * From then on the geometry's active count is *n_active: every call that
 * takes the geometry (build_cells, relax_step, project, relax_hvp, ...)
 * must be passed n = *n_active and touches only that prefix; the other
 * particles stay where they are. The forces, displacements and projections
 * of the movers are bitwise those of the calls on all n particles (the
 * skipped particles contribute exact zeros there). A move_mask with the volume
 * class (R = 3), or with no moving class, reaches every particle: out is a
 * copy of the input and the active count is n again.
 * R is the highest of rank 1 (feature, bit FPPG_TAG_FEATURE), 2 (surface)
 * and 3 (volume) set in move_mask. ws: at least fppg_workspace_size(n) bytes.
 * Synchronous (it reads the count back). Errors: FPPG_E_ARG for null or
 * misaligned arrays, aliasing outputs or n other than the descriptors'
 * particle count; FPPG_E_WORKSPACE.
 */
fppg_status fppg_tier_partition(fppg_ctx* ctx, fppg_geom* geom, int64_t n, float* pos_in, int32_t* id_in,
                                int32_t* owner_in, float* pos_out, int32_t* id_out, int32_t* owner_out,
                                uint32_t move_mask, int64_t* n_active, void* ws, size_t ws_bytes, void* stream);

/* ---- per-iteration calls (device pointers, stream-ordered, no allocation) ---------------- */

/*
 * Counting sort of the particles by cell key, then by id inside a cell.
 * in:  pos_in [n*4], id_in [n], owner_in [n] (ids unique per particle)
 * out: pos_out, id_out, owner_out (must not alias the inputs), the same
 *      particles in (key, id) order; cell_start [ncell + 2]: first sorted
 *      index of every cell, then cell_start[ncell] = first index of the
 *      quarantine range and cell_start[ncell + 1] = n. Particles with a
 *      non-finite coordinate get the key ncell (after every geometry, where no
 *      stencil reaches: they are nobody's neighbour) and FPPG_S_NONFINITE_POS.
 * The order is deterministic (independent of atomic ordering). Work per
 * cell of m particles: O(m^2) lane steps up to m = 64, a sort of
 * O(m log m) above that (a clump of particles, or many non-finite ones).
 */
fppg_status fppg_build_cells(fppg_ctx* ctx, const fppg_geom* geom, int64_t n,
                             const float* pos_in, const int32_t* id_in, const int32_t* owner_in,
                             float* pos_out, int32_t* id_out, int32_t* owner_out,
                             int32_t* cell_start, void* ws, size_t ws_bytes, void* stream);

/*
 * Forces, time step and displacement of one iteration (Eq. 15-17, 22-25).
 * pos [n*4] and cell_start come from fppg_build_cells. A particle moves iff
 * its tag is 1, 2 or 3 and bit `tag` of move_mask is set. For every moving
 * receiver i:
 *   a_i = K sum_{j in src(i)} (1 - |r_ij|/2h)^3 r_ij,  r_ij = x_i - x_j,
 *   K = 5 alpha / h^2, alpha = 21/(16 pi h^3) (Eq. 17's 3-D factor written
 *   with the coefficient that normalises the kernel), prefactor of Eq. 15 = 1,
 * where src(i) are the particles j != i of the geometry with
 *   fl32(fl32(fl32(dx^2) + fl32(dy^2)) + fl32(dz^2)) < fl32(2h)^2 (binary32)
 * and rank(tag_j) <= rank(tag_i), ranks 0,1,2,3,3 for tags 0..4
 * (section 2.2: each class is bounded by the classes of lower rank).
 * amax[g] = max |a_i| over moving i of geometry g; dt^2 = (h/16)/amax[g]
 * (time-step reading: dt = 0.25 sqrt(h/amax)); v reset to 0 (Eq. 22), so the
 * displacement is dr_i = dt^2 a_i, then restricted (Eq. 24-25):
 *   surface: dr - (dr . n) n, n the normal of facet owner[i]
 *   feature: du = dr . t in FP64, t the unit tangent of segment
 *            feat_seg[owner[i]]; the double du is stored in the bytes of
 *            disp[4i..4i+1] and disp[4i+2..4i+3] = 0.
 *   volume:  dr;  non-moving: 0.
 * Outputs: accel [n*4] (may be NULL: the workspace holds it; w = 0, or the
 * source count with FPPG_F_COUNT_PAIRS), amax [n_geom] (float), disp [n*4]
 * (not written, and may be NULL, with FPPG_F_FORCES_ONLY, which then needs
 * accel).
 * Non-finite accelerations are excluded from amax and give a zero
 * displacement (FPPG_S_NONFINITE_ACCEL); an out-of-range owner or feature
 * segment gives a zero displacement (FPPG_S_BAD_INDEX).
 * Receivers: all n particles (list = NULL), or only the n_list particles
 * whose sorted indices list [n_list] (device, distinct, in [0, n)) holds, e.g.
 * the moving particles from fppg_moving_list: a tier in which few particles
 * move then launches only their lanes. Rows of accel and disp outside the
 * list are not written.
 */
fppg_status fppg_relax_step(fppg_ctx* ctx, const fppg_geom* geom, int64_t n,
                            const float* pos, const int32_t* owner, const int32_t* cell_start,
                            const int32_t* feat_seg, int32_t n_feat, uint32_t move_mask, uint32_t flags,
                            float* accel, float* amax, float* disp, const int32_t* list, int32_t n_list,
                            void* ws, size_t ws_bytes, void* stream);

/*
 * Apply the displacement and project back onto the geometry (section 3.3.3).
 * One lane per particle in two kernels: a streaming pass applies the volume
 * rule and queues the surface and feature particles in the workspace, a
 * second pass projects the queued particles (and a third searches the few
 * surface particles whose own search cell accepts no facet).
 *  surface: y = x + dr (FP64); among the facets registered in the 27 search
 *           cells around y, the plane foot p = y - d n with all barycentric
 *           coordinates >= 0 and |d| <= R and the smallest |d| (ties: lowest
 *           facet) wins: pos = fl32(p), owner = that facet; none: pos stays x
 *           (revert). The own cell is searched first and a neighbouring cell
 *           only if it comes within the best |d| found (same result); a
 *           particle whose own cell accepts no facet has its 27 cells searched
 *           side by side by one wavefront in a further kernel (same result).
 *  feature: u' = u + du walked along the polyline of segment feat_seg[slot],
 *           carrying into neighbouring segments; leaving an open line
 *           reverts, a loop wraps; pos = fl32(p0 + u' t), feat_seg/feat_u
 *           updated in place (slot = owner[i]).
 *  volume:  y = fl32(x + dr); the move is reverted iff the segment [x, y]
 *           meets a facet (tested against the facets of the search cells the
 *           segment's bounding box touches). With x inside, this equals "the
 *           signed distance of y is >= 0" for meshes thicker than the step.
 *  Boolean assembly (fppg_geom_desc.csg_op): a surface foot point p on a
 *           facet of part k is accepted only on the assembly's boundary (FP64
 *           plane tests of the convex parts; a part's interior is where every
 *           plane test is < 0): union, p in no other part's interior;
 *           difference, for k = 0 p in no cut part's interior, for a cut part
 *           p in the closure of part 0 and in no other cut part's interior.
 *           A volume move is reverted iff its segment meets a facet at a point
 *           of the assembly's boundary (the same test on the crossing point):
 *           crossing a part's face inside the assembly is no revert.
 * pos [n*4] in: positions x, out: new positions; owner [n] in/out;
 * disp [n*4] from fppg_relax_step; feat_seg/feat_u [n_feat] in/out (may be
 * NULL if n_feat = 0); counters [FPPG_NCOUNTERS] int64 on the device,
 * incremented by the number of reverts per class (FPPG_C_*). list / n_list
 * as in fppg_relax_step (NULL: all particles). ws: device workspace, 256-byte
 * aligned, at least fppg_workspace_size bytes (it queues the surface and
 * feature particles for a second kernel); its contents are scratch.
 */
fppg_status fppg_project(fppg_ctx* ctx, const fppg_geom* geom, int64_t n,
                         float* pos, int32_t* owner, const float* disp,
                         int32_t* feat_seg, double* feat_u, int32_t n_feat, uint32_t move_mask,
                         int64_t* counters, const int32_t* list, int32_t n_list, void* ws, size_t ws_bytes,
                         void* stream);

/*
 * Jacobian-vector product of the force field of fppg_relax_step with respect
 * to the positions, at fixed neighbour sets (same traversal as the forces):
 *   transpose = 0:  Jv_i = sum_{j in src(i)} M(r_ij) (v_i - v_j)  for moving i, else 0
 *   transpose = 1:  Jv_k = [sum_{j in src(k)} M(r_kj)] v_k - sum_{i moving, k in src(i)} M(r_ik) v_i
 *                   (first term only for moving k)
 * with M(r) = K [ t^3 I - (3/2h) t^2 r r^T / |r| ], t = 1 - |r|/2h.
 * For one moving class with fixed other sources J = -Hess(E) of the pair
 * energy E and both products agree. v, Jv: [n*4] float (w ignored / 0).
 */
fppg_status fppg_relax_hvp(fppg_ctx* ctx, const fppg_geom* geom, int64_t n,
                           const float* pos, const int32_t* cell_start, uint32_t move_mask,
                           int32_t transpose, const float* v, float* Jv, void* stream);

/*
 * The Newton-Krylov operator in one sweep: out = scale P (J v), with J v as
 * fppg_relax_hvp(transpose = 0) computes it and P the tangent projection of
 * fppg_tangent_project applied to each receiver's row (owner, feat_seg as
 * there). For v in the tangent space (P v = v) and scale = -1 this is
 * -P J P v, the symmetric operator MINRES iterates with. out must not alias v.
 */
fppg_status fppg_relax_hvp_projected(fppg_ctx* ctx, const fppg_geom* geom, int64_t n,
                                     const float* pos, const int32_t* cell_start, const int32_t* owner,
                                     const int32_t* feat_seg, int32_t n_feat, uint32_t move_mask,
                                     const float* v, float scale, float* out, void* stream);

/*
 * Pair energy whose negative gradient is the force field of fppg_relax_step
 * for one moving class with fixed other sources (the line-search objective
 * of Newton-Krylov relaxation; not in the paper):
 *   E = sum_{i moving} sum_{j in src(i)} c_ij W(r_ij),  c_ij = 1/2 if j moves, else 1
 * with W the Wendland C2 kernel of Eq. 16 (alpha = 21/(16 pi h^3)), evaluated
 * in FP64 from the binary32 positions over the same neighbour sets. out: one
 * double on the device. Deterministic summation order. ws: at least
 * fppg_workspace_size bytes.
 */
fppg_status fppg_relax_energy(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                              const int32_t* cell_start, uint32_t move_mask, double* out,
                              void* ws, size_t ws_bytes, void* stream);

/*
 * Vector operations on particle fields (float4 rows, x/y/z used, w ignored),
 * for Krylov solvers:
 *   fppg_vec_dot    out[0] = sum_i a_i . b_i in FP64, fixed summation order
 *                   (device double; ws >= 2048 doubles, 256-byte aligned)
 *   fppg_vec_axpby  y <- alpha x + beta y; with beta = 0 the old y is not read
 *                   and with alpha = 0 x is not read (NaN there does not propagate)
 * Neither touches w.
 */
fppg_status fppg_vec_dot(fppg_ctx* ctx, int64_t n, const float* a, const float* b, double* out,
                         void* ws, size_t ws_bytes, void* stream);
fppg_status fppg_vec_axpby(fppg_ctx* ctx, int64_t n, float alpha, const float* x, float beta, float* y,
                           void* stream);

/*
 * fppg_vec_dot without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight solver loops, harnesses that
 * forbid hipMalloc): out[0] = sum_i a_i . b_i in FP64, bitwise equal to
 * fppg_vec_dot's result (same kernels, same block partition). The per-block
 * partial sums live in a static device array of the library (2048 doubles =
 * 16 KiB per device, held until the process ends; its device address is
 * resolved once by fppg_create). The call allocates nothing. Every call on one
 * device shares that array and overwrites it: calls that overlap on one GPU
 * (concurrent streams, several host threads) race and must be serialised by
 * the caller. n: 0 <= n < 2^31 (any n fits the fixed scratch: the rows are
 * split over at most 2048 blocks). Errors: FPPG_E_ARG for null or misaligned
 * a/b/out or n out of range.
 */
fppg_status fppg_vec_dot_noalloc(fppg_ctx* ctx, int64_t n, const float* a, const float* b, double* out,
                                 void* stream);
/* out[0] (device float) = max_i |a_i| (Euclidean norm of the xyz of row i);
 * a NaN row counts as +inf. */
fppg_status fppg_vec_maxnorm(fppg_ctx* ctx, int64_t n, const float* a, float* out, void* stream);
/* v_i <- v_i * min(1, cap / |v_i|) row by row (cap > 0): caps every particle's move. */
fppg_status fppg_vec_clamp(fppg_ctx* ctx, int64_t n, float* v, float cap, void* stream);

/*
 * out <- a x + b y + c z row by row, then acc <- acc + phi out if acc is not
 * NULL (a term with a zero coefficient is not read and may be NULL). out and
 * acc must not alias the inputs or each other. The direction and iterate
 * update of a MINRES iteration in one pass.
 */
fppg_status fppg_vec_combine3(fppg_ctx* ctx, int64_t n, float a, const float* x, float b, const float* y,
                              float c, const float* z, float* out, float phi, float* acc, void* stream);

/*
 * v <- P v row by row: P = I - n n^T for a moving surface particle (n the
 * unit normal of facet owner[i]), t t^T for a moving feature particle (t the
 * tangent of segment feat_seg[owner[i]]), I for a moving volume particle, 0
 * for a particle that does not move. The tangent space of Eq. 24-25.
 */
fppg_status fppg_tangent_project(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                 const int32_t* owner, const int32_t* feat_seg, int32_t n_feat,
                                 uint32_t move_mask, float* v, void* stream);

/*
 * disp <- alpha P v in the displacement format of fppg_project (as written by
 * fppg_relax_step, with alpha v in place of dt^2 a): the step of a
 * Newton-Krylov update, applied and projected by fppg_project.
 */
fppg_status fppg_displace(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                          const int32_t* owner, const int32_t* feat_seg, int32_t n_feat,
                          uint32_t move_mask, const float* v, float alpha, float* disp, void* stream);

/*
 * Sorted indices of the particles that move (tag 1..3 with its bit set in
 * move_mask), ascending, into list [n] (device); their number into count[0]
 * (device int32). Deterministic (block counts, prefix sum, write). ws: at
 * least fppg_workspace_size bytes. The receiver list of fppg_relax_step and
 * fppg_project for a tier in which one class moves.
 */
fppg_status fppg_moving_list(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                             uint32_t move_mask, int32_t* list, int32_t* count, void* ws, size_t ws_bytes,
                             void* stream);

/*
 * Particle generation front end (sections 3.1.1, 3.1.2, 3.2.1): on the
 * uniform background grid of edge dx with cell (i, j, k) spanning
 * origin + [i, i+1) dx etc. (centre origin + (i + 0.5) dx, FP64), classify
 * every cell and seed the initial particles of one closed mesh:
 *   surface   the cell's closed box meets a facet (separating-axis
 *             triangle-box test, FP64; touching counts);
 *   internal  not surface, and the vertical segment from below the mesh up
 *             to the centre crosses an odd number of facets (ray casting;
 *             a column through a shared edge or vertex of the facets' xy
 *             projections is counted once by an edge fill rule; vertical
 *             facets are not crossed);
 *   external  otherwise.
 * A volume particle is placed at the centre of every internal cell and a
 * surface particle at the projection of every surface cell's centre along the
 * normal of the facet meeting the cell whose foot lies inside it and whose
 * |plane distance| is smallest (ties: lowest facet); a surface cell without
 * such a facet gets no particle.
 * vert [n_vert*3] double, tri [n_tri*3] int32: host arrays, as in
 * fppg_geom_desc. origin [3] double, dims [3] int32: host; dims product below
 * 2^31. cell_class [dims[2]][dims[1]][dims[0]] uint8 (device, out): 0
 * external, 1 internal, 2 surface. pos [cap*4] float (device, 16-byte
 * aligned, out): particles in cell order (x fastest), w = the tag bits
 * (FPPG_TAG_VOLUME or FPPG_TAG_SURFACE, geometry 0); owner [cap] int32
 * (device, out): the facet of a surface particle, -1 for a volume particle.
 * counts [2] int64 (host, out): volume and surface particles written. More
 * particles than cap: FPPG_E_CAPACITY, counts[0] = -1 and counts[1] = the
 * total (call again with cap >= it). A set-up call: it allocates its device
 * temporaries (about 13 bytes per cell) and synchronises the stream.
 */
fppg_status fppg_generate(fppg_ctx* ctx, const double* vert, int32_t n_vert, const int32_t* tri, int32_t n_tri,
                          double dx, const double* origin, const int32_t* dims, uint8_t* cell_class, float* pos,
                          int32_t* owner, int64_t cap, int64_t* counts, void* stream);

/*
 * The particles of fppg_generate (the same classes, mapping, order and bits)
 * computed through the sparse storage of section 3.1.3 instead of a dense
 * per-cell class array: the cells the mesh meets are taken from a sparse grid
 * of the mesh (fppg_sparse_grid_create with cell = dx and pad = 1e-6 dx, a
 * superset of the meeting cells while the coordinates are far below 2^50 dx)
 * re-tested with the whole-facet separating-axis test; the vertical ray
 * crossings of section 3.1.2 become (column, height) events, radix-sorted, an
 * event of even multiplicity cancelling; a cell that is not a surface cell is
 * internal iff an odd number of its column's surviving events lie at or below
 * it. Memory: about 40 bytes per registered cell and per crossing event,
 * half a byte per grid column (nx * ny) and one per 256 background cells;
 * the sweep reads no per-cell array. Arguments as
 * fppg_generate without cell_class; dims each in [1, 2^21] (the Morton code),
 * nx * ny below 2^31, the cell count below 2^38. stats [4] int64 (host, out,
 * may be null): registered cells, crossing events, events left after
 * cancellation, subdivision levels. Errors as fppg_generate (capacity:
 * counts[0] = -1, counts[1] = the total). A set-up call: it allocates its
 * device temporaries and synchronises the stream.
 */
fppg_status fppg_generate_sparse(fppg_ctx* ctx, const double* vert, int32_t n_vert, const int32_t* tri,
                                 int32_t n_tri, double dx, const double* origin, const int32_t* dims, float* pos,
                                 int32_t* owner, int64_t cap, int64_t* counts, int64_t* stats, void* stream);

/*
 * Boolean combination of two solids classified by fppg_generate on the same
 * grid (section 3.2.3), cell by cell (I internal, S surface):
 *   op 0 union         I = Ai | Bi,           S = (As & ~Bi) | (Bs & ~Ai)
 *   op 1 intersection  I = Ai & Bi,           S = (As & (Bi | Bs)) | (Bs & (Ai | As))
 *   op 2 difference    I = Ai & ~(Bi | Bs),   S = (As & ~Bi) | (Bs & (Ai | As))
 * with S outside I, everything else external. a, b, out [n] uint8 (device;
 * out may alias a or b). The volume particles of the combination sit at the
 * centres of its internal cells.
 */
fppg_status fppg_cells_boolean(fppg_ctx* ctx, const uint8_t* a, const uint8_t* b, int64_t n, int32_t op,
                               uint8_t* out, void* stream);

/*
 * Sparse storage of the cells a mesh meets (section 3.1.1 facet subdivision,
 * section 3.1.3 Morton code and compact hash, Eq. 9-10), built on the device.
 *   subdivision  an edge whose extent along some axis exceeds `cell` is split
 *                at its midpoint (a + b) * 0.5, the others' midpoints are
 *                virtual; a triangle with no split edge (box within one cell
 *                per axis) is a leaf; three split edges give the 4 corner and
 *                centre triangles, two give the corner where they meet and the
 *                rest cut along the diagonal from the far end of the unsplit
 *                edge, one gives 2 triangles through the opposite vertex
 *   registration (cell, facet) for every cell whose box widened by pad a leaf
 *                of the facet meets (closed separating-axis test, FP64)
 *   C_compact    the registered cells in Morton order (Eq. 9: bits of x, y, z
 *                interleaved, x lowest), each with begin/length of its facets
 *                in the (Morton code, facet) ordered facet list
 *   hash table   H(x) = (p1 x + p2 y + p3 z) mod H_size (Eq. 10, the paper's
 *                primes, 64-bit unsigned arithmetic); C_compact's entries in
 *                (hash, Morton) order with H_begin/H_length per hash value
 * in:  vert [n_vert*3], tri [n_tri*3] (host, FP64 / int32); grid origin (the
 *      corner of cell (0,0,0)), cell edge, dims (each in [1, 2^21]); pad >= 0;
 *      hash_size (0: the number of registered cells).
 * out: *out, a device-resident structure (fppg_sparse_grid_destroy frees it).
 * Synchronous. Errors: FPPG_E_ARG (bad sizes, indices, non-finite input),
 * FPPG_E_CAPACITY (more than 48 subdivision levels or 2^31 entries).
 */
typedef struct fppg_sparse_grid fppg_sparse_grid;
typedef struct {
  int64_t n_entry;          /* length of the facet list */
  int64_t n_cell;           /* registered cells (C_compact) */
  int64_t hash_size;        /* H_size */
  int64_t levels;           /* subdivision level passes (items stored level by level) */
  const int32_t* facets;    /* [n_entry] facet ids, by (Morton code, facet) */
  const uint64_t* morton;   /* [n_cell] ascending */
  const int32_t* begin;     /* [n_cell] first entry of each cell in facets */
  const int32_t* length;    /* [n_cell] */
  const int32_t* order;     /* [n_cell] C_compact indices by (hash, Morton code) */
  const int32_t* h_begin;   /* [hash_size + 1] first position in order of each hash value */
  const int32_t* h_length;  /* [hash_size] */
} fppg_sparse_grid_view;  /* device pointers, valid until the grid is destroyed */

fppg_status fppg_sparse_grid_create(fppg_ctx* ctx, const double* vert, int32_t n_vert, const int32_t* tri,
                                    int32_t n_tri, const double origin[3], double cell, const int32_t dims[3],
                                    double pad, int64_t hash_size, fppg_sparse_grid** out);
fppg_status fppg_sparse_grid_info(const fppg_sparse_grid* grid, fppg_sparse_grid_view* view);
/* Copy the arrays of the view (sizes as there) into caller device buffers;
 * a null destination is skipped. Stream-ordered. */
fppg_status fppg_sparse_grid_copy(fppg_ctx* ctx, const fppg_sparse_grid* grid, int32_t* facets, uint64_t* morton,
                                  int32_t* begin, int32_t* length, int32_t* order, int32_t* h_begin,
                                  int32_t* h_length, void* stream);
/*
 * For each point [n*3] (device, FP64): the cell floor((p - origin) / cell)
 * (the FP64 product with 1/cell), its hash, a scan of that hash value's
 * entries for the cell's Morton code; begin [n] / length [n] (device int32)
 * of its facets in the view's facet list, or -1 / 0 for a cell outside the
 * grid or not registered. Stream-ordered.
 */
fppg_status fppg_sparse_grid_lookup(fppg_ctx* ctx, const fppg_sparse_grid* grid, int64_t n, const double* points,
                                    int32_t* begin, int32_t* length, void* stream);
fppg_status fppg_sparse_grid_destroy(fppg_sparse_grid* grid);

/*
 * Feature extraction and feature-line particles (section 3.2.2) of one mesh
 * (vert, tri as in fppg_geom_desc; host arrays):
 *   feature edge   a mesh edge with other than two facets, or whose two
 *                  facets' FP64 unit normals satisfy n1 . n2 < cos_threshold;
 *   singular       a vertex on one feature edge or on more than two;
 *   feature lines  maximal chains of feature edges between singular
 *                  vertices, each listed once from the end whose (vertex,
 *                  next vertex) pair is smaller, in the order of those pairs;
 *                  then the loops (chains without a singular vertex), each
 *                  from its smallest vertex towards its smaller neighbour, in
 *                  the order of that vertex;
 *   particles      per line of length L, n = max(1, ceil(L / dx)) equal steps
 *                  of arc length: the n - 1 interior points of an open line
 *                  (its ends are singular points), all n points of a loop
 *                  starting at its first vertex.
 * Outputs in *out (device arrays, caller-allocated, with capacities): edges
 * [2 * n_edges] int32 (u < v, ascending), singular [n_singular] int32
 * (ascending), line_begin [n_lines + 1] int32 and line_vert [n_line_vert]
 * int32 (line l is line_vert[line_begin[l] .. line_begin[l+1]-1]; a loop does
 * not repeat its first vertex), line_closed [n_lines] uint8, pos
 * [n_particles * 4] float (16-byte aligned; w = FPPG_TAG_FEATURE), line_of
 * [n_particles] int32, arc [n_particles] double (arc length from the line's
 * first vertex), seg [n_particles] int32 (the segment of the line, from its
 * vertex k to k + 1, that holds the particle) and u [n_particles] double (arc
 * length inside that segment). The n_* fields are set on return; with line_begin = NULL
 * the call only reports them (FPPG_OK); if one exceeds its capacity the call
 * returns FPPG_E_CAPACITY without writing the arrays. A set-up call: it
 * allocates device temporaries and synchronises the stream.
 */
typedef struct {
  int32_t* edges;      int64_t cap_edges;
  int32_t* singular;   int64_t cap_singular;
  int32_t* line_begin; int32_t* line_vert; uint8_t* line_closed;
  int64_t  cap_lines;  int64_t cap_line_vert;
  float*   pos;        int32_t* line_of;   double* arc;  int32_t* seg;  double* u;
  int64_t  cap_particles;
  int64_t  n_edges, n_singular, n_lines, n_line_vert, n_particles;   /* out */
} fppg_features_out;

fppg_status fppg_features(fppg_ctx* ctx, const double* vert, int32_t n_vert, const int32_t* tri, int32_t n_tri,
                          double cos_threshold, double dx, fppg_features_out* out, void* stream);

/*
 * Three-layer volume relaxation (section 3.3.4): re-tag as fixed
 * (FPPG_TAG_FIXED) every volume particle whose distance to its geometry's
 * surface mesh is at least width; the volume particles closer than width are
 * the intermediate layer that a volume tier then relaxes, with the surface
 * particles and the fixed core as sources. The distance is the exact FP64
 * point-triangle distance from the binary32 position to the facets registered
 * in the facet search cells that the box [x - width, x + width] touches.
 * pos [n*4] in/out (device; only the tag bits of w change); width: finite,
 * >= 0 (the same for every geometry); count [1] int32 (device): the number of
 * particles re-tagged. Non-finite positions keep their tags. Called once,
 * before the relaxation; its cost grows with (width / search cell edge)^3.
 * A batch with a Boolean assembly: FPPG_E_UNSUPPORTED.
 */
fppg_status fppg_volume_layers(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, float* pos, double width,
                               int32_t* count, void* stream);

/*
 * fppg_project with a per-particle record of its decisions, for reverse-mode
 * differentiation: accepted [n] uint8 (device) = 1 iff particle i moves
 * (move_mask) and its move was applied, 0 if it was reverted or does not move.
 * Otherwise identical to fppg_project (all particles, no list).
 */
fppg_status fppg_project_record(fppg_ctx* ctx, const fppg_geom* geom, int64_t n,
                                float* pos, int32_t* owner, const float* disp,
                                int32_t* feat_seg, double* feat_u, int32_t n_feat, uint32_t move_mask,
                                int64_t* counters, uint8_t* accepted, void* ws, size_t ws_bytes,
                                void* stream);

/*
 * Differentiation of a relaxation run with respect to the mesh vertices (an
 * addition to the paper's method; section 3.3 defines the step that is
 * differentiated). The discrete decisions of every step are frozen at their
 * forward values: dt^2, the owner facet (feature segment) before and after the
 * step, acceptance of the move, the direction of a feature walk, the neighbour
 * sets. Between decisions one step is the smooth map
 *   y  = x + dt^2 P_o a(x)        P_o = I - n_o n_o^T (surface), I (volume)
 *   x' = y - ((y - A_t) . n_t) n_t  accepted surface move onto facet t = owner_next
 *   x' = y                        accepted volume move
 *   x' = P0_s' + u' t_s',  u' = t_s.(x - P0_s) + dt^2 a(x).t_s + c
 *                                 accepted feature move from segment s to s', with
 *                                 c = -(lengths walked off forwards) + (lengths
 *                                 walked onto backwards), t = (P1 - P0)/|P1 - P0|
 *   x' = x                        reverted move, or a particle that does not move
 * with n = (B - A) x (C - A) / |.| of facet (A, B, C). Singular points are their
 * vertex (owner[i] = its global vertex id); every feature particle starts at
 * arc length u of its segment, P0 + u t.
 *
 * Vertex adjoints are accumulated in vbar_fixed [3 * n_vert] int64 (device,
 * zeroed by the caller) as signed fixed point with 2^-40 units by integer
 * atomics, so the result does not depend on the order of the atomics;
 * fppg_fixed_to_double converts. Global vertex ids number the vertices of
 * geometry g after those of geometries 0..g-1 (fppg_geom_desc.n_vert).
 */

/*
 * Rest density rho0 of the uniformity loss: the kernel sum of Eq. 7's form,
 * W(0) + sum over the non-zero points k dx of the infinite cubic lattice
 * (k in Z^3) of W(|k| dx), with W the Wendland C2 kernel of Eq. 16 (alpha =
 * 21/(16 pi h^3), support 2h): the density every particle of an exactly
 * uniform lattice of spacing dx has. FP64, host call (no device, no context).
 * out: one double (host). Errors: FPPG_E_ARG for a null out, dx or h not
 * finite and > 0, or 2h/dx > 1024.
 */
fppg_status fppg_lattice_density(double dx, double h, double* out);

/*
 * Uniformity loss of the positions (binary32 input, FP64 arithmetic):
 *   rho_i = W(0) + sum_{j != i, predicate(i, j)} W(|x_i - x_j|)  over all classes,
 *   L = (1/N) sum_{i moving} (rho_i / rho0 - 1)^2,  N = number of moving particles,
 * W the Wendland C2 kernel of Eq. 16 with alpha = 21/(16 pi h^3), the
 * neighbour predicate of fppg_relax_step. out [2] doubles (device): L, N.
 * grad [n*4] (device, may be NULL): dL/dx_i in binary32 (w = 0), with the
 * neighbour sets held fixed. One rho0 for the whole batch. ws: at least
 * 8 (n + 2 ceil(n/256)) + 64 bytes, 256-byte aligned.
 */
fppg_status fppg_uniformity_loss(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                                 const int32_t* cell_start, uint32_t move_mask, double rho0,
                                 double* out, float* grad, void* ws, size_t ws_bytes, void* stream);

/*
 * Adjoint of one step through the projection, the tangential displacement
 * and the feature walk. Particle arrays in the sorted order of that step: pos
 * and owner entering it (after fppg_build_cells), owner_next and accepted after
 * fppg_project_record, accel and amax written by fppg_relax_step; feature
 * tables by slot: fseg_before (segments entering the step), fseg_after and
 * fu_after (after it), n_feat slots (may be NULL if 0). Given xbar_next =
 * dL/dx', writes
 *   ybar_i = dL/da_i through this step (0 unless accepted)
 *   xbar_i = the direct part of dL/dx_i (xbar_next_i if not accepted)
 * and adds the facet- and segment-vertex terms to vbar_fixed. The caller
 * completes dL/dx = xbar + J^T ybar with fppg_relax_hvp(transpose = 1). xbar
 * must not alias xbar_next.
 */
fppg_status fppg_step_adjoint(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                              const uint8_t* accepted, const int32_t* owner, const int32_t* owner_next,
                              const float* accel, const float* amax, const int32_t* fseg_before,
                              const int32_t* fseg_after, const double* fu_after, int32_t n_feat,
                              uint32_t move_mask, const float* xbar_next, float* ybar, float* xbar,
                              int64_t* vbar_fixed, void* stream);

/*
 * Vertex terms of the initial positions that are functions of the mesh: for
 * each particle with adjoint xbar_i, a singular point adds xbar_i to vertex
 * owner[i]; a feature particle (slot owner[i], segment feat_seg[slot] of the
 * initial state with end vertices from fppg_geom_desc.seg_vert, arc length
 * feat_u[slot]) adds (u/L)(I - t t^T) xbar_i to P1 and the rest of xbar_i to
 * P0. Surface, volume and fixed particles start at given positions.
 */
fppg_status fppg_fixed_adjoint(fppg_ctx* ctx, const fppg_geom* geom, int64_t n, const float* pos,
                               const int32_t* owner, const int32_t* feat_seg, const double* feat_u,
                               int32_t n_feat, uint32_t move_mask, const float* xbar, int64_t* vbar_fixed,
                               void* stream);

/* Row permutation of a float4 field: scatter = 0: dst[i] = src[index[i]];
 * scatter = 1: dst[index[i]] = src[i]. index is a permutation of [0, n);
 * rows with an out-of-range index are skipped. dst must not alias src. */
fppg_status fppg_vec_permute(fppg_ctx* ctx, int64_t n, const float* src, const int32_t* index,
                             int32_t scatter, float* dst, void* stream);

/* out[i] = in[i] * 2^-40 (fixed-point vertex adjoints to double), device arrays. */
fppg_status fppg_fixed_to_double(fppg_ctx* ctx, int64_t count, const int64_t* in, double* out, void* stream);

/*
 * HIP-graph capture of whole iterations (build_cells -> relax_step ->
 * project). Iteration t reads particle buffer set A for even t and B for odd
 * t and writes the other one; `iters` must be even (>= 2) so the state
 * returns to set A and the graph can be replayed back to back. All other
 * buffers are those of the per-iteration calls (accel is the workspace's).
 * Capture uses `stream` (must not be the default stream) in thread-local mode;
 * profiling must be off. fppg_graph_launch enqueues `repeats` replays
 * (repeats * iters iterations) on `stream`. Every node is a kernel.
 */
typedef struct fppg_graph fppg_graph;
fppg_status fppg_graph_create(fppg_ctx* ctx, const fppg_geom* geom, int64_t n,
                              float* pos_a, int32_t* id_a, int32_t* owner_a,
                              float* pos_b, int32_t* id_b, int32_t* owner_b, int32_t* cell_start,
                              int32_t* feat_seg, double* feat_u, int32_t n_feat, uint32_t move_mask,
                              float* amax, float* disp, int64_t* counters, void* ws, size_t ws_bytes,
                              int32_t iters, void* stream, fppg_graph** out);
fppg_status fppg_graph_launch(fppg_ctx* ctx, fppg_graph* graph, int32_t repeats, void* stream);
void        fppg_graph_destroy(fppg_graph* graph);

/*
 * Test/diagnostic export of the neighbour sets seen by the force traversal:
 * for every particle i (moving or not), count[i] = |{j != i : predicate}| over
 * all tags of its geometry, and list[i*cap .. i*cap+min(count,cap)-1] the
 * sorted indices j in traversal order. count [n] int32, list [n*cap] int32.
 */
fppg_status fppg_debug_neighbors(fppg_ctx* ctx, const fppg_geom* geom, int64_t n,
                                 const float* pos, const int32_t* cell_start,
                                 int32_t* count, int32_t* list, int32_t cap, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FPPG_H */

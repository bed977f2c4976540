"""Cell list rebuilt every iteration ("updating data structures", Algorithm 1).

The paper keys its sparse background grid by Morton code and a compact hash
(section 3.1.3, Eq. 9-10). For the particle cell list of the relaxation loop
the key here is a linear index of a uniform grid with x fastest, offset per
geometry of a batch; particles are ordered by (key, id), and cell_start[c] is
the first sorted index of cell c. The grid's y range is cut into slabs of S
rows (the last one may be narrower); the key runs over the slabs, within a
slab over z, then over its rows y, then x:
    key = s S nx nz + cz nx w + (cy - s S) nx + cx,  s = cy div S,  w = min(S, ny - s S)
S = ny (or S <= 0) is the plain (cz ny + cy) nx + cx. Every key order with
contiguous x rows describes the same cell list; slabs keep the cells a
receiver's stencil touches close together in memory.

A particle with a non-finite coordinate gets the key ncell (one past every
geometry's cells; reading: such a particle is nobody's neighbour), so
cell_start has ncell + 2 entries, the last being N.

The cells are those of the geometry's grid (origin, inv_cell, dims) split in
X_SPLIT along x (nx = X_SPLIT dims[0] cells per row), a layout choice of the
library's stencil (half-width cells along x). The cell coordinate is defined
in binary32, one rounding per operation:
    t = fl32(fl32(x - origin) * inv),  c = clamp(floor(t), 0, n - 1)
with inv = fl32(X_SPLIT inv_cell) (exact) and n = nx along x, inv = inv_cell
and n = dims along y and z, NaN mapped to cell 0. Geometry g's keys start at
the total cell count of geometries 0..g-1.
"""
import numpy as np

X_SPLIT = 2


def grid_dims(geo):
    """Cells per axis of a geometry's particle grid (x split)."""
    return (X_SPLIT * int(geo.dims[0]), int(geo.dims[1]), int(geo.dims[2]))


def geometry_cells(geo) -> int:
    nx, ny, nz = grid_dims(geo)
    return nx * ny * nz


def cell_coords(pos32: np.ndarray, origin, inv_cell, dims) -> np.ndarray:
    """Integer cell coordinates [N, 3] of binary32 positions [N, 3] in the grid
    (origin, inv_cell, dims) with its cells split in X_SPLIT along x; dims are
    the unsplit grid's."""
    p = np.asarray(pos32, np.float32)
    t = (p - np.asarray(origin, np.float32)).astype(np.float32)
    inv = np.array([X_SPLIT * np.float32(inv_cell), inv_cell, inv_cell], np.float32)
    t = (t * inv).astype(np.float32)
    n = np.array([X_SPLIT * int(dims[0]), int(dims[1]), int(dims[2])], np.int64)
    t = np.fmin(np.fmax(t, np.float32(0.0)), (n - 1).astype(np.float32))   # fmax/fmin drop NaN -> 0
    return np.floor(t).astype(np.int64)


def cell_keys(wl, pos32=None, gid=None) -> np.ndarray:
    """Batch-global cell key of every particle of a workload."""
    pos32 = wl.pos if pos32 is None else pos32
    gid = wl.gid if gid is None else gid
    keys = np.empty(len(pos32), np.int64)
    begin = 0
    for g, geo in enumerate(wl.geoms):
        m = gid == g
        c = cell_coords(pos32[m], geo.origin, geo.inv_cell, geo.dims)
        keys[m] = begin + linear_key(c, grid_dims(geo), getattr(geo, "slab", 0))
        begin += geometry_cells(geo)
    keys[~np.all(np.isfinite(pos32), axis=1)] = total_cells(wl)
    return keys


def linear_key(c: np.ndarray, dims, slab: int) -> np.ndarray:
    """Key of integer cell coordinates c [N, 3] inside one geometry's grid."""
    nx, ny, nz = (int(d) for d in dims)
    S = ny if slab <= 0 else min(int(slab), ny)
    s = c[:, 1] // S
    w = np.minimum(S, ny - s * S)
    return s * (S * nx * nz) + c[:, 2] * (nx * w) + (c[:, 1] - s * S) * nx + c[:, 0]


def total_cells(wl) -> int:
    return int(sum(geometry_cells(g) for g in wl.geoms))


def sort_order(keys: np.ndarray, ids: np.ndarray) -> np.ndarray:
    """Permutation putting particles in (key, id) order."""
    return np.lexsort((ids, keys))


def cell_start(sorted_keys: np.ndarray, ncell: int) -> np.ndarray:
    """Exclusive prefix sum of the per-cell particle counts (the ncell cells
    and the non-finite key ncell), length ncell + 2."""
    counts = np.bincount(sorted_keys, minlength=ncell + 1)
    out = np.zeros(ncell + 2, np.int64)
    np.cumsum(counts, out=out[1:])
    return out

"""Pins of the oracle's facet registration and sparse storage
(oracle/register.py: section 3.1.1 subdivision, section 3.1.3 Eq. 9-10):

  * Morton codes of Eq. 9 by hand, and the octant order of a 2^k block
  * the subdivision tiles each facet: leaf areas sum to the facet's, every
    leaf keeps its facet's orientation and fits one cell; child counts of
    the three split patterns; a right triangle of legs 3 cells gives 16
  * the registration through the leaves equals the cells met by the whole
    facets (no subdivision), since a cell meets a facet iff it meets one of
    its leaves
  * the hash of Eq. 10 by hand; every registered cell is found through the
    hash table with exactly its facets, unregistered cells with none
"""
import numpy as np
import pytest

from oracle import generate as ogen
from oracle import register as R
from synth import meshes as M


def test_morton_codes_by_hand():
    assert [R.morton(1, 0, 0), R.morton(0, 1, 0), R.morton(0, 0, 1), R.morton(2, 0, 0)] == [1, 2, 4, 8]
    # x = 011, y = 101, z = 110: z2 y2 x2 | z1 y1 x1 | z0 y0 x0 = 110 101 011
    assert R.morton(3, 5, 6) == 0b110101011
    assert R.morton(2 ** 21 - 1, 2 ** 21 - 1, 2 ** 21 - 1) == 2 ** 63 - 1
    # a 4^3 block in Morton order visits each 2^3 octant whole before the next
    codes = {R.morton(x, y, z): (x, y, z) for x in range(4) for y in range(4) for z in range(4)}
    seq = [codes[c] for c in sorted(codes)]
    for o in range(8):
        octant = {(x // 2, y // 2, z // 2) for x, y, z in seq[8 * o: 8 * o + 8]}
        assert len(octant) == 1
    assert sorted(codes) == list(range(64))


def _area(a, b, c):
    return 0.5 * np.linalg.norm(np.cross(np.subtract(b, a), np.subtract(c, a)))


def _normal(a, b, c):
    n = np.cross(np.subtract(b, a), np.subtract(c, a))
    return n / np.linalg.norm(n)


def test_child_counts_of_the_three_split_patterns():
    cell = 1.0
    assert R.children((0, 0, 0), (0.5, 0, 0), (0, 0.5, 0), cell) is None
    assert len(R.children((0, 0, 0), (3, 0, 0), (0, 3, 0), cell)) == 4          # all three edges
    assert len(R.children((0, 0, 0), (3, 0, 0), (0, 0.5, 0), cell)) == 3        # (c, a) virtual
    assert len(R.children((0, 0, 0), (1.5, 0, 0), (0.75, 0.5, 0), cell)) == 2   # only (a, b)
    # the leaf count of a right triangle of legs 3 cells: 4 children of legs
    # 1.5, each into 4 of legs 0.75
    v = np.array([[0, 0, 0], [3, 0, 0], [0, 3, 0]], float)
    assert len(R.subdivide(v, np.array([[0, 1, 2]]), 1.0)) == 16


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_subdivision_tiles_every_facet(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    vert = rng.uniform(-2.0, 2.0, size=(60, 3))
    vert[:, 2] *= rng.uniform(0.01, 1.0)           # some thin, slanted facets
    tri = np.array([rng.choice(60, 3, replace=False) for _ in range(40)], np.int32)
    cell = 0.37
    leaves = R.subdivide(vert, tri, cell)
    area = np.zeros(len(tri))
    for t, a, b, c in leaves:
        box = np.ptp(np.array([a, b, c]), axis=0)
        assert (box <= cell).all()
        assert np.dot(_normal(a, b, c), _normal(*vert[tri[t]])) > 1 - 1e-9
        area[t] += _area(a, b, c)
    want = np.array([_area(*vert[f]) for f in tri])
    np.testing.assert_allclose(area, want, rtol=1e-12)


def _whole_facet_cells(vert, tri, origin, cell, dims, pad):
    """Every cell whose padded box the whole facet meets (no subdivision)."""
    rows = []
    for t, f in enumerate(tri):
        P = vert[f]
        lo = np.maximum(np.floor((P.min(0) - pad - origin) / cell).astype(int), 0)
        hi = np.minimum(np.floor((P.max(0) + pad - origin) / cell).astype(int), np.asarray(dims) - 1)
        for z in range(lo[2], hi[2] + 1):
            for y in range(lo[1], hi[1] + 1):
                for x in range(lo[0], hi[0] + 1):
                    c = origin + (np.array([x, y, z]) + 0.5) * cell
                    if ogen.tri_box_overlap(c[None], np.full((1, 3), 0.5 * cell + pad), P[0][None], P[1][None],
                                            P[2][None])[0]:
                        rows.append((x, y, z, t))
    return sorted(rows, key=lambda r: (r[2], r[1], r[0], r[3]))


@pytest.mark.parametrize("mesh,cell", [("sphere", 0.21), ("cube", 0.13), ("tetra", 0.05), ("cylinder", 0.09)])
def test_registration_through_leaves_equals_whole_facets(mesh, cell):
    m = {"sphere": lambda: M.icosphere(2), "cube": lambda: M.cube(), "tetra": lambda: M.tetrahedron(),
         "cylinder": lambda: M.cylinder(0.5, 1.0, 32)}[mesh]()
    lo, hi = m.vert.min(0), m.vert.max(0)
    origin = lo - 2.0 * cell
    dims = (np.ceil((hi - lo) / cell).astype(int) + 5).tolist()
    pad = 1e-6 * cell
    got = R.register(m.vert, m.tri, origin, cell, dims, pad)
    want = np.array(_whole_facet_cells(m.vert, m.tri, origin, cell, dims, pad), np.int64)
    assert np.array_equal(got, want)
    # the dense CSR lists each cell's facets ascending
    start, fac = R.dense_csr(got, dims)
    assert start[-1] == len(got) and np.all(np.diff(start) >= 0)


def test_hash_by_hand_and_lookup_through_the_table():
    assert R.hash_value(1, 0, 0, 1000) == 738560931 % 1000
    assert R.hash_value(1, 2, 3, 97) == (738560931 + 2 * 19349663 + 3 * 83492791) % 97
    big = 2 ** 21 - 1
    assert R.hash_value(big, big, big, 2 ** 31 - 1) == ((738560931 + 19349663 + 83492791) * big) % (2 ** 64) % (
        2 ** 31 - 1)
    m = M.icosphere(2)
    cell = 0.23
    origin = m.vert.min(0) - 2 * cell
    dims = (np.ceil(np.ptp(m.vert, 0) / cell).astype(int) + 5).tolist()
    rows = R.register(m.vert, m.tri, origin, cell, dims, 0.0)
    for size in (None, 7, 1):
        sp = R.sparse(rows, size)
        assert sp.h_length.sum() == len(sp.morton) and sp.h_begin[-1] + sp.h_length[-1] == len(sp.morton)
        cells = {}
        for x, y, z, t in rows:
            cells.setdefault((x, y, z), []).append(t)
        for (x, y, z), fs in cells.items():
            assert list(R.lookup(sp, x, y, z)) == sorted(fs)
        rng = np.random.Generator(np.random.PCG64(5))
        for x, y, z in rng.integers(0, min(dims), size=(200, 3)):
            if (x, y, z) not in cells:
                assert len(R.lookup(sp, x, y, z)) == 0

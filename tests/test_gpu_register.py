"""GPU parity of the facet registration (section 3.1.1 subdivision) and of
the sparse storage of the registered cells (section 3.1.3, Eq. 9-10)
against the oracle (oracle/register.py), bit for bit: the facet lists, the
Morton-ordered compact list, the hash table, lookups, and the facet search
grid that geometry creation registers on the device."""
import numpy as np
import pytest

import synth
from oracle import register as oreg
from synth import meshes as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _grid(mesh, cell):
    origin = mesh.vert.min(0) - 2.0 * cell
    dims = (np.ceil(np.ptp(mesh.vert, 0) / cell).astype(int) + 5).tolist()
    return origin, dims


MESHES = {
    "icosphere3": (lambda: M.icosphere(3), 0.07),
    "cube": (lambda: M.cube(), 0.13),
    "cylinder64": (lambda: M.cylinder(0.5, 1.0, 64), 0.05),
    "tetra_fine": (lambda: M.tetrahedron(), 0.011),
}


_ROWS = {}


def _rows(name, m, origin, cell, dims, pad):
    if name not in _ROWS:
        _ROWS[name] = oreg.register(m.vert, m.tri, origin, cell, dims, pad)
    return _ROWS[name]


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("hash_size", [0, 7])
def test_sparse_grid_bit_exact(name, hash_size):
    _need_gpu()
    from paper_2501_03056_amd.front import SparseGrid
    make, cell = MESHES[name]
    m = make()
    origin, dims = _grid(m, cell)
    pad = 1e-6 * cell
    print(f"[register] {name} facets={len(m.tri)} cell={cell} dims={dims} hash={hash_size}", flush=True)
    sg = SparseGrid(m.vert, m.tri, origin, cell, dims, pad=pad, hash_size=hash_size)
    rows = _rows(name, m, origin, cell, dims, pad)
    ref = oreg.sparse(rows, hash_size or None)
    a = {k: v.cpu().numpy() for k, v in sg.arrays().items()}
    assert sg.n_entry == len(rows) and sg.n_cell == len(ref.morton) and sg.hash_size == ref.size
    assert np.array_equal(a["facets"], ref.facets)
    assert np.array_equal(a["morton"].view(np.uint64), ref.morton)
    assert np.array_equal(a["begin"], ref.begin) and np.array_equal(a["length"], ref.length)
    assert np.array_equal(a["order"], ref.order)
    assert np.array_equal(a["h_begin"][:-1], ref.h_begin) and np.array_equal(a["h_length"], ref.h_length)
    assert a["h_begin"][-1] == len(ref.morton)
    # lookups: every registered cell's centre, random points, points outside, NaN
    rng = np.random.Generator(np.random.PCG64(11))
    cen = np.asarray(origin) + (ref.xyz.astype(np.float64) + 0.5) * cell
    lo, hi = np.asarray(origin) - cell, np.asarray(origin) + (np.asarray(dims) + 1) * cell
    pts = np.concatenate([cen, rng.uniform(lo, hi, size=(4000, 3)), [[np.nan, 0.0, 0.0]]])
    b, ln = sg.lookup(torch.as_tensor(pts))
    b, ln = b.cpu().numpy(), ln.cpu().numpy()
    fac = a["facets"]
    for i, p in enumerate(pts):
        if not np.all(np.isfinite(p)):
            assert b[i] == -1 and ln[i] == 0
            continue
        c = np.floor((p - origin) * (1.0 / cell)).astype(np.int64)
        if np.any(c < 0) or np.any(c >= dims):
            assert b[i] == -1 and ln[i] == 0
            continue
        want = oreg.lookup(ref, *c)
        got = fac[b[i]: b[i] + ln[i]] if b[i] >= 0 else np.zeros(0, np.int64)
        assert np.array_equal(got, want), (i, p)
    sg.close()


def test_sparse_grid_of_an_empty_mesh():
    _need_gpu()
    from paper_2501_03056_amd.front import SparseGrid
    sg = SparseGrid(np.zeros((0, 3)), np.zeros((0, 3), np.int32), (0, 0, 0), 0.1, (4, 4, 4))
    assert sg.n_entry == 0 and sg.n_cell == 0 and sg.hash_size == 1
    b, ln = sg.lookup(torch.tensor([[0.05, 0.05, 0.05]], dtype=torch.float64))
    assert int(b[0]) == -1 and int(ln[0]) == 0


def _search_grid(r):
    import ctypes
    from paper_2501_03056_amd._lib import check, ptr
    nc, ne = ctypes.c_int64(), ctypes.c_int64()
    check(r.ctx.lib.fppg_geom_info(r.geom.handle, None, None, None, ctypes.byref(nc), ctypes.byref(ne)))
    start = torch.empty(nc.value + 1, dtype=torch.int32, device=r.dev)
    tri = torch.empty(max(ne.value, 1), dtype=torch.int32, device=r.dev)
    flag = torch.empty(max(nc.value, 1), dtype=torch.uint8, device=r.dev)
    check(r.ctx.lib.fppg_geom_search_grid(r.ctx.handle, r.geom.handle, ptr(start), ptr(tri), ptr(flag), r.stream),
          r.ctx.handle)
    torch.cuda.synchronize()
    return start.cpu().numpy(), tri.cpu().numpy()[: ne.value], flag.cpu().numpy()[: nc.value]


@pytest.mark.parametrize("case", ["sphere_l3", "gear_coarse", "batch3"])
def test_search_grid_registered_on_the_device(case):
    """The facet search grid of the projection (cells of edge R (1 + 2^-6),
    pad 1e-6 cell, the geometries' grids one after another) equals the
    oracle's registration of each mesh."""
    _need_gpu()
    from paper_2501_03056_amd import Relaxer
    wl = {"sphere_l3": lambda: synth.sphere_workload(level=3, dx=0.08, seed=2),
          "gear_coarse": lambda: synth.gear_workload(dx=0.04, seed=3, samples_per_period=12, rings=4),
          "batch3": lambda: synth.workload.solid_batch_workload(n_geom=3, n_min=2e3, n_max=4e3, seed=77)}[case]()
    r = Relaxer(wl, device=0)
    start, tri, flag = _search_grid(r)
    base_cell, base_entry = 0, 0
    for g in wl.geoms:
        cell = float(g.proj_radius) * (1.0 + 1.0 / 64.0)
        lo = g.mesh.vert.min(0)
        origin = lo - 2.0 * cell
        dims = [int(np.ceil((g.mesh.vert[:, q].max() - lo[q]) * (1.0 / cell))) + 5 for q in range(3)]
        rows = oreg.register(g.mesh.vert, g.mesh.tri, origin, cell, dims, 1e-6 * cell)
        s_ref, f_ref = oreg.dense_csr(rows, dims)
        n = int(np.prod(dims))
        got_start = start[base_cell: base_cell + n + 1] - base_entry
        assert np.array_equal(got_start, s_ref), case
        assert np.array_equal(tri[base_entry: base_entry + len(f_ref)], f_ref + g.tri_begin)
        assert np.array_equal(flag[base_cell: base_cell + n] != 0, np.diff(s_ref) > 0)
        base_cell += n
        base_entry += len(f_ref)
    assert base_cell == len(flag) and base_entry == len(tri)

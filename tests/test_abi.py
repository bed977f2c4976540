"""The C-ABI library loads, exports every entry point of include/fppg.h and
validates its arguments on the host (no GPU needed); the product path and the
oracle stay independent."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fppg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fppg_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    from paper_2501_03056_amd import _lib
    L = _lib.lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib._SIGS), set(names) ^ set(_lib._SIGS)


def test_host_side_validation_without_gpu():
    from paper_2501_03056_amd import _lib
    L = _lib.lib()
    assert L.fppg_status_str(-3) == b"workspace too small"
    assert L.fppg_status_str(0) == b"ok"
    assert L.fppg_last_error(None) == b"null context"
    nul = None
    assert L.fppg_build_cells(nul, nul, 0, nul, nul, nul, nul, nul, nul, nul, nul, 0, nul) == _lib.E_ARG
    assert L.fppg_relax_step(nul, nul, 0, nul, nul, nul, nul, 0, 0, 0, nul, nul, nul, nul, 0, nul, 0, nul) == _lib.E_ARG
    assert L.fppg_project(nul, nul, 0, nul, nul, nul, nul, nul, 0, 0, nul, nul, 0, nul, 0, nul) == _lib.E_ARG
    assert L.fppg_moving_list(nul, nul, 0, nul, 0, nul, nul, nul, 0, nul) == _lib.E_ARG
    assert L.fppg_volume_layers(nul, nul, 0, nul, 0.1, nul, nul) == _lib.E_ARG
    assert L.fppg_set_launch(nul, 256, 1) == _lib.E_ARG
    assert L.fppg_set_schedule(nul, 1) == _lib.E_ARG
    assert L.fppg_tier_partition(nul, nul, 0, nul, nul, nul, nul, nul, nul, 0, nul, nul, 0, nul) == _lib.E_ARG
    assert L.fppg_generate(nul, nul, 0, nul, 0, 0.1, nul, nul, nul, nul, nul, 0, nul, nul) == _lib.E_ARG
    assert L.fppg_features(nul, nul, 0, nul, 0, 0.5, 0.1, nul, nul) == _lib.E_ARG
    assert L.fppg_cells_boolean(nul, nul, nul, 4, 0, nul, nul) == _lib.E_ARG
    assert L.fppg_relax_hvp(nul, nul, 0, nul, nul, 0, 0, nul, nul, nul) == _lib.E_ARG
    assert L.fppg_debug_neighbors(nul, nul, 0, nul, nul, nul, nul, 0, nul) == _lib.E_ARG
    assert L.fppg_project_record(nul, nul, 0, nul, nul, nul, nul, nul, 0, 0, nul, nul, nul, 0, nul) == _lib.E_ARG
    assert L.fppg_uniformity_loss(nul, nul, 0, nul, nul, 0, 1.0, nul, nul, nul, 0, nul) == _lib.E_ARG
    assert L.fppg_step_adjoint(nul, nul, 0, nul, nul, nul, nul, nul, nul, nul, nul, nul, 0, 0, nul, nul, nul, nul,
                               nul) == _lib.E_ARG
    assert L.fppg_fixed_adjoint(nul, nul, 0, nul, nul, nul, nul, 0, 0, nul, nul, nul) == _lib.E_ARG
    assert L.fppg_vec_permute(nul, 0, nul, nul, 0, nul, nul) == _lib.E_ARG
    assert L.fppg_fixed_to_double(nul, 0, nul, nul, nul) == _lib.E_ARG
    b = ctypes.c_size_t()
    assert L.fppg_workspace_size(nul, 10, ctypes.byref(b)) == _lib.E_ARG
    assert L.fppg_geom_info(nul, None, None, None, None, None) == _lib.E_ARG
    assert L.fppg_geom_create(nul, None, 0, None) == _lib.E_ARG
    import torch
    if not torch.cuda.is_available():
        h = ctypes.c_void_p()
        assert L.fppg_create(0, ctypes.byref(h)) == _lib.E_NODEVICE


def _py_sources(d):
    for base, _, files in os.walk(os.path.join(ROOT, d)):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                yield os.path.join(base, f)


def test_product_path_does_not_use_the_oracle():
    for f in _py_sources("paper_2501_03056_amd"):
        src = open(f).read()
        assert not re.search(r"^\s*(from|import)\s+oracle\b", src, re.M), f
        assert "oracle." not in src, f


def test_oracle_does_not_use_the_product_path():
    for f in _py_sources("oracle"):
        src = open(f).read()
        assert "paper_2501_03056_amd" not in src, f


def test_relaxer_refuses_to_run_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import synth
    from paper_2501_03056_amd import Relaxer
    with pytest.raises(RuntimeError):
        Relaxer(synth.cube_workload(n=4))


def test_loader_refuses_a_stale_build(tmp_path):
    """The library carries the hash of the sources it was built from; the
    loader compares it with the tree's sources (a stale build is rebuilt)."""
    from paper_2501_03056_amd import _lib, build as B
    L = _lib.lib()
    want = B.source_hash()
    assert L.fppg_source_hash().decode() == want
    assert B.built_hash(_lib.LIB_PATH) == want
    # a copy whose embedded hash differs is recognised as stale
    data = open(_lib.LIB_PATH, "rb").read()
    i = data.find(B.HASH_MARK) + len(B.HASH_MARK)
    stale = data[:i] + b"0" * 32 + data[i + 32:]
    p = tmp_path / "libfppg_stale.so"
    p.write_bytes(stale)
    assert B.built_hash(str(p)) != want
    assert B.built_hash(str(tmp_path / "missing.so")) is None


def test_rest_density_is_computed_by_the_library():
    """rho0 of the uniformity loss comes from fppg_lattice_density (the Python
    package holds no kernel arithmetic); it equals the oracle's lattice sum."""
    from oracle import metrics
    from paper_2501_03056_amd import _lib
    L = _lib.lib()
    for dx in (0.01, 0.045, 0.12, 1.0 / 24):
        h = float(np.float32(1.3 * dx))
        out = ctypes.c_double()
        assert L.fppg_lattice_density(dx, h, ctypes.byref(out)) == _lib.OK
        assert out.value == pytest.approx(metrics.lattice_density(dx, h), rel=1e-13)
    out = ctypes.c_double()
    assert L.fppg_lattice_density(0.0, 1.0, ctypes.byref(out)) == _lib.E_ARG
    assert L.fppg_lattice_density(1.0, float("nan"), ctypes.byref(out)) == _lib.E_ARG
    assert L.fppg_lattice_density(1.0, 1.0, None) == _lib.E_ARG
    for f in _py_sources("paper_2501_03056_amd"):
        if f.endswith(".py"):
            src = open(f).read()
            assert "np.pi" not in src and "math.pi" not in src and "21.0 /" not in src, f

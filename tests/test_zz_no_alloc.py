"""fppg_vec_dot_noalloc (the dot product without a workspace, for callers that
cannot allocate) through the C ABI: bitwise equal to fppg_vec_dot on the same
inputs, on two calls in a row with the second smaller, and on an empty input."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ctx():
    from paper_2501_03056_amd import _lib
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L = _lib.lib()
    h = ctypes.c_void_p()
    _lib.check(L.fppg_create(0, ctypes.byref(h)))
    return L, h


def _dot_ws(L, h, n, a, b, out, stream):
    """fppg_vec_dot with a caller workspace (the entry point the no-alloc one mirrors)."""
    from paper_2501_03056_amd._lib import check, ptr
    ws = torch.empty(2048 * 8 + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    check(L.fppg_vec_dot(h, n, ptr(a), ptr(b), ptr(out), ctypes.c_void_p(ws.data_ptr() + off), 2048 * 8, stream), h)
    return ws


def test_noalloc_dot_equals_workspace_dot_on_consecutive_calls():
    from paper_2501_03056_amd._lib import check, ptr
    L, h = _ctx()
    try:
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        rng = np.random.Generator(np.random.PCG64(77))
        for n in (3_000_001, 70_001, 1, 0):   # consecutive calls, each smaller than the one before
            print(f"[no_alloc] n={n}", flush=True)
            x = rng.normal(size=(max(n, 1), 4)).astype(np.float32)
            y = rng.normal(size=(max(n, 1), 4)).astype(np.float32)
            a = torch.from_numpy(x).cuda()
            b = torch.from_numpy(y).cuda()
            want = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
            got = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
            ws = _dot_ws(L, h, n, a, b, want, stream)
            check(L.fppg_vec_dot_noalloc(h, n, ptr(a), ptr(b), ptr(got), stream), h)
            torch.cuda.synchronize()
            del ws
            w, g = float(want.item()), float(got.item())
            assert np.float64(g).tobytes() == np.float64(w).tobytes(), (n, g, w)
            x64, y64 = x[:n, :3].astype(np.float64), y[:n, :3].astype(np.float64)
            # binary32 products are exact in FP64; two summation orders differ by at most 2 n u sum|x_i y_i|
            assert abs(g - float(np.sum(x64 * y64))) <= 2 * max(n, 1) * 2.0 ** -53 * float(np.sum(np.abs(x64 * y64)))
        # argument errors are reported, not launched
        assert L.fppg_vec_dot_noalloc(h, -1, None, None, None, stream) == -1
        assert L.fppg_vec_dot_noalloc(h, 4, None, None, ptr(got), stream) == -1
        assert L.fppg_vec_dot_noalloc(None, 4, None, None, None, stream) == -1
    finally:
        L.fppg_destroy(h)

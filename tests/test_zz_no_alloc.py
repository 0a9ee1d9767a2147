"""kv_project_mixed_static: the mixed-form projection whose scratch vector
lives in the library's static device array, for callers that cannot
allocate.  Through the C ABI, against kv_project with KV_MIXED (the same
kernels with the scratch in a caller workspace) on two calls in a row, the
second on a smaller grid, and against the oracle's projection; a grid whose
scratch exceeds the static size is rejected without touching its input."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import disc as O  # noqa: E402
from synth import inputs as S  # noqa: E402
from tests.gpu_util import assert_parity, faces, to_dev, to_host  # noqa: E402

pytestmark = pytest.mark.gpu


def _static(ctx):
    lib = ctx._lib
    fn = lib.kv_project_mixed_static
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    fn.restype = ctypes.c_int
    return fn


def _one(shape, seed):
    from paper_2210_08816_amd import kv
    print(f"case no-alloc mixed projection {shape}", flush=True)
    fx = [faces("clustered", n) for n in shape]
    g = O.Grid(*fx, Gr=4e7, Pr=0.71)
    ctx = kv.Context(*fx, Gr=4e7, Pr=0.71)
    try:
        y0 = S.perturbation(g.size, seed)
        ya = to_dev(y0)
        dm_a, sw_a = ctx.project(ya, mixed=True)           # workspace path
        yb = to_dev(y0)
        dm = ctypes.c_double()
        sw = ctypes.c_int()
        rc = _static(ctx)(ctx._h, ctypes.c_void_p(yb.data_ptr()), ctypes.byref(dm), ctypes.byref(sw))
        assert rc == kv.KV_OK, ctx._lib.kv_last_error(ctx._h)
        got_a, got_b = to_host(ya), to_host(yb)
        assert sw.value == sw_a and sw.value >= 2
        assert np.array_equal(got_a, got_b)                 # the same kernels on the same input
        assert dm.value == dm_a and dm.value <= 1e-10
        assert_parity(g, got_b, O.project(g, y0), 1e-5, label=f"static mixed P {shape}")
    finally:
        ctx.close()


def test_static_mixed_projection_matches_workspace_path():
    _one((48, 40, 32), 61)
    _one((16, 12, 10), 62)          # a second call, smaller: the array keeps the first call's contents


def test_static_mixed_projection_rejects_oversize_grid():
    from paper_2210_08816_amd import kv
    f = faces("clustered", 130)     # n = 8.74e6 unknowns: 70 MB of scratch, above the 64 MiB array
    ctx = kv.Context(f, f, f, Gr=4e7, Pr=0.71)
    try:
        y = torch.full((ctx.n,), 3.0, dtype=torch.float64, device="cuda")
        rc = _static(ctx)(ctx._h, ctypes.c_void_p(y.data_ptr()), None, None)
        assert rc == kv.KV_EINVAL
        assert "static" in ctx._lib.kv_last_error(ctx._h).decode()
        torch.cuda.synchronize()
        assert bool((y == 3.0).all())
    finally:
        ctx.close()

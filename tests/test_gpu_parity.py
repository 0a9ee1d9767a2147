"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Tolerance: FP64 results agree with the FP64 oracle to 1e-12 relative per
field (||delta y_f||_2 / ||y_f||_2).  Grids span several 64-wide tiles with
ragged tails, odd and unequal sizes, both grid kinds.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import disc as O  # noqa: E402
from synth import inputs as S  # noqa: E402
from tests.gpu_util import assert_parity, faces, to_dev, to_host  # noqa: E402

pytestmark = pytest.mark.gpu

TOL64 = 1e-12

GRIDS = [
    ("uniform", (32, 32, 32), 1e5, 3, 0.05),      # the 32^3 uniform workload's shape
    ("clustered", (7, 6, 5), 2e5, 2, 0.1),        # odd, unequal, smaller than one tile
    ("clustered", (70, 9, 66), 4e7, 4, 0.1),      # one full tile plus ragged tails
    ("uniform", (2, 3, 2), 1e3, 1, 0.1),          # minimal sizes
    ("clustered", (36, 20, 44), 4e7, 3, 0.1),     # even half sizes (pair loads), ragged FD tiles on every axis
    ("clustered", (7, 12, 8), 2e5, 2, 0.1),       # y pass: even half size, odd line length (single loads)
]


def make(kind, shape, Gr, K, amp, seed=0):
    from paper_2210_08816_amd import kv
    fx = [faces(kind, n) for n in shape]
    g = O.Grid(*fx, Gr=Gr, Pr=0.71)
    X0 = S.base_flow(*fx, K=K, amp=amp, seed=seed)
    ctx = kv.Context(*fx, Gr=Gr, Pr=0.71)
    assert ctx.n == g.size
    ctx.set_base_flow(to_dev(X0))
    return g, X0, ctx


@pytest.mark.parametrize("kind,shape,Gr,K,amp", GRIDS)
def test_jacobian_unprojected(kind, shape, Gr, K, amp):
    print(f"case J {kind} {shape}", flush=True)
    g, X0, ctx = make(kind, shape, Gr, K, amp)
    x = S.perturbation(g.size, 1000)
    y = torch.empty(g.size, dtype=torch.float64, device="cuda")
    ctx.apply_jacobian(to_dev(x), y, project=False)
    assert_parity(g, to_host(y), O.jacobian(g, X0, x), TOL64, label="J")


@pytest.mark.parametrize("kind,shape,Gr,K,amp", GRIDS)
def test_projected_jacobian(kind, shape, Gr, K, amp):
    print(f"case PJ {kind} {shape}", flush=True)
    g, X0, ctx = make(kind, shape, Gr, K, amp)
    for r in range(2):
        x = S.perturbation(g.size, 1000 + r)
        y = torch.empty(g.size, dtype=torch.float64, device="cuda")
        ctx.apply_jacobian(to_dev(x), y, project=True)
        got = to_host(y)
        ref = O.apply_jacobian(g, X0, x)
        assert_parity(g, got, ref, TOL64, label="PJ")
        assert O.div_measure(g, got) < 1e-11


# The stencil writes the divergence that the projection starts from, partial
# on the cells whose high faces another block computes (a tile's last
# column and row, a z-chunk's last plane), which a second pass completes;
# KV_FUSED_DIV=0 selects the separate divergence pass instead.  Both against
# the oracle, and against each other element by element, on grids with x-tile
# edges (nx > 64), y-tile edges, z-chunk ends (4-plane chunks on grids this
# small) and ragged tails.
FUSED_GRIDS = [GRIDS[2], ("clustered", (130, 21, 37), 4e7, 3, 0.1), ("uniform", (65, 5, 9), 1e5, 2, 0.1)]


@pytest.mark.parametrize("kind,shape,Gr,K,amp", FUSED_GRIDS)
def test_fused_divergence_matches_separate_pass(monkeypatch, kind, shape, Gr, K, amp):
    print(f"case fused divergence {kind} {shape}", flush=True)
    g, X0, ctx = make(kind, shape, Gr, K, amp)
    x = S.perturbation(g.size, 1234)
    ref = O.apply_jacobian(g, X0, x)
    got = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("KV_FUSED_DIV", flag)
        y = torch.empty(g.size, dtype=torch.float64, device="cuda")
        ctx.apply_jacobian(to_dev(x), y, project=True)
        got[flag] = to_host(y)
        assert_parity(g, got[flag], ref, TOL64, label=f"PJ KV_FUSED_DIV={flag}")
        assert O.div_measure(g, got[flag]) < 1e-11
    for a, b in zip(g.unpack(got["1"]), g.unpack(got["0"])):
        assert np.max(np.abs(a - b)) <= 1e-13 * max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("kind,shape,Gr,K,amp", GRIDS[:3])
def test_project_and_divergence(kind, shape, Gr, K, amp):
    g, X0, ctx = make(kind, shape, Gr, K, amp)
    y0 = S.perturbation(g.size, 7)
    y = to_dev(y0)
    dm, sweeps = ctx.project(y)
    got = to_host(y)
    assert sweeps == 1
    assert_parity(g, got, O.project(g, y0), TOL64, label="P")
    assert dm < 1e-11 and abs(dm - O.div_measure(g, got)) <= 1e-3 * max(dm, 1e-300) + 1e-16


@pytest.mark.parametrize("kind,shape,Gr,K,amp", GRIDS[:3])
def test_residual(kind, shape, Gr, K, amp):
    g, X0, ctx = make(kind, shape, Gr, K, amp)
    F = torch.empty(g.size, dtype=torch.float64, device="cuda")
    norm = ctx.residual(F)
    ref = O.residual(g, X0)
    assert_parity(g, to_host(F), ref, TOL64, label="F")
    assert abs(norm - O.wnorm(g.weights(), ref)) <= 1e-12 * norm


# The split FD passes choose their tile shape and load width from the sizes
# (32 x 32 on small grids, 64 x 64 and 128 x 128 on large ones, element pairs
# when the half size and line length are even).  KV_FD_TILE and KV_FD_PAIRS
# force each variant, so the shapes used only at full size are checked here
# on small ragged grids too.
FD_VARIANTS = [("KV_FD_TILE", "64"), ("KV_FD_TILE", "32"), ("KV_FD_PAIRS", "0")]


@pytest.mark.parametrize("var,val", FD_VARIANTS)
@pytest.mark.parametrize("kind,shape,Gr,K,amp", [GRIDS[0], GRIDS[2], GRIDS[4]])
def test_projection_fd_variants(monkeypatch, var, val, kind, shape, Gr, K, amp):
    print(f"case FD variant {var}={val} {kind} {shape}", flush=True)
    monkeypatch.setenv(var, val)
    g, X0, ctx = make(kind, shape, Gr, K, amp)
    y0 = S.perturbation(g.size, 11)
    y = to_dev(y0)
    ctx.project(y)
    assert_parity(g, to_host(y), O.project(g, y0), TOL64, label=f"P {var}={val}")


# The full-size workloads: 100^3 clustered at Gr 4e7 and 256^3 clustered at
# Gr 2e8, the launch configuration the benchmark times (every output compared).
FULL = [("cube100_clustered_gr4e7", 1000), ("cube256_clustered_gr2e8", 1000)]


@pytest.mark.parametrize("workload,seed", FULL)
def test_projected_jacobian_full_size(workload, seed):
    from paper_2210_08816_amd import kv
    print(f"case PJ full {workload}", flush=True)
    spec = S.WORKLOADS[workload]
    fx = S.workload_grid(spec)
    g = O.Grid(*fx, Gr=spec["Gr"], Pr=spec["Pr"])
    X0 = S.base_flow(*fx, K=spec["K"], amp=spec["amp"], seed=spec["base_seed"])
    ctx = kv.Context(*fx, Gr=spec["Gr"], Pr=spec["Pr"])
    ctx.set_base_flow(to_dev(X0))
    x = S.perturbation(g.size, seed)
    y = torch.empty(g.size, dtype=torch.float64, device="cuda")
    ctx.apply_jacobian(to_dev(x), y, project=True)
    got = to_host(y)
    del y
    ref = O.apply_jacobian(g, X0, x)
    assert_parity(g, got, ref, TOL64, label=f"PJ {workload}")


def test_axpby():
    from paper_2210_08816_amd import kv
    g, X0, ctx = make("clustered", (9, 7, 8), 1e5, 2, 0.1)
    a = S.perturbation(g.size, 3)
    b = S.perturbation(g.size, 4)
    y = to_dev(b)
    ctx.axpby(2.5, to_dev(a), -0.75, y)
    assert np.allclose(to_host(y), 2.5 * a - 0.75 * b, rtol=1e-15, atol=1e-15)
    with pytest.raises(kv.KVError):
        ctx.axpby(float("nan"), y, 1.0, y)


def test_weighted_dot_and_symmetry():
    g, X0, ctx = make("clustered", (33, 20, 17), 1e6, 3, 0.1)
    a = S.perturbation(g.size, 1)
    b = S.perturbation(g.size, 2)
    w = g.weights()
    assert abs(ctx.dot(to_dev(a), to_dev(b)) - O.wdot(w, a, b)) <= 1e-12 * O.wnorm(w, a) * O.wnorm(w, b)
    X = X0 + 0.01 * a
    got = ctx.symmetry_measures(to_dev(X))
    ref = O.symmetry_measures(g, X)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-15)


def test_error_codes():
    from paper_2210_08816_amd import kv
    f = S.faces_uniform(8)
    ctx = kv.Context(f, f, f, Gr=1e5, Pr=0.71)
    x = torch.zeros(ctx.n, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(kv.KVError) as e:
        ctx.apply_jacobian(x, y)
    assert e.value.code == kv.KV_ESTATE
    bad = x.clone()
    bad[5] = float("nan")
    with pytest.raises(kv.KVError) as e:
        ctx.set_base_flow(bad)
    assert e.value.code == kv.KV_ENONFINITE
    with pytest.raises(kv.KVError) as e:
        kv.Context(f[::-1].copy(), f, f, Gr=1e5, Pr=0.71)
    assert e.value.code == kv.KV_EINVAL


# ---- mixed form: fast diagonalization in FP32 storage (bf16x3 split products on
# the bf16 matrix cores, or FP32 ones) refined on the FP64 residual ---------
MIXED_GRIDS = [
    ("uniform", (32, 32, 32), 1e5, 3, 0.05),
    ("clustered", (24, 18, 20), 4e7, 4, 0.1),
    ("clustered", (64, 64, 64), 2e8, 6, 0.1),
    ("clustered", (36, 20, 44), 4e7, 3, 0.1),     # FP32 pair loads with ragged FD tiles
]
TOL_MIXED = 1e-5


@pytest.mark.parametrize("kind,shape,Gr,K,amp", MIXED_GRIDS)
def test_mixed_projected_jacobian(kind, shape, Gr, K, amp):
    print(f"case mixed PJ {kind} {shape}", flush=True)
    g, X0, ctx = make(kind, shape, Gr, K, amp)
    x = S.perturbation(g.size, 1000)
    y = torch.empty(g.size, dtype=torch.float64, device="cuda")
    ctx.apply_jacobian(to_dev(x), y, project=True, mixed=True)
    got = to_host(y)
    ref = O.apply_jacobian(g, X0, x)
    assert_parity(g, got, ref, TOL_MIXED, label="mixed PJ")
    assert O.div_measure(g, got) <= 1e-10


@pytest.mark.parametrize("var,val", FD_VARIANTS)
def test_mixed_fd_variants(monkeypatch, var, val):
    kind, shape, Gr, K, amp = MIXED_GRIDS[3]
    print(f"case mixed FD variant {var}={val} {kind} {shape}", flush=True)
    monkeypatch.setenv(var, val)
    g, X0, ctx = make(kind, shape, Gr, K, amp)
    x = S.perturbation(g.size, 1000)
    y = torch.empty(g.size, dtype=torch.float64, device="cuda")
    ctx.apply_jacobian(to_dev(x), y, project=True, mixed=True)
    got = to_host(y)
    assert_parity(g, got, O.apply_jacobian(g, X0, x), TOL_MIXED, label=f"mixed {var}={val}")
    assert O.div_measure(g, got) <= 1e-10


@pytest.mark.parametrize("kind,shape,Gr,K,amp", MIXED_GRIDS[:2])
def test_mixed_project_reports_sweeps(kind, shape, Gr, K, amp):
    g, X0, ctx = make(kind, shape, Gr, K, amp)
    y0 = S.perturbation(g.size, 8)
    y = to_dev(y0)
    dm, sweeps = ctx.project(y, mixed=True)
    print(f"mixed sweeps {sweeps} div {dm:.3e}", flush=True)
    assert 2 <= sweeps <= 8      # checked after every sweep from the second
    assert dm <= 1e-10
    assert_parity(g, to_host(y), O.project(g, y0), TOL_MIXED, label="mixed P")


def test_mixed_falls_back_on_unsplit_grid():
    """Odd cell counts have no even/odd split: the FP64 projection runs."""
    g, X0, ctx = make("clustered", (7, 6, 5), 2e5, 2, 0.1)
    y0 = S.perturbation(g.size, 9)
    y = to_dev(y0)
    dm, sweeps = ctx.project(y, mixed=True)
    assert sweeps == 1
    assert_parity(g, to_host(y), O.project(g, y0), TOL64, label="P unsplit")


@pytest.mark.parametrize("fd", ["bf16x3", "fp32"])
def test_mixed_odd_and_even_sweep_counts(monkeypatch, fd):
    """Both transform precisions of the mixed sweeps, on a grid where their
    sweep counts differ: an odd count ends with the copy of the velocity
    back into y; either way the result meets the mixed bar against the
    oracle and the normalized divergence bar."""
    monkeypatch.setenv("KV_MIXED_FD", fd)
    kind, shape, Gr, K, amp = MIXED_GRIDS[1]
    g, X0, ctx = make(kind, shape, Gr, K, amp)
    for seed in (8, 9):
        y0 = S.perturbation(g.size, seed)
        y = to_dev(y0)
        dm, sweeps = ctx.project(y, mixed=True)
        print(f"{fd}: sweeps {sweeps} div {dm:.3e}", flush=True)
        assert 2 <= sweeps <= 8 and dm <= 1e-10
        assert_parity(g, to_host(y), O.project(g, y0), TOL_MIXED, label=f"mixed P {fd} sweeps {sweeps}")

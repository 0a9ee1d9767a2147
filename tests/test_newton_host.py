"""Host logic around the library, with stand-in contexts on the CPU.

The Newton iteration (continuation.newton_solve): the residual F(X) = X - X*, and corrections
that solve J d = -F only partly, reported as out of budget (KV_ENOCONV) with
a given relative residual.  A partial correction that halves the linearized
residual is taken as an inexact Newton step; one that does not ends the
iteration.

The growth check (growth.measure) against a flow that advances the
perturbation exactly as exp(lambda t)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2210_08816_amd import continuation as C  # noqa: E402
from paper_2210_08816_amd.kv import KV_ENOCONV, KV_OK  # noqa: E402


class FakeContext:
    def __init__(self, target, relres, status):
        self.target, self.relres, self.status = target, relres, status
        self.X = None

    def set_base_flow(self, X):
        self.X = X.clone()

    def residual(self, F):
        F.copy_(self.X - self.target)
        return float(torch.linalg.vector_norm(F))

    def newton_correction(self, F, d, tol, max_matvec, delta0=None, check=False, sym=None):
        d.copy_(-(1.0 - self.relres) * F)    # leaves relres of the linear residual
        return {"status": self.status, "relres": self.relres, "matvecs": 10, "used_gmres": 1}

    def axpby(self, a, x, b, y):
        y.mul_(b).add_(a * x)


@pytest.fixture(autouse=True)
def no_device_sync(monkeypatch):
    monkeypatch.setattr(torch.cuda, "synchronize", lambda: None)


def test_budget_limited_correction_that_halves_the_residual_is_taken():
    target = torch.arange(8, dtype=torch.float64)
    X = torch.zeros(8, dtype=torch.float64)
    ctx = FakeContext(target, relres=0.1, status=KV_ENOCONV)
    out = C.newton_solve(ctx, X, tol_rel=1e-8, tol_abs=0.0, max_iter=30)
    assert out["converged"]
    h = np.array(out["hist"])
    assert np.allclose(h[1:] / h[:-1], 0.1)       # each inexact step keeps relres of the residual
    assert torch.allclose(X, target, rtol=0, atol=1e-6)


def test_correction_that_does_not_halve_the_residual_stops_newton():
    target = torch.arange(8, dtype=torch.float64)
    X = torch.zeros(8, dtype=torch.float64)
    ctx = FakeContext(target, relres=0.7, status=KV_ENOCONV)
    out = C.newton_solve(ctx, X, tol_rel=1e-8, tol_abs=0.0, max_iter=30)
    assert not out["converged"] and out["iters"] == 0
    assert torch.equal(X, torch.zeros(8, dtype=torch.float64))   # the rejected step is not applied


def test_converged_corrections_reach_the_target():
    target = torch.arange(8, dtype=torch.float64)
    X = torch.zeros(8, dtype=torch.float64)
    ctx = FakeContext(target, relres=1e-3, status=KV_OK)
    out = C.newton_solve(ctx, X, tol_rel=1e-10, tol_abs=0.0, max_iter=30)
    assert out["converged"] and out["iters"] == 4


class LinearFlow:
    """Stand-in context whose time steps advance the perturbation from X
    exactly as exp(A t) for a 2 x 2 block A with eigenvalues a +- i b."""

    def __init__(self, X, a, b):
        self.X, self.a, self.b = X, a, b

    def axpby(self, a, x, b, y):
        y.mul_(b).add_(a * x)

    def dot(self, x, y):
        return float(torch.dot(x, y))

    def time_steps(self, Y, Yp, dt, n, start=True):
        import math
        d = Y - self.X
        t = dt * n
        c, s = math.cos(self.b * t), math.sin(self.b * t)
        e = math.exp(self.a * t)
        d2 = d.clone()
        d2[0] = e * (c * d[0] - s * d[1])
        d2[1] = e * (s * d[0] + c * d[1])
        Yp.copy_(Y)
        Y.copy_(self.X + d2)


@pytest.mark.parametrize("a", [0.0069, -0.02])
def test_growth_measure_on_an_exact_linear_flow(a):
    """growth.measure against a flow that is exactly exp(lambda t) on the
    perturbation: the growth over a period is exp(Re lambda T), the rate is
    Re lambda, and half a period flips the sign."""
    import math
    from paper_2210_08816_amd import growth
    b = 0.0306
    X = torch.tensor([0.3, -0.2, 0.5], dtype=torch.float64)
    v = torch.tensor([1.0, 0.0, 0.0], dtype=torch.float64)
    out = growth.measure(LinearFlow(X, a, b), X, v, complex(a, b), 1000, eps=1e-3, log=lambda m: None, chunk=300)
    T = 2 * math.pi / b
    assert out["growth_over_period"] == pytest.approx(math.exp(a * T), rel=1e-12)
    assert out["rate_measured"] == pytest.approx(a, rel=1e-10)
    assert out["projection_half_period"] == pytest.approx(-math.exp(a * T / 2), rel=1e-12)

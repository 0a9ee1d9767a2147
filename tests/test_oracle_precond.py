"""Pins of the Stokes/heat preconditioner oracle (oracle/precond.py): the
eigen route inverts the discretization's own diffusion operators (checked
by applying those operators from oracle/disc.py), the result is
divergence-free, and each Helmholtz inverse is self-adjoint in the volume
inner product."""
import numpy as np
import pytest

from oracle import disc as O
from oracle import precond as PC
from synth import inputs as S

GRIDS = [("clustered", (7, 6, 5), 1e6), ("uniform", (8, 8, 8), 2e4), ("clustered", (5, 9, 4), 0.0)]


def grid(kind, shape, Gr):
    f = [S.faces_uniform(n) if kind == "uniform" else S.faces_clustered(n) for n in shape]
    return f, O.Grid(*f, Gr=Gr, Pr=0.71)


@pytest.mark.parametrize("kind,shape,Gr", GRIDS)
@pytest.mark.parametrize("sigma", [0.0, 3.5])
def test_helmholtz_inverts_the_discrete_diffusion(kind, shape, Gr, sigma):
    f, g = grid(kind, shape, Gr)
    g0 = O.Grid(*f, Gr=0.0, Pr=0.71)           # nu = 1, kappa = 1/Pr, no buoyancy
    r = S.perturbation(g.size, 3)
    blocks = g.unpack(r)
    z = g.pack([PC.helmholtz_solve(g, b, blocks[b], sigma, g.nu if b < 3 else g.kappa) for b in range(4)])
    lap = g0.unpack(O.jacobian(g0, np.zeros(g.size), z))   # J at rest: pure diffusion
    zb = g.unpack(z)
    for b in range(4):
        coef = g.nu if b < 3 else g.kappa * 0.71        # Lap_T = Pr * (J0)_T
        back = sigma * zb[b] - coef * lap[b]
        assert np.allclose(back, blocks[b], rtol=0, atol=1e-9 * np.abs(blocks[b]).max()), b


@pytest.mark.parametrize("kind,shape,Gr", GRIDS[:2])
def test_preconditioner_output_is_divergence_free_and_projected(kind, shape, Gr):
    f, g = grid(kind, shape, Gr)
    y = PC.apply(g, S.perturbation(g.size, 4), 0.5)
    assert O.div_measure(g, y) < 1e-12
    assert np.allclose(O.project(g, y), y, rtol=0, atol=1e-13 * np.abs(y).max())


@pytest.mark.parametrize("block", [0, 1, 2, 3])
def test_helmholtz_inverse_is_self_adjoint(block):
    f, g = grid("clustered", (6, 7, 5), 1e5)
    w = g.unpack(g.weights())[block]
    rng = np.random.default_rng(block)
    a = rng.standard_normal(w.shape)
    b = rng.standard_normal(w.shape)
    za = PC.helmholtz_solve(g, block, a, 1.0, 0.3)
    zb = PC.helmholtz_solve(g, block, b, 1.0, 0.3)
    lhs, rhs = np.sum(w * a * zb), np.sum(w * za * b)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_one_dimensional_operators_closed_form_on_a_uniform_grid():
    """Uniform h: the face-Dirichlet operator is the n-1 point Dirichlet
    Laplacian, eigenvalues (4/h^2) sin^2(k pi / (2n)); the centre-Dirichlet
    one has (4/h^2) sin^2(k pi / (2n)), k = 1..n (the staggered Dirichlet
    spectrum)."""
    n = 10
    f = S.faces_uniform(n)
    g = O.Grid(f, f, f, Gr=1e4, Pr=0.71)
    h = 1.0 / n
    K, H = PC.stiffness_1d(g, 0, "fD")
    ev = np.sort(np.linalg.eigvalsh(K / H[:, None]))
    k = np.arange(1, n)
    assert np.allclose(ev, np.sort(4 / h ** 2 * np.sin(k * np.pi / (2 * n)) ** 2), rtol=1e-12)
    K, H = PC.stiffness_1d(g, 0, "cD")
    ev = np.sort(np.linalg.eigvalsh(K / H[:, None]))
    k = np.arange(1, n + 1)
    assert np.allclose(ev, np.sort(4 / h ** 2 * np.sin(k * np.pi / (2 * n)) ** 2), rtol=1e-12)
    K, H = PC.stiffness_1d(g, 0, "cN")
    ev = np.sort(np.linalg.eigvalsh(K / H[:, None]))
    k = np.arange(0, n)
    assert np.allclose(ev, np.sort(4 / h ** 2 * np.sin(k * np.pi / (2 * n)) ** 2), rtol=1e-10, atol=1e-9)

"""Pins of the oracle's time stepper (oracle/timestep.py): closed-form decay
of a temperature eigenmode at Gr = 0, second-order convergence in dt on a
nonlinear flow, and steady states as fixed points."""
import numpy as np

from oracle import disc as O
from oracle import solvers as SV
from oracle import timestep as TS
from synth import inputs as S


def test_temperature_mode_follows_the_closed_form_recurrence():
    """Gr = 0 (viscous scaling, no buoyancy) on a uniform grid: T' = a psi
    with psi an eigenvector of the discrete T Laplacian (sine in x between the
    Dirichlet walls, cosine along the adiabatic y and z) stays on psi, and its
    amplitude follows the scheme's scalar recurrence with mu = kappa lambda:
    a1 = a0 / (1 - dt mu), then a_{n+1} = (4 a_n - a_{n-1}) / (3 - 2 dt mu);
    that recurrence tends to exp(mu t) at second order."""
    nx, ny, nz = 8, 6, 5
    f = [S.faces_uniform(k) for k in (nx, ny, nz)]
    g = O.Grid(*f, Gr=0.0, Pr=0.71)
    Xc = S.conduction_state(*f)
    mx, my, mz = 2, 1, 3
    cx = (np.arange(nx) + 0.5) / nx
    cy = (np.arange(ny) + 0.5) / ny
    cz = (np.arange(nz) + 0.5) / nz
    psi = np.sin(mx * np.pi * cx)[None, None, :] * np.cos(my * np.pi * cy)[None, :, None] * \
        np.cos(mz * np.pi * cz)[:, None, None]
    lam = sum(-(4.0 * n * n) * np.sin(m * np.pi / (2 * n)) ** 2 for m, n in ((mx, nx), (my, ny), (mz, nz)))
    mu = g.kappa * lam
    d = np.zeros(g.size)
    d[g.size - g.ncell:] = psi.ravel()
    # psi is an eigenvector of the discretization's T diffusion
    assert np.allclose(TS.homogeneous_diffusion(g, d), mu * d, rtol=0, atol=1e-12 * abs(mu))
    a0, dt, n = 1e-3, 0.02, 12
    X, Xm = TS.integrate(g, Xc + a0 * d, dt, n)
    a = [a0, a0 / (1.0 - dt * mu)]
    for _ in range(n - 1):
        a.append((4.0 * a[-1] - a[-2]) / (3.0 - 2.0 * dt * mu))
    assert np.allclose(X, Xc + a[-1] * d, rtol=0, atol=1e-14)
    assert np.allclose(Xm, Xc + a[-2] * d, rtol=0, atol=1e-14)
    # the recurrence itself: second order towards exp(mu t) (t = 0.24)
    errs = []
    for k in range(3):
        h = dt / 2 ** k
        b = [a0, a0 / (1.0 - h * mu)]
        for _ in range(n * 2 ** k - 1):
            b.append((4.0 * b[-1] - b[-2]) / (3.0 - 2.0 * h * mu))
        errs.append(abs(b[-1] - a0 * np.exp(mu * n * dt)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.7


def test_second_order_in_dt_on_a_nonlinear_flow():
    """Errors at t = 0.4 against a fine-dt solution fall about 4x per halving
    of dt (a wrong extrapolation coefficient gives first order or blows up)."""
    f = [S.faces_clustered(k) for k in (8, 6, 6)]
    g = O.Grid(*f, Gr=2e4, Pr=0.71)
    X0 = O.project(g, S.base_flow(*f, K=2, amp=0.2, seed=51))
    t_end = 0.4
    ref, _ = TS.integrate(g, X0, t_end / 320, 320)
    w = g.weights()
    errs = []
    for nsteps in (20, 40, 80):
        X, _ = TS.integrate(g, X0, t_end / nsteps, nsteps)
        errs.append(O.wnorm(w, X - ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.8 and 3.6 < r2 < 4.5, errs
    # the solution moved, and stays divergence free
    assert O.wnorm(w, ref - X0) > 1e2 * errs[-1]
    assert O.div_measure(g, ref) < 1e-12


def test_steady_state_is_a_fixed_point():
    f = S.faces_uniform(8)
    g = O.Grid(f, f, f, Gr=1e4, Pr=0.71)
    Xs, hist, _ = SV.newton(g, S.conduction_state(f, f, f), rtol=1e-13, max_iter=12)
    X, Xm = TS.integrate(g, Xs, 0.05, 10)
    assert O.wnorm(g.weights(), X - Xs) <= 1e-11 * O.wnorm(g.weights(), Xs)

"""Pins of the oracle's Krylov solvers.

The solvers are checked against results fixed independently of them:
dense generalized eigenproblems and dense saddle-point solves of the
discrete equations (no projection, no fast diagonalization involved), the
closed-form spectrum of the Gr = 0 conduction state, and Newton's quadratic
convergence to a state with the cube's symmetries (paper Sec. 2, Eqs. 7-9:
symmetry measures of symmetric solutions at round-off level).
"""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import disc as O
from oracle import solvers as SV
from synth import inputs as S


def dense(fn, nin):
    cols = []
    for i in range(nin):
        e = np.zeros(nin)
        e[i] = 1.0
        cols.append(np.ravel(fn(e)))
    return np.array(cols).T


def saddle(g, X0):
    """Dense J, D, G of the discrete equations (no projection involved)."""
    J = dense(lambda v: O.jacobian(g, X0, v), g.size)
    D = dense(lambda v: O.divergence(g, v), g.size)
    G = dense(lambda p: O.gradient(g, p.reshape(g.shapes[3])), g.ncell)
    return J, D, G


def generalized_eigs(g, X0):
    """Finite eigenvalues of [J -G; D 0] z = lam [I 0; 0 0] z.  The constant
    pressure mode is removed (one pressure unknown and the redundant last
    divergence row dropped) so that the pencil is regular."""
    J, D, G = saddle(g, X0)
    D, G = D[:-1], G[:, :-1]
    n, C = g.size, g.ncell - 1
    A = np.block([[J, -G], [D, np.zeros((C, C))]])
    B = np.zeros_like(A)
    B[:n, :n] = np.eye(n)
    lam = sl.eig(A, B, right=False)
    lam = lam[np.isfinite(lam)]
    return lam[np.argsort(-lam.real, kind="stable")]


def closest_match(a, b):
    """max over a of the distance to the nearest element of b."""
    return max(np.min(np.abs(b - x)) for x in a)


def test_gr0_leading_eigenvalues_closed_form():
    """Gr = 0 (viscous scaling, beta = 0) conduction state: J is block
    triangular, so its leading eigenvalues are those of kappa Lap_T:
    kappa * sum_a -(4/h_a^2) sin^2(m_a pi / 2N_a), sine modes (m = 1..N) in
    the Dirichlet x-direction, cosine modes (m = 0..N-1) in y and z.  With
    Pr = 10 the first several T-modes lie far ahead of the Stokes modes."""
    nx, ny, nz = 7, 6, 5
    f = [S.faces_uniform(k) for k in (nx, ny, nz)]
    g = O.Grid(*f, Gr=0.0, Pr=10.0)
    X0 = S.conduction_state(*f)
    lx = -(4.0 * nx * nx) * np.sin(np.arange(1, nx + 1) * np.pi / (2 * nx)) ** 2
    ly = -(4.0 * ny * ny) * np.sin(np.arange(ny) * np.pi / (2 * ny)) ** 2
    lz = -(4.0 * nz * nz) * np.sin(np.arange(nz) * np.pi / (2 * nz)) ** 2
    closed = np.sort((lx[:, None, None] + ly[None, :, None] + lz[None, None, :]).ravel() * g.kappa)[::-1]
    lam = generalized_eigs(g, X0)
    assert np.max(np.abs(lam[:8].imag)) < 1e-9
    assert np.allclose(lam[:8].real, closed[:8], rtol=1e-9)
    # the projected-operator eigen-solver finds the same values
    A = SV.Operator(g, X0)
    vals, res, _, info = SV.cheb_arnoldi(A, S.perturbation(g.size, 77), m=30, n_eigs=4,
                                         tol=1e-10, cheb_degree_max=300)
    assert info["converged"]
    assert np.allclose(np.sort(vals.real)[::-1][:4], closed[:4], rtol=1e-8)


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_cheb_arnoldi_matches_dense_saddle_eigs(kind):
    """Leading eigenvalues of P J on divergence-free vectors = leading finite
    eigenvalues of the generalized saddle problem (no shift-and-invert)."""
    fx = S.faces_uniform if kind == "uniform" else S.faces_clustered
    f = [fx(6), fx(5), fx(4)]
    g = O.Grid(*f, Gr=2e4, Pr=0.71)
    X0 = S.base_flow(*f, K=2, amp=0.3, seed=21)
    lam = generalized_eigs(g, X0)
    A = SV.Operator(g, X0)
    vals, res, Y, info = SV.cheb_arnoldi(A, S.perturbation(g.size, 77), m=40, n_eigs=4,
                                         tol=1e-11, cheb_degree_max=300)
    assert info["converged"]
    scale = np.max(np.abs(lam[:4]))
    assert closest_match(vals, lam[:6]) < 1e-8 * scale
    # a-posteriori: the returned Ritz vectors are eigenvectors of A
    for i in range(len(vals)):
        y = Y[i]
        if abs(vals[i].imag) > 0:
            r = A(y.real) + 1j * A(y.imag) - vals[i] * y
            rn = np.sqrt(A.norm(r.real) ** 2 + A.norm(r.imag) ** 2)
            yn = np.sqrt(A.norm(y.real) ** 2 + A.norm(y.imag) ** 2)
        else:
            rn, yn = A.norm(A(y.real) - vals[i].real * y.real), A.norm(y.real)
        assert rn <= 1e-8 * scale * yn


def test_single_cycle_ritz_values_match_dense_krylov():
    """Ritz values of K_m(A, v0) do not depend on the orthogonalization:
    compare CGS2 Arnoldi with a dense W-orthonormal Krylov basis."""
    f = [S.faces_uniform(6), S.faces_uniform(5), S.faces_uniform(4)]
    g = O.Grid(*f, Gr=1e5, Pr=0.71)
    X0 = S.base_flow(*f, K=2, amp=0.05, seed=22)
    A = SV.Operator(g, X0)
    v0 = O.project(g, S.perturbation(g.size, 77))
    m = 8
    vals, _ = SV.arnoldi_ritz(A, v0, m, n_eigs=m)
    # dense route: power basis, W-orthonormalized by QR with weights
    K = [v0 / A.norm(v0)]
    for _ in range(m - 1):
        k = A(K[-1])
        K.append(k / A.norm(k))
    K = np.array(K).T
    sw = np.sqrt(A.w)[:, None]
    Qw, _ = np.linalg.qr(sw * K)
    Q = Qw / sw
    AQ = np.array([A(Q[:, i]) for i in range(m)]).T
    Hm = Qw.T @ (sw * AQ)
    ref = np.linalg.eigvals(Hm)
    assert closest_match(vals, ref) < 1e-7 * np.max(np.abs(ref))


@pytest.mark.parametrize("solver", ["bicgstab2", "gmres"])
def test_linear_solvers_match_dense_saddle_solve(solver):
    """delta with P J delta = -F equals the velocity part of the dense
    saddle solve J delta - G q = -N, D delta = 0."""
    f = [S.faces_clustered(6), S.faces_clustered(5), S.faces_clustered(4)]
    g = O.Grid(*f, Gr=1e4, Pr=0.71)
    X0 = O.project(g, S.base_flow(*f, K=2, amp=0.1, seed=23) + 0.01 * S.perturbation(g.size, 24))
    J, D, G = saddle(g, X0)
    N = O.nonlinear(g, X0)
    n, C = g.size, g.ncell
    M = np.block([[J, -G], [D, np.zeros((C, C))]])
    rhs = np.concatenate([-N, np.zeros(C)])
    z = np.linalg.lstsq(M, rhs, rcond=None)[0]
    delta_ref = z[:n]
    A = SV.Operator(g, X0)
    F = SV.A_project(A, O.residual(g, X0))      # as the Newton correction does
    if solver == "bicgstab2":
        delta, info = SV.bicgstab2(A, -F, tol=1e-12, max_matvec=4000)
    else:
        delta, info = SV.gmres(A, -F, tol=1e-11, m=100, max_matvec=4000)
    assert info["status"] == "converged"
    assert np.linalg.norm(delta - delta_ref) <= 1e-8 * np.linalg.norm(delta_ref)


def test_newton_quadratic_convergence_and_symmetry():
    """Newton from the conduction state (Gr = 1e4, 16^3): quadratic
    convergence, and the steady state keeps all three symmetries of the
    cube to round-off (the paper reports ~1e-9 for symmetric solutions)."""
    f = S.faces_uniform(16)
    g = O.Grid(f, f, f, Gr=1e4, Pr=0.71)
    X, hist, mv = SV.newton(g, S.conduction_state(f, f, f), rtol=1e-11, max_iter=12)
    assert hist[-1] <= 1e-11 * hist[0]
    # once in the quadratic regime, ||F_{k+1}|| <= C ||F_k||^2
    k = next(i for i, r in enumerate(hist) if r < 1e-3)
    assert hist[k + 1] <= 10.0 * hist[k] ** 2
    assert max(O.symmetry_measures(g, X)) < 1e-9
    assert O.div_measure(g, X) < 1e-11


@pytest.mark.parametrize("with_delta0", [False, True])
def test_forced_gmres_handover_matches_dense_saddle_solve(with_delta0):
    """A stagnation limit of 0 cycles hands the Newton correction to GMRES
    before the first BiCGstab(2) cycle (Sec. 1: BiCGstab(2) combined with
    GMRES).  The continuation must still reach the unique correction of the
    dense saddle system J delta - G q = -N, D delta = 0 (no projection and no
    fast diagonalization involved), also from a nonzero initial iterate."""
    f = [S.faces_clustered(6), S.faces_clustered(5), S.faces_clustered(4)]
    g = O.Grid(*f, Gr=1e4, Pr=0.71)
    X0 = O.project(g, S.base_flow(*f, K=2, amp=0.1, seed=25) + 0.01 * S.perturbation(g.size, 26))
    J, D, G = saddle(g, X0)
    n, C = g.size, g.ncell
    M = np.block([[J, -G], [D, np.zeros((C, C))]])
    rhs = np.concatenate([-O.nonlinear(g, X0), np.zeros(C)])
    delta_ref = np.linalg.lstsq(M, rhs, rcond=None)[0][:n]
    A = SV.Operator(g, X0)
    d0 = O.project(g, S.perturbation(g.size, 27)) * 1e-3 if with_delta0 else None
    d, info = SV.newton_correction(A, O.residual(g, X0), tol=1e-11, max_matvec=4000, delta0=d0,
                                   stall_cycles=0, gmres_m=100)
    assert info["used_gmres"] == 1 and info["cycles"] >= 1
    assert info["status"] == "converged"
    assert np.linalg.norm(d - delta_ref) <= 1e-8 * np.linalg.norm(delta_ref)
    # the default limit keeps BiCGstab(2) on this easy system
    d2, info2 = SV.newton_correction(A, O.residual(g, X0), tol=1e-11, max_matvec=4000, delta0=d0)
    assert info2["used_gmres"] == 0 and info2["status"] == "converged"
    assert np.linalg.norm(d2 - delta_ref) <= 1e-8 * np.linalg.norm(delta_ref)


def test_chebyshev_growth_rate_and_restart_weights():
    """growth_rate is the per-degree growth of the filter polynomial: on a
    scalar operator the filter's value at two points outside the ellipse
    approaches (rate_1 / rate_2)^degree (real and complex points, b < a and
    b > a).  The restart weights undo that growth."""
    class Scalar:
        def __init__(self, lam):
            self.lam = lam

        def __call__(self, v):
            return self.lam * v

    for a, b in ((1.0, 0.5), (1.0, 2.0)):
        c2 = a * a - b * b
        for lam in (3.0, 1.5 + 2.5j, -4.0):
            deg = 200
            wr = 2.0 * a + 0.5
            p = SV.cheb_filter(Scalar(lam), np.array([1.0 + 0j]), 0.0, c2, wr, deg)[0]
            # the filter is normalized to 1 at wr
            est = deg * np.log(SV.growth_rate(lam, a, b, c2) / SV.growth_rate(wr, a, b, c2))
            assert abs(np.log(abs(p)) - est) < 1.5, (a, b, lam, np.log(abs(p)), est)
    # restart weights: filtering the weighted wanted components of a diagonal
    # operator leaves them of comparable size (within the same constant)
    lam = np.array([8.0, 3.0, 1.5 + 2.5j, 1.5 - 2.5j])
    a, b = 1.0, 0.5
    c2 = a * a - b * b
    wr, deg = 2.5, 150
    wts = SV.restart_weights(lam, 0.0, a, b, c2, wr, deg)
    assert wts.max() == 1.0 and wts[0] < 1e-40
    out = SV.cheb_filter(Scalar(lam), wts.astype(complex), 0.0, c2, wr, deg)
    assert np.max(np.abs(np.log(np.abs(out) / np.abs(out[1])))) < 3.0, out
    assert np.array_equal(SV.restart_weights(lam, 0.0, a, b, c2, wr, 0), np.ones(4))


class ClassOperator(SV.Operator):
    """P J restricted to a symmetry class: the class projection after P J."""

    def __init__(self, g, X0, cls):
        super().__init__(g, X0)
        self.cls = cls

    def __call__(self, x):
        return O.symmetry_project(self.g, super().__call__(x), *self.cls)


def test_locked_cheb_arnoldi_in_a_symmetry_class():
    """At a symmetric base flow, Arnoldi on one symmetry class returns the
    leading eigenvalues of the saddle problem whose eigenvectors lie in that
    class.  Here the leading pair converges cycles before the next one and is
    locked, and the returned vectors are eigenvectors of A."""
    f = [S.faces_clustered(n) for n in (5, 7, 5)]
    g = O.Grid(*f, Gr=2e4, Pr=0.71)
    X0 = O.symmetry_project(g, S.base_flow(*f, K=2, amp=0.3, seed=21), 1, 1)
    J, D, G = saddle(g, X0)
    D, G = D[:-1], G[:, :-1]
    n, C = g.size, g.ncell - 1
    lam, vec = sl.eig(np.block([[J, -G], [D, np.zeros((C, C))]]),
                      np.block([[np.eye(n), np.zeros((n, C))], [np.zeros((C, n + C))]]))
    cls = (-1, 1)
    keep = [q for q in range(len(lam)) if np.isfinite(lam[q]) and np.linalg.norm(
        O.symmetry_project(g, vec[:n, q].real, *cls) + 1j * O.symmetry_project(g, vec[:n, q].imag, *cls)
        - vec[:n, q]) <= 1e-6 * np.linalg.norm(vec[:n, q])]
    ref = lam[keep][np.argsort(-lam[keep].real, kind="stable")]
    A = ClassOperator(g, X0, cls)
    vals, res, Y, info = SV.cheb_arnoldi(A, O.symmetry_project(g, S.perturbation(g.size, 77), *cls), m=30,
                                         n_eigs=4, tol=1e-11, max_matvec=20000, cheb_degree_max=300)
    assert info["converged"] and info["locked"] >= 2, info
    scale = np.max(np.abs(ref[:4]))
    assert closest_match(vals, ref[:6]) < 1e-8 * scale
    assert closest_match(ref[:4], vals) < 1e-8 * scale
    for i in range(len(vals)):
        y = Y[i]
        r = A(y.real) + 1j * A(y.imag) - vals[i] * y
        assert np.sqrt(A.norm(r.real) ** 2 + A.norm(r.imag) ** 2) <= 1e-8 * scale * np.sqrt(
            A.norm(y.real) ** 2 + A.norm(y.imag) ** 2)


def test_lift_from_deflated_operator():
    """lift(): with Q an orthonormal basis of an invariant subspace of M (its
    leading real Schur vectors), every eigenvector y of the deflated operator
    (I - Q Q^T) M on the complement of span(Q) lifts to an eigenvector of M
    with the same eigenvalue; the Deflated operator has the remaining
    eigenvalues of M (and 0 on span(Q))."""
    class Dense:
        def __init__(self, M):
            self.M, self.w, self.matvecs = M, np.ones(M.shape[0]), 0
            self.g = self.fd = None

        def __call__(self, x):
            self.matvecs += 1
            return self.M @ x

        def dot(self, a, b):
            return float(np.dot(a, b))

        def norm(self, a):
            return float(np.sqrt(np.dot(a, a)))

    rng = np.random.default_rng(3)
    n, k = 12, 4
    M = rng.standard_normal((n, n))
    T, Z = sl.schur(M, output="real")
    if abs(T[k, k - 1]) > 0:          # do not split a 2x2 block
        k += 1
    Q = Z[:, :k].T                     # rows: W-orthonormal (W = I) basis
    A = Dense(M)
    B = SV.Deflated(A, Q)
    Bm = np.array([B(e) for e in np.eye(n)]).T
    A.matvecs = 0
    lamB, vecB = np.linalg.eig(Bm)
    lamM = np.linalg.eigvals(M)
    for lam, y in zip(lamB, vecB.T):
        if abs(lam) < 1e-10:
            continue                   # span(Q) itself
        assert np.min(np.abs(lamM - lam)) < 1e-10
        x = SV.lift(A, Q, y, lam)
        assert np.linalg.norm(M @ x - lam * x) <= 1e-10 * np.linalg.norm(x)
    assert A.matvecs == 0              # lift does not count matvecs

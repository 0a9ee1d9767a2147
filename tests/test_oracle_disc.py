"""Pins of the oracle's discretization against facts fixed by the mathematics.

Each test checks the oracle against something other than itself: closed
forms, exact polynomial/trigonometric consistency, conservation, the three
symmetries of the cube (paper Sec. 2), adjointness, and brute-force dense
solves on tiny grids.  A plausible mistake (dropped term, wrong sign, wrong
index or metric) breaks at least one of these.
"""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import disc as O
from synth import inputs as S


def grid(nx, ny, nz, kind="uniform", Gr=1e5, Pr=0.71):
    fx = S.faces_uniform if kind == "uniform" else S.faces_clustered
    return O.Grid(fx(nx), fx(ny), fx(nz), Gr, Pr)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ---- manufactured smooth fields ------------------------------------------------
# Separable trigonometric fields with analytic derivatives.  Velocity
# components are sine products (zero on every wall, odd about each wall);
# T = 1/2 - x + sin(pi x) cos(pi y) cos(2 pi z) meets Eqs. 4-6.
PI = np.pi


def _f(kind, k, t):
    """value, first and second derivative of one 1-D factor."""
    if kind == "s":
        return np.sin(k * PI * t), k * PI * np.cos(k * PI * t), -(k * PI) ** 2 * np.sin(k * PI * t)
    if kind == "c":
        return np.cos(k * PI * t), -k * PI * np.sin(k * PI * t), -(k * PI) ** 2 * np.cos(k * PI * t)
    raise ValueError(kind)


def sep(terms, x, y, z):
    """sum of coef * f(x) g(y) h(z): returns value, gradient (3), Laplacian."""
    val = 0.0
    grad = [0.0, 0.0, 0.0]
    lap = 0.0
    for coef, fs in terms:
        (a0, a1, a2), (b0, b1, b2), (c0, c1, c2) = (_f(kd, k, t) for (kd, k), t in zip(fs, (x, y, z)))
        val = val + coef * a0 * b0 * c0
        grad[0] = grad[0] + coef * a1 * b0 * c0
        grad[1] = grad[1] + coef * a0 * b1 * c0
        grad[2] = grad[2] + coef * a0 * b0 * c1
        lap = lap + coef * (a2 * b0 * c0 + a0 * b2 * c0 + a0 * b0 * c2)
    return val, grad, lap


U_TERMS = [(1.0, [("s", 1), ("s", 1), ("s", 2)]), (0.5, [("s", 2), ("s", 1), ("s", 1)])]
V_TERMS = [(0.8, [("s", 2), ("s", 1), ("s", 1)]), (-0.3, [("s", 1), ("s", 2), ("s", 1)])]
W_TERMS = [(0.7, [("s", 1), ("s", 2), ("s", 1)]), (0.4, [("s", 1), ("s", 1), ("s", 3)])]
T_TERMS = [(0.3, [("s", 1), ("c", 1), ("c", 2)])]


def fields_at(x, y, z):
    """(value, grad, lap) of u, v, w, T at points (x, y, z)."""
    out = [sep(t, x, y, z) for t in (U_TERMS, V_TERMS, W_TERMS)]
    tv, tg, tl = sep(T_TERMS, x, y, z)
    tv = tv + 0.5 - x
    tg[0] = tg[0] - 1.0
    out.append((tv, tg, tl))
    return out


def continuous_N(g, x, y, z, comp):
    """Conservative continuous right-hand side of Eqs. 1-2 at given points."""
    F = fields_at(x, y, z)
    vel = F[:3]
    q = F[comp] if comp < 4 else None
    qv, qg, ql = q
    # -div(v q) = -(sum_b d(v_b q)/dx_b)
    adv = 0.0
    for b in range(3):
        vb, vbg, _ = vel[b]
        adv = adv + vbg[b] * qv + vb * qg[b]
    diffc = g.kappa if comp == 3 else g.nu
    r = -adv + diffc * ql
    if comp == 2:
        r = r + g.beta * F[3][0]
    return r


def stored_points(g, comp):
    """Coordinates (x, y, z) of the stored unknowns of a packed block."""
    pos = []
    for a in range(3):
        if comp == a:
            pos.append(g.faces[a][1:-1])
        else:
            pos.append(g.c[a])
    z, y, x = np.meshgrid(pos[2], pos[1], pos[0], indexing="ij")
    return x, y, z


def discrete_state(g):
    blocks = []
    for comp in range(4):
        x, y, z = stored_points(g, comp)
        blocks.append(fields_at(x, y, z)[comp][0])
    return g.pack(blocks)


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_nonlinear_operator_second_order(kind):
    """N converges to the continuous right-hand side at second order on
    manufactured fields that meet every boundary condition.

    Uniform grids: everywhere (the fields are odd/even about each wall as
    the half-cell wall treatment assumes).  Wall-clustered grids: on the
    region [0.15, 0.85]^3, because next to the wall the cosine grid's width
    ratio h_1/h_0 = 3, 5/3, ... is not close to 1 and the truncation error of
    the cell-centred even (adiabatic) T field there stays O(1)."""
    errs = []
    for n in (12, 24, 48):
        g = grid(n, n, n, kind, Gr=400.0, Pr=0.71)
        Nd = g.unpack(O.nonlinear(g, discrete_state(g)))
        e = []
        for comp in range(4):
            x, y, z = stored_points(g, comp)
            err = np.abs(Nd[comp] - continuous_N(g, x, y, z, comp))
            if kind == "clustered":
                inside = ((x > 0.15) & (x < 0.85) & (y > 0.15) & (y < 0.85)
                          & (z > 0.15) & (z < 0.85))
                err = err[inside]
            e.append(np.max(err))
        errs.append(e)
    errs = np.array(errs)
    order = np.log2(errs[:-1] / errs[1:])
    assert np.all(order[-1] > 1.8), (errs, order)


def test_diffusion_exact_on_quadratics_uniform():
    """Interior cells: the two-point diffusion is exact for quadratics."""
    g = grid(10, 9, 8, "uniform", Gr=0.0, Pr=2.0)     # nu = 1, kappa = 1/2
    X = np.zeros(g.size)
    bl = g.unpack(X)
    # u = y^2 alone: nu Lap u = 2 away from walls (u u is flux-free in y, z)
    x, y, z = stored_points(g, 0)
    bl[0][...] = y ** 2
    N = g.unpack(O.nonlinear(g, X))
    # x-advection of u = y^2 (constant along x) cancels in the interior
    assert np.allclose(N[0][1:-1, 1:-1, 1:-1], 2.0, atol=1e-10)
    # T = 1/2 - x + z^2 at rest: kappa Lap T = 2 kappa away from walls
    X = np.zeros(g.size)
    x, y, z = stored_points(g, 3)
    g.unpack(X)[3][...] = 0.5 - x + z ** 2
    N = g.unpack(O.nonlinear(g, X))
    assert np.allclose(N[3][1:-1, 1:-1, 1:-1], 0.5 * 2.0, atol=1e-10)


def test_conduction_profile_is_exact_for_heat_equation():
    """T = 1/2 - x with zero velocity makes the T residual vanish exactly,
    the x-wall fluxes included (Eq. 4 at half-cell distance)."""
    g = grid(8, 7, 6, "clustered", Gr=1e5)
    X = S.conduction_state(*g.faces)
    NT = g.unpack(O.nonlinear(g, X))[3]
    assert np.max(np.abs(NT)) < 1e-12


def test_heat_budget_telescopes():
    """sum_c V_c N_T = kappa * (net conductive heat flux through x-walls):
    interior fluxes cancel and there is no flux through the other walls."""
    g = grid(7, 6, 5, "clustered", Gr=3e4)
    X = S.base_flow(*g.faces, K=3, amp=0.05, seed=3)
    X = X + 0.01 * S.perturbation(g.size, 4)
    T = g.unpack(X)[3]
    NT = g.unpack(O.nonlinear(g, X))[3]
    lhs = np.sum(NT * g.cell_volume())
    area = g.along(g.h[1], 1)[:, :, 0] * g.along(g.h[2], 2)[:, :, 0]
    west = (T[:, :, 0] - 0.5) / g.d[0][0]
    east = (-0.5 - T[:, :, -1]) / g.d[0][-1]
    rhs = g.kappa * np.sum(area * (east - west))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(rhs))


# ---- symmetries of the cube (Sec. 2, the three maps) --------------------------
def sym_map(g, X, which):
    u, v, w, T = [b.copy() for b in g.unpack(X)]
    if which == "centro":      # {u,v,w,theta} -> -(...)(1-x, 1-y, 1-z)
        out = [-u[::-1, ::-1, ::-1], -v[::-1, ::-1, ::-1], -w[::-1, ::-1, ::-1], -T[::-1, ::-1, ::-1]]
    elif which == "refl_y":    # {u,v,w,theta} -> {u,-v,w,theta}(x, 1-y, z)
        out = [u[:, ::-1, :], -v[:, ::-1, :], w[:, ::-1, :], T[:, ::-1, :]]
    elif which == "rot2d":     # {u,v,w,theta} -> -{u,-v,w,theta}(1-x, y, 1-z)
        out = [-u[::-1, :, ::-1], v[::-1, :, ::-1], -w[::-1, :, ::-1], -T[::-1, :, ::-1]]
    else:
        raise ValueError(which)
    return g.pack(out)


@pytest.mark.parametrize("which", ["centro", "refl_y", "rot2d"])
def test_equivariance(which):
    """N(S X) = S N(X), J(S X0) S x = S J(X0) x and P S y = S P y for each
    symmetry map S (theta sign flips are linear in T - 1/2)."""
    g = grid(8, 7, 6, "clustered", Gr=2e5)
    X = S.base_flow(*g.faces, K=3, amp=0.05, seed=5) + 0.1 * S.perturbation(g.size, 6)
    x = S.perturbation(g.size, 7)
    assert rel(O.nonlinear(g, sym_map(g, X, which)), sym_map(g, O.nonlinear(g, X), which)) < 1e-13
    assert rel(O.jacobian(g, sym_map(g, X, which), sym_map(g, x, which)),
               sym_map(g, O.jacobian(g, X, x), which)) < 1e-13
    assert rel(O.project(g, sym_map(g, x, which)), sym_map(g, O.project(g, x), which)) < 1e-12


# ---- Jacobian against the nonlinear operator -------------------------------------
@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_jacobian_is_exact_central_difference(kind):
    """N is quadratic, so J x = [N(X0 + x) - N(X0 - x)] / 2 for any amplitude,
    and N(X0 + x) - N(X0) - J x does not depend on X0."""
    g = grid(9, 8, 7, kind, Gr=1e6)
    X0 = S.base_flow(*g.faces, K=3, amp=0.1, seed=8)
    x = S.perturbation(g.size, 9)
    for amp in (1e-3, 1.0, 1e3):
        J = O.jacobian(g, X0, amp * x)
        Jc = 0.5 * (O.nonlinear(g, X0 + amp * x) - O.nonlinear(g, X0 - amp * x))
        assert rel(J, Jc) < 1e-12
    X1 = X0 + S.perturbation(g.size, 10)
    q0 = O.nonlinear(g, X0 + x) - O.nonlinear(g, X0) - O.jacobian(g, X0, x)
    q1 = O.nonlinear(g, X1 + x) - O.nonlinear(g, X1) - O.jacobian(g, X1, x)
    assert rel(q0, q1) < 1e-12
    # the quadratic remainder is nonzero: the advection terms are present
    assert np.linalg.norm(q0) > 1e-3 * np.linalg.norm(O.jacobian(g, X0, x))


# ---- divergence, gradient, adjointness ---------------------------------------------
def test_discrete_curl_is_divergence_free():
    g = grid(9, 8, 10, "clustered")
    X = S.base_flow(*g.faces, K=3, amp=1.0, seed=11)
    vel_scale = np.max(np.abs(X[: g.off[3]]))
    assert np.max(np.abs(O.divergence(g, X))) < 1e-12 * vel_scale / min(min(h) for h in g.h)


def test_divergence_exact_cell_average():
    """u = sin(2 pi x) sin(pi y) at x-faces: D u is exactly the cell average
    of du/dx, i.e. (u(x_{i+1}) - u(x_i)) / h_i with walls zero."""
    g = grid(9, 6, 5, "clustered")
    X = np.zeros(g.size)
    x, y, z = stored_points(g, 0)
    g.unpack(X)[0][...] = np.sin(2 * PI * x) * np.sin(PI * y)
    fx = g.faces[0]
    cell = (np.sin(2 * PI * fx[1:]) - np.sin(2 * PI * fx[:-1])) / g.h[0]
    expect = cell[None, None, :] * np.sin(PI * g.c[1])[None, :, None]
    assert np.allclose(O.divergence(g, X), np.broadcast_to(expect, (5, 6, 9)), atol=1e-12)


def test_gradient_exact_on_linear_pressure():
    g = grid(7, 8, 9, "clustered")
    z, y, x = np.meshgrid(g.c[2], g.c[1], g.c[0], indexing="ij")
    Gp = g.unpack(O.gradient(g, 2.0 * x - 3.0 * y + 0.5 * z))
    for comp, val in enumerate((2.0, -3.0, 0.5)):
        assert np.allclose(Gp[comp], val, atol=1e-12)


def test_divergence_is_minus_adjoint_of_gradient():
    g = grid(7, 6, 5, "clustered")
    rng = np.random.default_rng(12)
    y = rng.standard_normal(g.size)
    p = rng.standard_normal(g.shapes[3])
    w = g.weights()
    lhs = np.sum(g.cell_volume() * O.divergence(g, y) * p)
    rhs = -np.dot(w * y, O.gradient(g, p))
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


# ---- fast diagonalization ----------------------------------------------------------
def test_fd_eigenvalues_closed_form_uniform():
    """Uniform Neumann cell-centred Laplacian: lam_m = -(4/h^2) sin^2(m pi / 2N)."""
    for n in (8, 13, 32):
        g = grid(n, n, n, "uniform")
        fd = O.FastDiag(g)
        m = np.arange(n)
        lam = -(4.0 * n * n) * np.sin(m * PI / (2 * n)) ** 2
        assert np.allclose(np.sort(fd.lam[0]), np.sort(lam), atol=1e-10 * n * n)
        assert np.allclose(fd.Q[0].T @ fd.Q[0], np.eye(n), atol=1e-13)


def dense(fn, nin, nout=None):
    cols = []
    for i in range(nin):
        e = np.zeros(nin)
        e[i] = 1.0
        cols.append(np.ravel(fn(e)))
    return np.array(cols).T


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_projection_matches_dense_least_squares(kind):
    """P y via fast diagonalization equals y - G p with p from a dense
    least-squares solve of (D G) p = D y."""
    g = grid(6, 5, 4, kind)
    C = g.ncell
    Dm = dense(lambda v: O.divergence(g, v), g.size)
    Gm = dense(lambda p: O.gradient(g, p.reshape(g.shapes[3])), C)
    L = Dm @ Gm
    assert np.linalg.matrix_rank(L) == C - 1
    assert np.allclose(L @ np.ones(C), 0.0, atol=1e-10)
    y = S.perturbation(g.size, 13)
    p = np.linalg.lstsq(L, Dm @ y, rcond=None)[0]
    assert rel(O.project(g, y), y - Gm @ p) < 1e-12


def test_projection_invariants():
    g = grid(9, 8, 7, "clustered")
    w = g.weights()
    y = S.perturbation(g.size, 14)
    z = S.perturbation(g.size, 15)
    Py = O.project(g, y)
    assert rel(O.project(g, Py), Py) < 1e-13                         # P^2 = P
    assert O.div_measure(g, Py) < 1e-13                              # D P = 0
    p = np.random.default_rng(16).standard_normal(g.shapes[3])
    Gp = O.gradient(g, p)
    assert np.linalg.norm(O.project(g, Gp)) < 1e-12 * np.linalg.norm(Gp)   # P G = 0
    a = np.dot(w * O.project(g, y), z)
    b = np.dot(w * y, O.project(g, z))
    assert abs(a - b) < 1e-12 * abs(a)                               # W-self-adjoint
    assert O.wnorm(w, Py) <= O.wnorm(w, y) * (1 + 1e-14)             # ||P||_W <= 1
    assert np.array_equal(g.unpack(Py)[3], g.unpack(y)[3])           # T untouched


def test_symmetry_measures_vanish_on_symmetric_field():
    g = grid(8, 8, 8, "clustered")
    X = S.base_flow(*g.faces, K=3, amp=0.1, seed=17) + 0.1 * S.perturbation(g.size, 18)
    Xs = X
    for which in ("centro", "refl_y", "rot2d"):
        Xs = 0.5 * (Xs + sym_map(g, Xs, which))
    assert max(O.symmetry_measures(g, Xs)) < 1e-14
    assert min(O.symmetry_measures(g, X)) > 1e-3


CLASSES = [(1, 1), (1, -1), (-1, 1), (-1, -1)]


def brute_symmetry_map(g, x, which):
    """S x found by matching physical positions: each unknown takes the value
    of the same field at the mirrored point (searched over all unknowns of
    that field), times the field's sign under the map."""
    mir = {"ref": (1,), "rot": (0, 2)}[which]
    sign = {"ref": (1, -1, 1, 1), "rot": (-1, 1, -1, -1)}[which]
    out = np.empty(g.size)
    for a, f in enumerate(g.unpack(x)):
        coords = []
        for ax in range(3):   # interior faces along the field's own axis, centres otherwise
            coords.append(g.faces[ax][1:-1] if ax == a else g.c[ax])
        pts = [(k, j, i) for k in range(f.shape[0]) for j in range(f.shape[1]) for i in range(f.shape[2])]
        pos = {tuple(round(coords[ax][(i, j, k)[ax]], 12) for ax in range(3)): (k, j, i) for (k, j, i) in pts}
        res = np.empty(f.shape)
        for (k, j, i) in pts:
            p = [coords[ax][(i, j, k)[ax]] for ax in range(3)]
            for ax in mir:
                p[ax] = 1.0 - p[ax]
            res[k, j, i] = sign[a] * f[pos[tuple(round(t, 12) for t in p)]]
        out[g.off[a]:g.off[a + 1]] = res.ravel()
    return out


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_symmetry_map_against_mirrored_positions(kind):
    g = grid(5, 4, 3, kind)
    x = S.perturbation(g.size, 31)
    for which in ("ref", "rot"):
        assert np.array_equal(O.symmetry_map(g, x, which), brute_symmetry_map(g, x, which))


def test_symmetry_maps_commute_with_the_equations():
    """The maps are symmetries of the discrete problem: N(S X) = S N(X) and
    P S = S P (a wrong sign on any field breaks the advection or buoyancy
    coupling), each map is an involution, and their product maps every field
    to minus its centro-symmetric image (Eq. 9)."""
    g = grid(8, 7, 6, "clustered", Gr=2e5)
    X = S.base_flow(*g.faces, K=3, amp=0.05, seed=5) + 0.1 * S.perturbation(g.size, 6)
    y = S.perturbation(g.size, 7)
    for which in ("ref", "rot"):
        Sm = lambda v: O.symmetry_map(g, v, which)  # noqa: E731
        assert rel(O.nonlinear(g, Sm(X)), Sm(O.nonlinear(g, X))) < 1e-13
        assert rel(O.project(g, Sm(y)), Sm(O.project(g, y))) < 1e-12
        assert np.array_equal(Sm(Sm(y)), y)
    c = O.symmetry_map(g, O.symmetry_map(g, y, "rot"), "ref")
    assert np.array_equal(c, g.pack([-f[::-1, ::-1, ::-1] for f in g.unpack(y)]))


def test_symmetry_classes_project_and_split():
    """The four class projections are W-orthogonal projections that sum to the
    identity; at a state with all three symmetries they commute with J and P."""
    g = grid(8, 7, 6, "clustered", Gr=2e5)
    w = g.weights()
    x = S.perturbation(g.size, 8)
    parts = [O.symmetry_project(g, x, er, eo) for er, eo in CLASSES]
    assert rel(sum(parts), x) < 1e-15
    for a in range(4):
        assert rel(O.symmetry_project(g, parts[a], *CLASSES[a]), parts[a]) < 1e-15
        for b in range(a):
            assert abs(O.wdot(w, parts[a], parts[b])) < 1e-14 * O.wdot(w, x, x)
    assert np.array_equal(O.symmetry_project(g, x, 0, 0), x)
    assert rel(O.symmetry_project(g, x, 1, 0) + O.symmetry_project(g, x, -1, 0), x) < 1e-15
    X0 = O.symmetry_project(g, S.base_flow(*g.faces, K=3, amp=0.05, seed=5), 1, 1)
    for cl in CLASSES:
        Pi = lambda v: O.symmetry_project(g, v, *cl)  # noqa: E731
        assert rel(Pi(O.jacobian(g, X0, x)), O.jacobian(g, X0, Pi(x))) < 1e-13
        assert rel(Pi(O.project(g, x)), O.project(g, Pi(x))) < 1e-12


def test_symmetry_classes_against_the_measures():
    """Eqs. 7-9: a state in class (+,+) has all three measures zero; adding a
    class (e_ref, e_rot) perturbation keeps exactly the measures whose map has
    sign +1 on it (the centro-symmetry's sign is e_ref e_rot) at zero."""
    g = grid(8, 8, 8, "clustered")
    Xs = O.symmetry_project(g, S.base_flow(*g.faces, K=3, amp=0.1, seed=17), 1, 1)
    assert max(O.symmetry_measures(g, Xs)) < 1e-14
    x = S.perturbation(g.size, 19)
    for er, eo in CLASSES:
        m = O.symmetry_measures(g, Xs + 0.1 * O.symmetry_project(g, x, er, eo))
        for val, e in zip(m, (er, eo, er * eo)):
            assert (val < 1e-14) if e == 1 else (val > 1e-3), (er, eo, m)


def test_workload_grids():
    f = S.faces_clustered(256)
    assert f[0] == 0.0 and f[-1] == 1.0 and np.all(np.diff(f) > 0)
    assert np.max(np.abs(f[::-1] - (1.0 - f))) <= 2.0 ** -53
    h = np.diff(f)
    assert abs(h.min() - 3.765e-5) < 1e-8 and abs(h.max() - 6.136e-3) < 1e-5
    assert S.packed_size(256, 256, 256) == 66_912_256
    assert S.packed_size(32, 32, 32) == 128_000
    assert S.packed_size(100, 100, 100) == 3_970_000


def _div_measure_brute(xf, yf, zf, y, shapes):
    """max |net flux| / max |face flux| by explicit loops over the cells of
    a small grid: each interior face carries (normal velocity) x (its area,
    the product of the two cell widths across it, taken from the face
    coordinates); a cell's net flux is the sum of its six face fluxes with
    outward signs, wall faces carrying none (no penetration)."""
    nx, ny, nz = len(xf) - 1, len(yf) - 1, len(zf) - 1
    sizes = [int(np.prod(s)) for s in shapes]
    u = y[:sizes[0]].reshape(shapes[0])
    v = y[sizes[0]:sizes[0] + sizes[1]].reshape(shapes[1])
    w = y[sizes[0] + sizes[1]:sizes[0] + sizes[1] + sizes[2]].reshape(shapes[2])

    def fx(i, j, k):    # flux through x-face i (0..nx) of cell row (j, k)
        return 0.0 if i in (0, nx) else u[k, j, i - 1] * (yf[j + 1] - yf[j]) * (zf[k + 1] - zf[k])

    def fy(i, j, k):
        return 0.0 if j in (0, ny) else v[k, j - 1, i] * (xf[i + 1] - xf[i]) * (zf[k + 1] - zf[k])

    def fz(i, j, k):
        return 0.0 if k in (0, nz) else w[k - 1, j, i] * (xf[i + 1] - xf[i]) * (yf[j + 1] - yf[j])

    net, face = 0.0, 0.0
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                b = fx(i + 1, j, k) - fx(i, j, k) + fy(i, j + 1, k) - fy(i, j, k) + fz(i, j, k + 1) - fz(i, j, k)
                net = max(net, abs(b))
                face = max(face, abs(fx(i, j, k)), abs(fy(i, j, k)), abs(fz(i, j, k)))
    return net / face


def test_div_measure_against_brute_force_face_loops():
    """The normalized divergence (the mixed form's stopping quantity, Sec. 3:
    divergence-free Krylov vectors) equals an explicit loop over cells and
    faces on a 6 x 5 x 4 wall-clustered grid, for a field that is not
    divergence free and for a projected one; a copy of the oracle's formula
    with one axis's face area taken across the wrong axis is caught."""
    xf, yf, zf = S.faces_clustered(6), S.faces_clustered(5), S.faces_clustered(4)
    g = O.Grid(xf, yf, zf, Gr=1e5, Pr=0.71)
    for seed in (41, 42):
        y = S.perturbation(g.size, seed)
        ref = _div_measure_brute(xf, yf, zf, y, g.shapes)
        assert abs(O.div_measure(g, y) - ref) <= 1e-13 * ref
        yp = O.project(g, y)
        refp = _div_measure_brute(xf, yf, zf, yp, g.shapes)
        # at round-off level the two summation orders differ; both are ~eps
        assert refp < 1e-13 and O.div_measure(g, yp) < 1e-13

    def planted(g, y, wrong):
        b = O.divergence(g, y) * g.cell_volume()
        vel = g.unpack(y)[:3]
        fl = 0.0
        for a in range(3):
            areas = [g.along(g.h[c], c) for c in range(3)]
            areas[a] = 1.0
            if a == wrong:      # the z-width of an x-face read along y
                areas[2] = g.along(g.h[1], 1)
            fl = max(fl, float(np.max(np.abs(vel[a] * areas[0] * areas[1] * areas[2]))))
        return float(np.max(np.abs(b))) / fl

    # an x-velocity field alone, so the largest face flux is an x-face's
    y = np.zeros(g.size)
    y[:g.shapes[0][0] * g.shapes[0][1] * g.shapes[0][2]] = S.perturbation(g.size, 43)[:np.prod(g.shapes[0])]
    ref = _div_measure_brute(xf, yf, zf, y, g.shapes)
    assert abs(O.div_measure(g, y) - ref) <= 1e-13 * ref
    assert abs(planted(g, y, 0) - ref) > 1e-2 * ref

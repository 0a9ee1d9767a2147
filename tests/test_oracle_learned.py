"""Pins of the learned-guess oracle (oracle/unet.py, oracle/transfer.py)
against brute force, finite differences, closed forms and library routines.
CPU only."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import disc as O  # noqa: E402
from oracle import transfer as TR  # noqa: E402
from oracle import unet as U  # noqa: E402
from synth import inputs as S  # noqa: E402


# ---- brute-force network on tiny inputs (numpy, explicit taps and blocks) ---------------
def bf_conv(x, W, b, relu):
    """x [ci, r, r, r], W [co, ci, k, k, k]: cross-correlation with zero padding."""
    co, ci, k = W.shape[0], W.shape[1], W.shape[2]
    r = x.shape[1]
    h = k // 2
    xp = np.zeros((ci, r + 2 * h, r + 2 * h, r + 2 * h))
    xp[:, h:h + r, h:h + r, h:h + r] = x
    y = np.zeros((co, r, r, r)) + b[:, None, None, None]
    for dz in range(k):
        for dy in range(k):
            for dx in range(k):
                patch = xp[:, dz:dz + r, dy:dy + r, dx:dx + r]          # [ci, r, r, r]
                y += np.tensordot(W[:, :, dz, dy, dx], patch, axes=(1, 0))
    return np.maximum(y, 0.0) if relu else y


def bf_pool(x):
    c, r = x.shape[0], x.shape[1]
    out = np.zeros((c, r // 2, r // 2, r // 2))
    for a in range(2):
        for b in range(2):
            for d in range(2):
                out += x[:, a::2, b::2, d::2]
    return out / 8


def bf_up(x):
    c, r = x.shape[0], x.shape[1]
    out = np.zeros((c, 2 * r, 2 * r, 2 * r))
    for a in range(2):
        for b in range(2):
            for d in range(2):
                out[:, a::2, b::2, d::2] = x
    return out


def bf_network(w, x):
    p = U.split_params(w)

    def cv(i, t, relu=True):
        return bf_conv(t, p[i][0], p[i][1], relu)

    e1 = cv(1, cv(0, x))
    e2 = cv(3, cv(2, bf_pool(e1)))
    e3 = cv(5, cv(4, bf_pool(e2)))
    d2 = cv(7, cv(6, np.concatenate([bf_up(e3), e2])))
    d1 = cv(9, cv(8, np.concatenate([bf_up(d2), e1])))
    return cv(10, d1, relu=False)


def random_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    out = []
    for ci, co, k in U.CONVS:
        out.append(rng.standard_normal(co * ci * k ** 3) * scale * np.sqrt(2.0 / (ci * k ** 3)))
        out.append(0.1 * rng.standard_normal(co))
    return np.concatenate(out).astype(np.float32)


def test_parameter_count():
    assert U.num_params() == 354628
    assert len(random_params(0)) == U.num_params()


def test_network_matches_brute_force():
    w = random_params(1)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 4, 4, 4, 4))
    got = U.output(w, x)
    wq = U.bf16_round(w).astype(np.float64)
    for b in range(2):
        ref = bf_network(wq, x[b])
        assert np.allclose(got[b], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_bf16_rounding_against_torch_and_ties():
    rng = np.random.default_rng(3)
    a = (rng.standard_normal(100000) * 10.0 ** rng.uniform(-30, 30, 100000)).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(U.bf16_round(a), ref)
    one = np.float32(1.0)
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 1 + 2.0 ** -8 + 2.0 ** -20],
                    dtype=np.float32)
    assert list(U.bf16_round(ties)) == [one, np.float32(1 + 2.0 ** -6), -one, np.float32(1 + 2.0 ** -7)]
    special = np.array([np.inf, -np.inf, 0.0, -0.0], dtype=np.float32)
    assert np.array_equal(U.bf16_round(special), special)
    assert np.isnan(U.bf16_round(np.array([np.nan], dtype=np.float32)))[0]


def test_gradient_matches_finite_differences():
    w = random_params(4)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, 4, 4, 4, 4))
    gout = rng.standard_normal((2, 4, 4, 4, 4))
    g = U.grad_of_dot(w, x, gout)
    wq = U.bf16_round(w).astype(np.float64)
    xt, gt = torch.from_numpy(x), torch.from_numpy(gout)

    def f(wv):
        with torch.no_grad():
            return float((U.forward(torch.from_numpy(wv), xt) * gt).sum())

    for s in range(3):
        d = np.random.default_rng(10 + s).standard_normal(len(w))
        eps = 1e-6
        fd = (f(wq + eps * d) - f(wq - eps * d)) / (2 * eps)
        assert abs(fd - g @ d) <= 1e-6 * (abs(fd) + np.abs(g).sum() * 1e-3)
    # one coordinate of each convolution's weights and biases
    o = 0
    for ci, co, k in U.CONVS:
        for j in (o + 3, o + co * ci * k ** 3):         # a weight and the first bias
            e = np.zeros(len(w))
            e[j] = 1.0
            fd = (f(wq + 1e-6 * e) - f(wq - 1e-6 * e)) / 2e-6
            assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(fd))
        o += co * ci * k ** 3 + co


def test_mse_gradient_is_gradient_of_dot_with_residual():
    w = random_params(6)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((1, 4, 8, 8, 8))
    t = rng.standard_normal((1, 4, 8, 8, 8))
    loss, g = U.mse_loss_and_grad(w, x, t)
    y = U.output(w, x)
    assert np.isclose(loss, np.mean((y - t) ** 2), rtol=1e-13)
    g2 = U.grad_of_dot(w, x, 2 * (y - t) / y.size)
    assert np.allclose(g, g2, rtol=1e-10, atol=1e-14)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are exactly g and
    g^2, so every step moves by lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w = np.array([1.0, 1.0, 1.0, 1.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr = 0.01
    for t in range(1, 6):
        w_prev = w
        w, m, v = U.adam_step(w, g, m, v, t, lr)
        assert np.allclose(w_prev - w, lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_make_inputs():
    c = S.faces_clustered(8)
    cen = 0.5 * (c[1:] + c[:-1])
    x = U.make_inputs((cen, cen, cen), (6.0, 8.5), [1e6, 10 ** 8.5, 10 ** 7.25])
    assert x.shape == (3, 4, 8, 8, 8)
    assert np.allclose(x[0, 3], -1) and np.allclose(x[1, 3], 1) and np.allclose(x[2, 3], 0)
    assert np.allclose(x[0, 0, 2, 5, :], 2 * cen - 1)
    assert np.allclose(x[0, 2, :, 1, 6], 2 * cen - 1)


# ---- transfers ----------------------------------------------------------------------
def grid(kind, n):
    f = S.faces_uniform(n) if kind == "uniform" else S.faces_clustered(n)
    return O.Grid(f, f, f, Gr=1e6, Pr=0.71), f


ID = (np.zeros(4), np.ones(4))


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_conduction_state_maps_to_zero_and_back(kind):
    g, f = grid(kind, 8)
    X = S.conduction_state(f, f, f)
    cells = TR.cells_from_state(g, X, 2, *ID)
    assert np.abs(cells).max() <= 1e-15
    # network centres: any increasing set inside (0, 1)
    cen = [np.linspace(0.1, 0.9, 4)] * 3
    Y = TR.state_from_cells(g, np.zeros((4, 4, 4, 4)), cen, *ID)
    assert np.array_equal(Y, X)


def test_cells_of_constant_face_velocity():
    """u = 1 on every interior x-face: centre value 1, except 1/2 next to the
    x-walls; block means are the volume-weighted means of those."""
    g, f = grid("clustered", 8)
    X = np.zeros(g.size)
    u = g.unpack(X)[0]
    u[:] = 1.0
    c1 = TR.cells_from_state(g, X, 1, *ID)
    expect = np.ones(8)
    expect[0] = expect[-1] = 0.5
    assert np.allclose(c1[0], expect[None, None, :], rtol=0, atol=1e-15)
    assert np.abs(c1[1:3]).max() == 0.0
    assert np.allclose(c1[3], -(0.5 - g.c[0])[None, None, :], rtol=0, atol=1e-15)
    c2 = TR.cells_from_state(g, X, 2, *ID)
    h = g.h[0]
    first = (0.5 * h[0] + h[1]) / (h[0] + h[1])
    assert np.isclose(c2[0, 0, 0, 0], first, rtol=1e-14)
    assert np.isclose(c2[0, 0, 0, 1], 1.0, rtol=1e-14)


def test_cells_conserve_volume_integrals():
    g, f = grid("clustered", 12)
    X = S.base_flow(f, f, f, K=3, amp=0.1, seed=5) + 0.01 * S.perturbation(g.size, 6)
    for fac in (1, 2, 3, 4):
        c = TR.cells_from_state(g, X, fac, *ID)
        hc = [np.add.reduceat(g.h[a], np.arange(0, 12, fac)) for a in range(3)]
        vc = hc[2][:, None, None] * hc[1][None, :, None] * hc[0][None, None, :]
        vol = g.h[2][:, None, None] * g.h[1][None, :, None] * g.h[0][None, None, :]
        for ch, fld in enumerate(TR.centre_fields(g, X)):
            assert np.isclose((vc * c[ch]).sum(), (vol * fld).sum(), rtol=1e-12, atol=1e-15)


def test_affine_normalization():
    g, f = grid("uniform", 8)
    X = S.base_flow(f, f, f, K=2, amp=0.1, seed=1)
    shift, scale = np.array([0.1, -0.2, 0.3, 0.05]), np.array([2.0, 0.5, 4.0, 0.25])
    a = TR.cells_from_state(g, X, 2, *ID)
    b = TR.cells_from_state(g, X, 2, shift, scale)
    assert np.allclose(b, (a - shift[:, None, None, None]) / scale[:, None, None, None], rtol=1e-14, atol=1e-15)


def test_state_from_cells_reproduces_linear_theta_inside_the_hull():
    """Trilinear interpolation is exact for linear data: T unknowns whose
    position lies inside the hull of the network centres get the linear
    function exactly."""
    g, f = grid("clustered", 16)
    cen = [np.sort(np.random.default_rng(a).uniform(0.05, 0.95, 5 + a)) for a in range(3)]

    def lin(x, y, z):
        return 0.3 + 0.7 * x - 0.2 * y + 0.45 * z

    cells = np.zeros((4, len(cen[2]), len(cen[1]), len(cen[0])))
    cells[3] = lin(cen[0][None, None, :], cen[1][None, :, None], cen[2][:, None, None])
    Y = TR.state_from_cells(g, cells, cen, *ID)
    T = g.unpack(Y)[3] - (0.5 - g.c[0])[None, None, :]
    inside = [(g.c[a] >= cen[a][0]) & (g.c[a] <= cen[a][-1]) for a in range(3)]
    sel = np.ix_(inside[2], inside[1], inside[0])
    ref = lin(g.c[0][None, None, :], g.c[1][None, :, None], g.c[2][:, None, None])
    assert np.allclose(T[sel], ref[sel], rtol=0, atol=1e-14)
    # adiabatic walls: beyond the last centre in y the value is that of the last centre row
    jy = g.c[1] > cen[1][-1]
    ix = inside[0]
    kz = inside[2]
    sub = T[np.ix_(kz, jy, ix)]
    ref_edge = lin(g.c[0][None, None, ix], cen[1][-1], g.c[2][kz][:, None, None])
    assert np.allclose(sub, np.broadcast_to(ref_edge, sub.shape), atol=1e-14)
    # x walls: theta is 0 at x = 0, so it ramps linearly up to the first centre
    i0 = g.c[0] < cen[0][0]
    ramp = T[np.ix_(kz, inside[1], i0)]
    full = lin(cen[0][0], g.c[1][inside[1]][None, :, None], g.c[2][kz][:, None, None])
    assert np.allclose(ramp, full * (g.c[0][i0] / cen[0][0])[None, None, :], atol=1e-14)


def test_state_from_cells_velocity_ramps_to_the_walls():
    g, f = grid("uniform", 10)
    cen = [np.linspace(0.2, 0.8, 4)] * 3
    cells = np.zeros((4, 4, 4, 4))
    cells[0] = 1.0
    Y = TR.state_from_cells(g, cells, cen, *ID)
    u = g.unpack(Y)[0]
    xf = g.faces[0][1:-1]

    def hat(s):
        return np.clip(np.minimum(s / 0.2, (1 - s) / 0.2), 0, 1)

    ref = hat(g.c[2])[:, None, None] * hat(g.c[1])[None, :, None] * hat(xf)[None, None, :]
    assert np.allclose(u, ref, atol=1e-14)
    assert np.abs(g.unpack(Y)[1]).max() == 0 and np.abs(g.unpack(Y)[2]).max() == 0


def test_round_trip_on_the_same_grid():
    """Network centres = solver centres: T comes back exactly; a face value
    becomes the distance-weighted mean of its two neighbouring centre values,
    i.e. (u_{i-1} + 2 u_i + u_{i+1}) / 4 on a uniform grid."""
    g, f = grid("uniform", 8)
    X = S.base_flow(f, f, f, K=2, amp=0.1, seed=3)
    cells = TR.cells_from_state(g, X, 1, *ID)
    Y = TR.state_from_cells(g, cells, [g.c[0], g.c[1], g.c[2]], *ID)
    assert np.allclose(g.unpack(Y)[3], g.unpack(X)[3], rtol=0, atol=1e-15)
    u = g.unpack(X)[0]
    up = np.pad(u, ((0, 0), (0, 0), (1, 1)))
    ref = 0.25 * up[:, :, :-2] + 0.5 * up[:, :, 1:-1] + 0.25 * up[:, :, 2:]
    assert np.allclose(g.unpack(Y)[0], ref, rtol=0, atol=1e-15)


def test_cell_increment_of_equal_predictions_is_zero_and_linear():
    g, f = grid("clustered", 8)
    cen = [np.linspace(0.1, 0.9, 4)] * 3
    rng = np.random.default_rng(8)
    a = rng.standard_normal((4, 4, 4, 4))
    b = rng.standard_normal((4, 4, 4, 4))
    X = S.base_flow(f, f, f, K=2, amp=0.1, seed=9)
    scale = np.array([0.5, 2.0, 1.5, 0.25])
    assert np.allclose(TR.add_cell_increment(g, X, a, a, cen, scale), X, rtol=0, atol=1e-14)
    # linear in the difference: S(a) - S(b) = S(a - b) - S(0), and S(0) is the conduction state
    d = TR.add_cell_increment(g, X, a, b, cen, scale) - X
    ref = TR.state_from_cells(g, a - b, cen, np.zeros(4), scale) - S.conduction_state(f, f, f)
    assert np.allclose(d, ref, rtol=0, atol=1e-13)

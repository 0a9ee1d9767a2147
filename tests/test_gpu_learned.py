"""GPU parity of the learned-guess kernels (include/kvnn.h and the transfer
calls of include/kv.h) against the CPU oracle (oracle/unet.py,
oracle/transfer.py), through the C ABI.

Tolerances follow from the arithmetic: the network runs in FP32 with
BF16-rounded weights, against an FP64 evaluation with the same rounded
weights.  A convolution output sums K <= 96 * 27 = 2592 products; eleven
layers compound, so the relative error is ~ 11 sqrt(K) u_32 = 4e-5 at worst
(u_32 = 6e-8); the bar is 1e-4 on outputs and gradients (relative 2-norm).
ReLU kinks within rounding of zero can switch a gradient term; they are
rare and inside that bar.  The transfers are FP64 (from FP32 cells) or end
in one FP32 rounding.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import disc as O  # noqa: E402
from oracle import transfer as TR  # noqa: E402
from oracle import unet as U  # noqa: E402
from synth import inputs as S  # noqa: E402
from tests.gpu_util import faces, to_dev, to_host  # noqa: E402

pytestmark = pytest.mark.gpu

TOL_NET = 1e-4


def rel(a, b):
    nb = np.linalg.norm(np.ravel(b))
    d = np.linalg.norm(np.ravel(a) - np.ravel(b))
    return float(d / nb) if nb > 0 else float(d)


def centres(kind, r):
    f = faces(kind, r)
    c = 0.5 * (f[1:] + f[:-1])
    return (c, c, c)


def net(kind, r, batch_max=2, seed=3):
    from paper_2210_08816_amd import kvnn
    return kvnn.Net(centres(kind, r), (4.0, 8.5), batch_max=batch_max, seed=seed)


def fdev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("kind,r,batch", [("clustered", 8, 2), ("uniform", 16, 1), ("clustered", 12, 2),
                                          ("uniform", 4, 1), ("clustered", 20, 2)])
def test_forward_and_inputs(kind, r, batch):
    print(f"case kvnn forward {kind} r={r} batch={batch}", flush=True)
    N = net(kind, r, batch_max=batch)
    grs = [10 ** (4.0 + 1.7 * b) for b in range(batch)]
    inp = torch.empty(batch * 4 * r ** 3, dtype=torch.float32, device="cuda")
    N.make_inputs(grs, inp)
    ref_in = U.make_inputs(N.centres, (4.0, 8.5), grs)
    assert np.allclose(to_host(inp).reshape(ref_in.shape), ref_in, rtol=0, atol=1e-7)
    out = torch.empty_like(inp)
    N.forward(inp, batch, out)
    w = N.get_params()
    ref = U.output(w, to_host(inp).reshape(ref_in.shape).astype(np.float64))
    assert rel(to_host(out), ref) <= TOL_NET
    # predict = make_inputs + forward for one Gr
    one = torch.empty(4 * r ** 3, dtype=torch.float32, device="cuda")
    N.predict(grs[-1], one)
    assert np.array_equal(to_host(one), to_host(out)[-4 * r ** 3:])


@pytest.mark.parametrize("kind,r,batch", [("clustered", 8, 2), ("uniform", 16, 1), ("uniform", 4, 1),
                                          ("clustered", 20, 2)])
def test_backward(kind, r, batch):
    print(f"case kvnn backward {kind} r={r}", flush=True)
    N = net(kind, r, batch_max=batch, seed=11)
    rng = np.random.default_rng(12)
    x = rng.standard_normal((batch, 4, r, r, r)).astype(np.float32)
    gout = rng.standard_normal((batch, 4, r, r, r)).astype(np.float32)
    g = N.backward(fdev(x), fdev(gout), batch)
    ref = U.grad_of_dot(N.get_params(), x.astype(np.float64), gout.astype(np.float64))
    assert rel(g, ref) <= TOL_NET
    # every convolution's block of the gradient, not only the total
    o = 0
    for ci, co, k in U.CONVS:
        n = co * ci * k ** 3 + co
        assert rel(g[o:o + n], ref[o:o + n]) <= TOL_NET, (ci, co, k)
        o += n


def test_train_step_loss_and_adam():
    r, batch = 8, 2
    N = net("clustered", r, batch_max=batch, seed=21)
    rng = np.random.default_rng(22)
    x = fdev(rng.standard_normal((batch, 4, r, r, r)))
    t = fdev(rng.standard_normal((batch, 4, r, r, r)))
    w0 = N.get_params()
    # the gradient the step will use: same inputs, same weights, fixed-order sums
    out = torch.empty_like(x)
    N.forward(x, batch, out)
    sc = torch.tensor(np.float32(2.0 / out.numel()), device="cuda")   # the loss kernel's FP32 factor
    g = N.backward(x, ((out - t) * sc).contiguous(), batch).astype(np.float64)
    loss_ref, g_ref = U.mse_loss_and_grad(w0, to_host(x).reshape(batch, 4, r, r, r).astype(np.float64),
                                          to_host(t).reshape(batch, 4, r, r, r).astype(np.float64))
    assert rel(g, g_ref) <= TOL_NET
    lr = 1e-3
    loss = N.train_step(x, t, batch, lr)
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    w1 = N.get_params().astype(np.float64)
    w1_ref, m, v = U.adam_step(w0.astype(np.float64), g, 0.0, 0.0, 1, lr)
    assert np.max(np.abs(w1 - w1_ref) - 1e-6 * lr - 2e-7 * np.abs(w1_ref)) <= 0
    # second step from the new weights (bias corrections of step 2)
    N.forward(x, batch, out)
    g2 = N.backward(x, ((out - t) * sc).contiguous(), batch).astype(np.float64)
    N.train_step(x, t, batch, lr)
    w2 = N.get_params().astype(np.float64)
    w2_ref, _, _ = U.adam_step(w1, g2, m, v, 2, lr)
    assert np.max(np.abs(w2 - w2_ref) - 1e-6 * lr - 2e-7 * np.abs(w2_ref)) <= 0


def test_training_reduces_the_loss_and_params_round_trip():
    r, batch = 8, 2
    N = net("uniform", r, batch_max=batch, seed=31)
    inp = torch.empty(batch * 4 * r ** 3, dtype=torch.float32, device="cuda")
    N.make_inputs([1e5, 1e7], inp)
    # a smooth target that depends on position and Gr
    xin = inp.view(batch, 4, r, r, r)
    t = torch.stack([xin[:, 0] * xin[:, 3], torch.sin(2 * xin[:, 1]), xin[:, 2] ** 2, xin[:, 3]], dim=1)
    t = t.contiguous().view(-1)
    first = N.train_step(inp, t, batch, 3e-3)
    for _ in range(150):
        last = N.train_step(inp, t, batch, 3e-3)
    assert last < 0.1 * first, (first, last)
    w = N.get_params()
    N2 = net("uniform", r, batch_max=batch, seed=99)
    N2.set_params(w)
    o1 = torch.empty_like(inp)
    o2 = torch.empty_like(inp)
    N.forward(inp, batch, o1)
    N2.forward(inp, batch, o2)
    assert torch.equal(o1, o2)


def test_network_rejects_bad_input():
    from paper_2210_08816_amd import kvnn
    N = net("uniform", 8, batch_max=1)
    x = torch.zeros(2 * 4 * 512, dtype=torch.float32, device="cuda")
    with pytest.raises(kvnn.KVNNError) as e:
        N.forward(x, 2, x)
    assert e.value.code == kvnn.KVNN_EINVAL
    with pytest.raises(kvnn.KVNNError):
        N.predict(-1.0, x[:4 * 512])
    with pytest.raises(kvnn.KVNNError):
        kvnn.Net(centres("uniform", 6), (4.0, 8.0))


# ---- transfers --------------------------------------------------------------------------
TRANSFER_CASES = [("clustered", (16, 16, 16), 2), ("uniform", (12, 8, 20), 4), ("clustered", (10, 6, 8), 1)]


@pytest.mark.parametrize("kind,shape,fac", TRANSFER_CASES)
def test_cells_from_state(kind, shape, fac):
    from paper_2210_08816_amd import kv
    fx = [faces(kind, n) for n in shape]
    g = O.Grid(*fx, Gr=1e6, Pr=0.71)
    X = S.base_flow(*fx, K=3, amp=0.1, seed=41) + 0.01 * S.perturbation(g.size, 42)
    shift, scale = np.array([0.01, -0.02, 0.0, 0.1]), np.array([0.05, 0.07, 0.2, 0.3])
    ctx = kv.Context(*fx, Gr=1e6, Pr=0.71)
    nc = (shape[0] // fac) * (shape[1] // fac) * (shape[2] // fac)
    out = torch.empty(4 * nc, dtype=torch.float32, device="cuda")
    ctx.cells_from_state(to_dev(X), fac, shift, scale, out)
    ref = TR.cells_from_state(g, X, fac, shift, scale).astype(np.float32)
    got = to_host(out).reshape(ref.shape)
    assert np.max(np.abs(got - ref) / (np.abs(ref) + 1e-6)) <= 2 ** -23
    with pytest.raises(kv.KVError):
        ctx.cells_from_state(to_dev(X), 7, shift, scale, out)


@pytest.mark.parametrize("kind,shape,r", [("clustered", (32, 32, 32), 16), ("uniform", (12, 8, 20), 8),
                                          ("clustered", (64, 64, 64), 32)])
def test_state_from_cells(kind, shape, r):
    from paper_2210_08816_amd import kv
    fx = [faces(kind, n) for n in shape]
    g = O.Grid(*fx, Gr=1e6, Pr=0.71)
    cen = centres("clustered", r)
    rng = np.random.default_rng(51)
    cells = rng.standard_normal((4, r, r, r)).astype(np.float32)
    shift, scale = np.array([0.01, -0.02, 0.0, 0.1]), np.array([0.05, 0.07, 0.2, 0.3])
    ctx = kv.Context(*fx, Gr=1e6, Pr=0.71)
    X = torch.empty(g.size, dtype=torch.float64, device="cuda")
    ctx.state_from_cells(fdev(cells), cen, shift, scale, X)
    ref = TR.state_from_cells(g, cells.astype(np.float64), cen, shift, scale)
    assert np.max(np.abs(to_host(X) - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_state_add_cell_increment():
    from paper_2210_08816_amd import kv
    shape, r = (24, 24, 24), 12
    fx = [faces("clustered", n) for n in shape]
    g = O.Grid(*fx, Gr=1e6, Pr=0.71)
    cen = centres("clustered", r)
    rng = np.random.default_rng(61)
    a = rng.standard_normal((4, r, r, r)).astype(np.float32)
    b = rng.standard_normal((4, r, r, r)).astype(np.float32)
    X0 = S.base_flow(*fx, K=3, amp=0.1, seed=62)
    scale = np.array([0.05, 0.07, 0.2, 0.3])
    ctx = kv.Context(*fx, Gr=1e6, Pr=0.71)
    X = to_dev(X0)
    ctx.state_add_cell_increment(fdev(a), fdev(b), cen, scale, X)
    ref = TR.add_cell_increment(g, X0, a.astype(np.float64), b.astype(np.float64), cen, scale)
    assert np.max(np.abs(to_host(X) - ref)) <= 1e-13 * np.max(np.abs(ref))

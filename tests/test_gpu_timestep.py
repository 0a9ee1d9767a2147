"""GPU parity of the time stepper (kv_time_steps) against the oracle's
SBDF2 scheme (oracle/timestep.py), through the C ABI: the first step at
order 1, then order 2, and a continued call from (X, Xprev)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import disc as O  # noqa: E402
from oracle import timestep as TS  # noqa: E402
from synth import inputs as S  # noqa: E402
from tests.gpu_util import assert_parity, faces, to_dev, to_host  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,shape,Gr", [("clustered", (16, 12, 10), 1e5), ("uniform", (9, 7, 8), 2e4)])
def test_time_steps_match_oracle(kind, shape, Gr):
    from paper_2210_08816_amd import kv
    print(f"case time steps {kind} {shape}", flush=True)
    fx = [faces(kind, n) for n in shape]
    g = O.Grid(*fx, Gr=Gr, Pr=0.71)
    X0 = O.project(g, S.base_flow(*fx, K=2, amp=0.1, seed=52))
    ctx = kv.Context(*fx, Gr=Gr, Pr=0.71)
    try:
        dt = 0.01
        X = to_dev(X0)
        Xp = torch.empty_like(X)
        ctx.time_steps(X, Xp, dt, 4, start=True)
        ref, ref_p = TS.integrate(g, X0, dt, 4)
        assert_parity(g, to_host(X), ref, 1e-12, label="X after 4 steps")
        assert_parity(g, to_host(Xp), ref_p, 1e-12, label="Xprev after 4 steps")
        ctx.time_steps(X, Xp, dt, 3, start=False)            # continued at order 2
        ref2, ref2_p = TS.integrate(g, ref, dt, 3, Xprev=ref_p)
        assert_parity(g, to_host(X), ref2, 1e-12, label="X after 7 steps")
        assert O.div_measure(g, to_host(X)) < 1e-11
        # zero steps change nothing; bad arguments are refused
        before = to_host(X).copy()
        ctx.time_steps(X, Xp, dt, 0, start=False)
        assert np.array_equal(to_host(X), before)
        for bad in ((-1.0, 1), (dt, -1)):
            with pytest.raises(kv.KVError) as e:
                ctx.time_steps(X, Xp, bad[0], bad[1])
            assert e.value.code == kv.KV_EINVAL
    finally:
        ctx.close()


def test_time_steps_keep_a_steady_state():
    """A converged steady state (GPU Newton, 16^3 uniform, Gr 1e4) is a fixed
    point of the stepper."""
    from paper_2210_08816_amd import kv
    from paper_2210_08816_amd.continuation import newton_solve
    f = S.faces_uniform(16)
    ctx = kv.Context(f, f, f, Gr=1e4, Pr=0.71)
    try:
        X = to_dev(S.conduction_state(f, f, f))
        info = newton_solve(ctx, X, tol_rel=1e-13, tol_abs=1e-13, max_matvec=4000)
        assert info["converged"], info
        Xs = to_host(X).copy()
        Xp = torch.empty_like(X)
        ctx.time_steps(X, Xp, 0.05, 10)
        w = O.Grid(f, f, f, Gr=1e4, Pr=0.71).weights()
        assert O.wnorm(w, to_host(X) - Xs) <= 1e-10 * O.wnorm(w, Xs)
    finally:
        ctx.close()

"""The critical-Gr finder end to end on the GPU, on a tiny grid where the
branch is stable over the range: continuation, Newton to each new Gr from
the nearest state, class-restricted Arnoldi, and the record it returns."""
import pytest

pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def test_finder_on_a_stable_range():
    from paper_2210_08816_amd.critical import run
    out = run(n=8, grid="clustered", gr_lo=1e5, gr_hi=2.25e5, ratio=1.5, sym=(1, -1), krylov=20, n_eigs=2,
              tol=1e-8, max_matvec=6000, log=lambda m: print(m, flush=True))
    assert out["gr_critical"] is None and out["converged"] is False and out["note"] == "no crossing in the range"
    grs = [h["Gr"] for h in out["history"]]
    assert grs == pytest.approx([1e5, 1.5e5, 2.25e5])
    for h in out["history"]:
        assert h["re_lambda1"] is not None and h["re_lambda1"] < 0, h
        assert h["residuals"][0] <= 1e-8 * max(abs(complex(*v)) for v in h["values"]), h
    assert out["newton_matvecs"] > 0 and out["arnoldi_matvecs"] > 0

"""Host logic of the critical-Gr finder: bracketing on a geometric sweep and
regula falsi in log Gr, pinned on closed-form sigma(Gr) curves (the GPU
side, continuation and Arnoldi, is covered by the solver tests)."""
import math

from paper_2210_08816_amd.critical import find_crossing


def curve(fn, skip=()):
    calls = []

    def sigma(gr):
        calls.append(gr)
        if any(abs(gr / s - 1.0) < 1e-9 for s in skip):
            return None, {"arnoldi": "not converged"}
        return fn(gr), {}
    return sigma, calls


def test_log_linear_crossing():
    sigma, calls = curve(lambda gr: 0.02 * math.log(gr / 3.3e7))
    out = find_crossing(sigma, 1e7, 2e8, ratio=1.6, rtol=1e-6)
    assert abs(out["gr"] / 3.3e7 - 1.0) < 1e-9          # regula falsi is exact on a line in log Gr
    a, b = out["bracket"]
    assert a <= 3.3e7 <= b
    assert calls[:3] == [1e7, 1.6e7, 2.56e7]            # the sweep steps by the ratio


def test_curved_crossing_within_tolerance():
    root = 2e7 * math.sqrt(1.7)
    sigma, calls = curve(lambda gr: (gr / 2e7) ** 2 - 1.7)
    out = find_crossing(sigma, 1e6, 1e9, ratio=2.0, rtol=1e-8)
    assert abs(out["gr"] / root - 1.0) < 1e-7
    assert len(calls) < 40                               # Illinois keeps regula falsi from stalling


def test_unconverged_points_are_skipped():
    root = 4.5e7
    f = lambda gr: math.tanh(5.0 * math.log(gr / root))  # noqa: E731
    sigma, calls = curve(f, skip=(1.6e7, 4.096e7))
    out = find_crossing(sigma, 1e7, 2e8, ratio=1.6, rtol=1e-6)
    assert abs(out["gr"] / root - 1.0) < 1e-5
    assert any(h[1] is None for h in out["history"])


def test_no_crossing_and_unstable_start():
    sigma, calls = curve(lambda gr: -0.01 - 1.0 / math.log(gr))
    out = find_crossing(sigma, 1e6, 1e8, ratio=1.6)
    assert out["gr"] is None and out["bracket"] is None
    assert calls[-1] == 1e8                              # the last step is clipped to the range end
    sigma, calls = curve(lambda gr: 0.1)
    out = find_crossing(sigma, 1e6, 1e8)
    assert out["gr"] is None and out["note"] == "unstable at the start" and len(calls) == 1


def test_branch_lost_ends_the_sweep():
    calls = []

    def sigma(gr):
        calls.append(gr)
        if gr > 5e7:
            return None, {"newton": "not converged", "stop": True}
        return -0.05, {}
    out = find_crossing(sigma, 1e7, 1e9, ratio=1.6)
    assert out["gr"] is None and out["note"].startswith("branch not followed")
    assert calls[-1] > 5e7 and len([c for c in calls if c > 5e7]) == 1


def test_symmetry_class_arguments():
    """Classes on the command line: letters or signs; a value argparse has
    eaten ('--sym=--' arrives as an empty list) is an error, not 'no class'."""
    import argparse
    import pytest
    from paper_2210_08816_amd.stability import parse_sym
    assert parse_sym("mm") == [(-1, -1)] and parse_sym("mp,pm") == [(-1, 1), (1, -1)]
    assert parse_sym("-+") == [(-1, 1)] and parse_sym(None) is None and len(parse_sym("all")) == 4
    ap = argparse.ArgumentParser()
    ap.add_argument("--sym", default=None)
    for bad in (ap.parse_args(["--sym=--"]).sym, "", "mx", "m"):
        with pytest.raises(ValueError):
            parse_sym(bad)

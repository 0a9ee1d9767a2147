"""Host logic of the critical-Gr finder: bracketing on a geometric sweep and
regula falsi in log Gr, pinned on closed-form sigma(Gr) curves (the GPU
side, continuation and Arnoldi, is covered by the solver tests)."""
import math

import pytest

from paper_2210_08816_amd.critical import find_crossing, same_mode_by_frequency


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
    assert out["converged"] is False
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


def test_aborted_refinement_is_not_a_result():
    """Refinement points that do not converge (the regula-falsi point and its
    bisection fallback) stop the refinement; the bracket is then wider than
    1 + rtol, so no critical value is returned, only an estimate."""
    root = 3.3e7
    f = lambda gr: 0.02 * math.log(gr / root)  # noqa: E731
    calls = []

    def sigma(gr):
        calls.append(gr)
        if len(calls) > 4:                    # every point after the bracket fails
            return None, {"arnoldi": "not converged"}
        return f(gr), {}
    out = find_crossing(sigma, 1e7, 2e8, ratio=1.6, rtol=1e-6)
    assert out["gr"] is None and out["converged"] is False
    assert out["note"].startswith("refinement stopped")
    a, b = out["bracket"]
    assert b / a > 1.0 + 1e-6 and a <= root <= b and a <= out["gr_estimate"] <= b
    ok = find_crossing(curve(f)[0], 1e7, 2e8, ratio=1.6, rtol=1e-6)
    assert ok["converged"] is True and abs(ok["gr"] / root - 1.0) < 1e-9


def test_mode_switch_is_not_a_crossing():
    """Two modes of the near-axis cluster: mode 1 (Im 0.67) leads below
    4e7 and stays stable; mode 2 (Im 0.043) leads above and is unstable.  A
    bracket across the switch is not a crossing of one mode; inside a
    one-mode bracket a point that returns the other mode counts as not
    converged."""
    def sigma_switch(gr):
        if gr < 4e7:
            return -0.01, {"values": [[-0.01, 0.67]]}
        return 0.005, {"values": [[0.005, 0.043]]}
    out = find_crossing(sigma_switch, 1e7, 2e8, ratio=1.6, same_mode=same_mode_by_frequency)
    assert out["gr"] is None and out["converged"] is False and "different eigenmodes" in out["note"]
    # without the check the switch would be taken for a crossing
    assert find_crossing(sigma_switch, 1e7, 2e8, ratio=1.6)["gr"] is not None

    root = 3.3e7

    def sigma_one(gr):
        val = 0.02 * math.log(gr / root)
        if 3.0e7 < gr < 3.2e7:          # another mode leads in a window below the root
            return -0.2, {"values": [[-0.2, 0.9]]}
        return val, {"values": [[val, 0.05]]}
    out = find_crossing(sigma_one, 1e7, 2e8, ratio=1.6, rtol=1e-6, same_mode=same_mode_by_frequency)
    assert out["converged"] and abs(out["gr"] / root - 1.0) < 1e-6
    assert same_mode_by_frequency({"values": [[0, 0.05]]}, {"values": [[0, 0.055]]})
    assert not same_mode_by_frequency({"values": [[0, 0.043]]}, {"values": [[0, 0.67]]})
    assert not same_mode_by_frequency({"values": []}, {"values": [[0, 0.1]]})


def test_run_rejects_state_gr_without_state_or_above_gr_lo():
    from paper_2210_08816_amd.critical import run
    with pytest.raises(ValueError):
        run(n=8, gr_lo=2e7, gr_hi=3e7, state=None, state_gr=1e7)
    with pytest.raises(ValueError):
        run(n=8, gr_lo=2e7, gr_hi=3e7, state=[0.0], state_gr=2e7)

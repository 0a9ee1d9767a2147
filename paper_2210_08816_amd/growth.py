"""The time stepper against the eigenvalue: a steady state perturbed along
the real part of a leading eigenvector grows (or decays) and oscillates as
exp(lambda t) while the perturbation is small, so one period T = 2 pi / Im
lambda of the fully nonlinear time integration (kv_time_steps) must multiply
it by exp(Re lambda T) and half a period by -exp(Re lambda T / 2).  This
cross-checks the time stepper (Eqs. 1-6 integrated in time, the paper's
Sec. 4.2.3 computations) with the linear stability result (Sec. 1 and
Sec. 3) on the same grid.  Every step runs in the library; this module only
sequences the calls and compares the numbers.

    python -m paper_2210_08816_amd.growth --n 64 --gr 5e7 --load-state s.npy --sym mp --steps-per-period 20000
"""
from __future__ import annotations

import json
import math
import time


def measure(ctx, X, v, lam, steps_per_period, eps=1e-6, log=print, chunk=10000):
    """X: converged steady state (device); v: unit real vector, the real part
    of the eigenvector of lam (device); lam: the eigenvalue (Im >= 0).
    Integrates X + eps v over one period T = 2 pi / Im lam (for a real lam,
    over T = 1 / |lam|) in steps_per_period steps and returns the measured
    factors against the predicted ones: exp(Re lam T) over T and, for a
    complex lam, -exp(Re lam T / 2) for the projection on the start after
    half a period."""
    import torch
    T = 2.0 * math.pi / lam.imag if lam.imag > 0 else 1.0 / abs(lam.real)
    dt = T / steps_per_period
    half = steps_per_period // 2
    Y = X.clone()
    ctx.axpby(eps, v, 1.0, Y)                # Y = X + eps v
    Yp = torch.empty_like(Y)
    d = torch.empty_like(Y)

    def pert():
        d.copy_(Y)
        ctx.axpby(-1.0, X, 1.0, d)           # d = Y - X
        return d

    d0 = pert().clone()
    n0 = ctx.dot(d0, d0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = [0]

    def advance(k):
        # in chunks (the same SBDF2 sequence: a call continues from (Y, Yp)),
        # one progress line per chunk
        while k > 0:
            c = min(k, chunk)
            ctx.time_steps(Y, Yp, dt, c, start=done[0] == 0)
            done[0] += c
            k -= c
            log(f"[growth] {done[0]}/{steps_per_period} steps, |d|/|d0| = "
                f"{math.sqrt(ctx.dot(pert(), pert()) / n0):.6f}")

    advance(half)
    c_half = ctx.dot(pert(), d0) / n0
    advance(steps_per_period - half)
    dT = pert()
    ratio = math.sqrt(ctx.dot(dT, dT) / n0)
    c_full = ctx.dot(dT, d0) / n0
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    t_half = half * dt
    out = {"lambda": [lam.real, lam.imag], "period": T, "dt": dt, "steps": steps_per_period, "eps": eps,
           "seconds": round(sec, 3),
           "growth_over_period": ratio, "predicted_growth": math.exp(lam.real * T),
           "rate_measured": math.log(ratio) / T, "rate_predicted": lam.real,
           "projection_half_period": c_half,
           "predicted_half_period": (-1.0 if lam.imag > 0 else 1.0) * math.exp(lam.real * t_half),
           "projection_full_period": c_full}
    log(json.dumps(out))
    return out


def run(n=64, grid="clustered", Gr=5e7, Pr=0.71, state=None, sym=(-1, 1), steps_per_period=20000, eps=1e-6,
        krylov=200, keep=63, tol=1e-8, max_matvec=200000, v0_seed=77, log=print):
    """Leading eigenpair of class sym at the steady state (thick-restarted
    Arnoldi), then one period of the time stepper from the perturbed state."""
    import numpy as np
    import torch
    from synth import inputs as S  # seeded grid faces (input construction only)
    from . import kv
    f = S.faces_uniform(n) if grid == "uniform" else S.faces_clustered(n)
    X = torch.from_numpy(np.asarray(state, dtype=np.float64)).cuda()
    ctx = kv.Context(f, f, f, Gr=Gr, Pr=Pr)
    try:
        ctx.set_base_flow(X)
        F = torch.empty_like(X)
        fn = ctx.residual(F)
        v0 = torch.from_numpy(np.random.default_rng(v0_seed).standard_normal(ctx.n)).cuda()
        ev = torch.empty(3 * ctx.n, dtype=torch.float64, device="cuda")
        t0 = time.perf_counter()
        vals, res, info = ctx.arnoldi_leading_eigs(v0, krylov, 2, tol=tol, max_matvec=max_matvec, sym=sym,
                                                   keep=keep, evecs=ev, check=False)
        t_eig = time.perf_counter() - t0
        if not info["converged"]:
            raise RuntimeError(f"leading eigenvalue not converged: {vals}, {info}")
        lam = complex(vals[0])
        log(f"[growth] Gr={Gr:.4e} |F|={fn:.2e} lambda={lam} ({info['matvecs']} matvecs, {t_eig:.1f}s)")
        v = ev[:ctx.n].clone()
        out = measure(ctx, X, v, lam, steps_per_period, eps=eps, log=log)
        out.update({"grid": f"{n}^3 {grid}", "Gr": Gr, "residual": fn, "symmetry_class": list(sym),
                    "arnoldi_matvecs": info["matvecs"], "arnoldi_seconds": round(t_eig, 3)})
        return out
    finally:
        ctx.close()


def main(argv=None):
    import argparse

    import numpy as np

    from .stability import parse_sym
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--grid", choices=("uniform", "clustered"), default="clustered")
    ap.add_argument("--gr", type=float, required=True)
    ap.add_argument("--load-state", required=True, help="a converged steady state at --gr (.npy)")
    ap.add_argument("--sym", default="mp", help="symmetry class of the eigenmode, e.g. mp")
    ap.add_argument("--steps-per-period", type=int, default=20000)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--krylov", type=int, default=200)
    ap.add_argument("--keep", type=int, default=63)
    ap.add_argument("--tol", type=float, default=1e-8, help="Arnoldi tolerance")
    ap.add_argument("--max-matvec", type=int, default=200000, help="Arnoldi budget")
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    res = run(n=a.n, grid=a.grid, Gr=a.gr, state=np.load(a.load_state), sym=parse_sym(a.sym)[0],
              steps_per_period=a.steps_per_period, eps=a.eps, krylov=a.krylov, keep=a.keep, tol=a.tol,
              max_matvec=a.max_matvec,
              log=lambda m: print(m, flush=True))
    text = json.dumps(res)
    if a.json:
        with open(a.json, "w") as fh:
            fh.write(text + "\n")
    print(text, flush=True)


if __name__ == "__main__":
    main()

"""Steady states along a Grashof-number sweep by Newton continuation on the GPU.

Newton's method (paper Sec. 1) with corrections from kv_newton_correction
(BiCGstab(2) + GMRES); Gr is raised gradually and each converged state
starts the next solve, as the paper does when it follows a branch.  Every
step runs in the library's kernels; this module only sequences the calls.
"""
from __future__ import annotations

import math
import time

import numpy as np


def newton_solve(ctx, X, tol_rel=1e-10, tol_abs=1e-12, max_iter=30, max_matvec=20000, delta0_fn=None,
                 log=None, sym=None):
    """Newton iteration on a context (its Gr fixed).  X: torch float64 CUDA
    tensor, updated in place (left at the last iterate on failure).  Stops
    when ||F|| <= max(tol_abs, tol_rel * ||F(X_start)||).  The inner solve
    tolerance is max(1e-10, min(1e-2, ||F||)), loosened to a tenth of the
    target over ||F|| near the end.  delta0_fn(X) gives the first
    BiCGstab(2) iterate of the first Newton step (None: zero); sym: None or a
    symmetry class (e_ref, e_rot) the corrections are sought in.  A correction
    that exhausts its budget is taken when its relative residual is below 0.5
    (an inexact Newton step); otherwise the iteration stops.  Returns a dict
    with the residual history, matvecs, wall time and whether it converged."""
    import torch
    F = torch.empty_like(X)
    d = torch.empty_like(X)
    hist, mv = [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ok = False
    for it in range(max_iter + 1):
        ctx.set_base_flow(X)
        fn = ctx.residual(F)
        hist.append(fn)
        if log:
            log(f"  newton it={it} |F|={fn:.3e} matvecs={mv}")
        if not np.isfinite(fn):
            break
        if fn <= max(tol_abs, tol_rel * hist[0]):
            ok = True
            break
        if it == max_iter:
            break
        # inner tolerance: min(1e-2, ||F||) (quadratic convergence), floored at
        # 1e-10, but never tighter than what brings ||F|| to a tenth of the
        # target (solving the last correction to 1e-10 relative is wasted
        # work once a 1e-3 reduction reaches the target)
        target = max(tol_abs, tol_rel * hist[0])
        eta = max(1e-10, min(1e-2, fn), min(0.5, 0.1 * target / fn))
        d0 = delta0_fn(X) if delta0_fn is not None and it == 0 else None
        info = ctx.newton_correction(F, d, tol=eta, max_matvec=max_matvec, delta0=d0, check=False, sym=sym)
        mv += info["matvecs"]
        if log:
            log(f"  correction: tol {eta:.2e} matvecs {info['matvecs']} relres {info['relres']:.2e} "
                f"gmres {info['used_gmres']} status {info['status']}")
        if info["status"] != 0:
            # a correction that ran out of budget is still an inexact Newton
            # step when it halved the linearized residual: take it and let the
            # next residual decide (near a converged state the last solves
            # can stagnate above a tolerance the step does not need)
            from .kv import KV_ENOCONV
            if not (info["status"] == KV_ENOCONV and info["relres"] < 0.5):
                break
        ctx.axpby(1.0, d, 1.0, X)  # X <- X + delta on the device
    torch.cuda.synchronize()
    return dict(converged=ok, hist=hist, matvecs=mv, iters=len(hist) - 1, seconds=time.perf_counter() - t0)


def sweep(faces, grs, Pr=0.71, X0=None, log=print, max_halvings=3, tol_rel=1e-10, tol_abs=1e-12,
          precond_sigma=None, gmres_restart=None, gr0=None, gmres_deflation=0, mixed=False, **kw):
    """Continuation over increasing Gr values, from X0 (default: the
    conduction state) converged at Gr = gr0 (None: X0 is not a converged
    state).  A failed step is retried from the last converged state at the
    geometric midpoint in Gr, at most max_halvings times per requested value
    (a first step from an X0 without gr0 is not retried).  precond_sigma: None, or the shift of the Stokes/heat
    preconditioner of the Newton corrections; gmres_restart: None (the
    library's default) or the restart length of their GMRES continuation;
    gmres_deflation: harmonic Ritz vectors kept across its restarts (0: none);
    mixed: the corrections' projections in the mixed form.
    Returns (states, infos) for
    the requested Gr values reached; a value that cannot be reached ends the
    sweep."""
    import torch
    from . import kv
    if X0 is None:
        X0 = _conduction_state(*faces)
    X = torch.as_tensor(X0, dtype=torch.float64).cuda().clone()
    states, infos = [], []
    gr_last = gr0
    for Gr in grs:
        target, halvings = Gr, 0
        spent_mv, spent_s = 0, 0.0   # over every attempt for this value
        while True:
            Xtry = X.clone()
            ctx = kv.Context(*faces, Gr=target, Pr=Pr)
            try:
                if precond_sigma is not None:
                    ctx.set_preconditioner(True, precond_sigma)
                if gmres_restart is not None:
                    ctx.set_gmres_restart(gmres_restart)
                if gmres_deflation:
                    ctx.set_gmres_deflation(gmres_deflation)
                if mixed:
                    ctx.set_solver_projection(True)
                ctx.project(Xtry)
                info = newton_solve(ctx, Xtry, tol_rel=tol_rel, tol_abs=tol_abs, log=log, **kw)
            finally:
                ctx.close()
            info["Gr"] = target
            spent_mv += info["matvecs"]
            spent_s += info["seconds"]
            log(f"[continuation] Gr={target:.4e}: converged={info['converged']} iters={info['iters']} "
                f"matvecs={info['matvecs']} |F|={info['hist'][-1]:.2e} {info['seconds']:.1f}s")
            if info["converged"]:
                X = Xtry
                gr_last = target
                if target == Gr:
                    break
                target = Gr  # midpoint reached: try the requested value again
                continue
            if gr_last is None or halvings >= max_halvings:
                return states, infos + [info]
            halvings += 1
            target = math.sqrt(gr_last * target)
        info["matvecs_all_attempts"] = spent_mv
        info["seconds_all_attempts"] = spent_s
        infos.append(info)
        states.append(X.clone())
    return states, infos


def _conduction_state(xf, yf, zf):
    """Zero velocity and T = 1/2 - x at the cell centres, packed."""
    xf = np.asarray(xf, dtype=np.float64)
    nx, ny, nz = len(xf) - 1, len(yf) - 1, len(zf) - 1
    n_vel = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    X = np.zeros(n_vel + nx * ny * nz)
    cx = 0.5 * (xf[:-1] + xf[1:])
    X[n_vel:] = np.broadcast_to((0.5 - cx)[None, None, :], (nz, ny, nx)).ravel()
    return X

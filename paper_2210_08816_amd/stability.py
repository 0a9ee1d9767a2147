"""Linear stability of a steady state, end to end on the GPU: Newton
continuation in Gr to a target value, then the leading eigenvalues of the
Jacobian at the converged state by Chebyshev-preconditioned Arnoldi
iteration (the paper's method, Sec. 1 and Sec. 3).  Reports the wall time
and matvec count of each stage.  With --sym the Arnoldi iteration runs once
per symmetry class of perturbations (Sec. 2, Eqs. 7-9), its Krylov space
restricted to the class.

    python -m paper_2210_08816_amd.stability --n 64 --gr 4e7 --krylov 60 --eigs 10
    python -m paper_2210_08816_amd.stability --n 64 --gr 4e7 --sym all
    python -m paper_2210_08816_amd.stability --n 64 --gr 4e7 --sym mp,mm
"""
from __future__ import annotations

import json
import time

import numpy as np

from . import kv
from .continuation import sweep


def run(n=64, grid="clustered", Gr=4e7, Pr=0.71, ratio=1.6, krylov=60, n_eigs=10, tol=1e-8, max_matvec=200000,
        cheb_degree_max=200, precond_sigma=10.0, v0_seed=77, state=None, save_state=None, sym=None, keep=0,
        from_state=None, from_gr=None, gmres_restart=None, gmres_deflation=0, newton_max_matvec=20000,
        max_restarts=100000, newton_sym=None, cayley=None, inner_tol=1e-10, inner_max_matvec=20000, mixed=False,
        log=print):
    """state: a converged packed state at Gr (host array) to start from
    instead of continuation; save_state: file to store the converged state;
    sym: None (one unrestricted Arnoldi run) or a list of symmetry classes
    (e_ref, e_rot), one restricted run each; cayley: None, or (pole, zero) of
    a Cayley transform for the (thick-restarted) Arnoldi runs, whose inner
    solves take the Stokes/heat preconditioner of precond_sigma, the GMRES
    restart gmres_restart, inner_tol and inner_max_matvec; mixed: the
    projections inside Newton and Arnoldi in the mixed form."""
    import torch
    from synth import inputs as S  # seeded grid faces (input construction only)
    f = S.faces_uniform(n) if grid == "uniform" else S.faces_clustered(n)
    faces = (f, f, f)
    cont = None
    if state is None:
        grs = []
        g = 1e4 if from_state is None else from_gr * ratio
        while g < Gr:
            grs.append(g)
            g *= ratio
        grs.append(Gr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        states, infos = sweep(faces, grs, Pr=Pr, max_matvec=newton_max_matvec, max_iter=20,
                              precond_sigma=precond_sigma, gmres_restart=gmres_restart,
                              gmres_deflation=gmres_deflation, X0=from_state, gr0=from_gr, log=log,
                              sym=newton_sym, mixed=mixed)
        torch.cuda.synchronize()
        t_cont = time.perf_counter() - t0
        if len(states) < len(grs):
            raise RuntimeError(f"continuation stopped at Gr = {infos[-1]['Gr']:.4e}")
        X = states[-1]
        last = infos[-1]
        cont = {"steps": len(grs), "seconds": round(t_cont, 3),
                "matvecs": int(sum(i["matvecs_all_attempts"] for i in infos)),
                "last_newton_iters": last["iters"], "last_newton_matvecs": last["matvecs"],
                "last_newton_seconds": round(last["seconds"], 3), "precond_sigma": precond_sigma}
        if save_state:
            np.save(save_state, X.cpu().numpy())
    else:
        X = torch.from_numpy(np.asarray(state, dtype=np.float64)).cuda()
    ctx = kv.Context(*faces, Gr=Gr, Pr=Pr)
    try:
        ctx.set_base_flow(X)
        F = torch.empty_like(X)
        fn = ctx.residual(F)
        meas = ctx.symmetry_measures(X)
        v0 = torch.from_numpy(np.random.default_rng(v0_seed).standard_normal(ctx.n)).cuda()
        if mixed:
            ctx.set_solver_projection(True)
        if cayley is not None:
            if precond_sigma is not None:
                ctx.set_preconditioner(True, precond_sigma)
            if gmres_restart:
                ctx.set_gmres_restart(gmres_restart)
            ctx.set_spectral_transform(kv.KV_ST_CAYLEY, pole=cayley[0], zero=cayley[1], inner_tol=inner_tol,
                                       inner_max_matvec=inner_max_matvec)
        runs = []
        for cls in (sym or [None]):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            vals, res, info = ctx.arnoldi_leading_eigs(v0, krylov, n_eigs, tol=tol, max_matvec=max_matvec,
                                                       cheb_degree_max=cheb_degree_max, sym=cls, check=False,
                                                       keep=keep, max_restarts=max_restarts)
            torch.cuda.synchronize()
            t_eig = time.perf_counter() - t1
            runs.append({"symmetry_class": list(cls) if cls else None, "krylov_dim": krylov, "n_eigs": n_eigs,
                         "restart": f"thick, keep {keep}" if keep else "Chebyshev filter",
                         "cayley": list(cayley) if cayley is not None else None, "mixed": bool(mixed),
                         "inner_matvecs": info["inner_matvecs"],
                         "tol": tol, "seconds": round(t_eig, 3), "matvecs": info["matvecs"],
                         "restarts": info["restarts"], "converged": info["converged"], "status": info["status"],
                         "eigenvalues": [[float(v.real), float(v.imag)] for v in vals],
                         "residuals": [float(r) for r in res]})
            log(json.dumps(runs[-1]))
    finally:
        ctx.close()
    if cont is not None:
        cont["residual"] = fn
    return {
        "grid": f"{n}^3 {grid}", "Gr": Gr, "Pr": Pr, "unknowns": int(X.numel()), "residual": fn,
        "continuation": cont,
        "symmetry_measures": list(meas),
        "arnoldi": runs[0] if sym is None else runs,
    }


def parse_sym(text):
    """'all', or comma-separated classes, each two signs (reflection, 2-D
    rotation): '+' or 'p' kept, '-' or 'm' broken, '0' free; e.g. 'mp,mm'
    (the letters avoid argparse reading a leading '--' as an option end)."""
    if text is None:
        return None
    if not isinstance(text, str) or not text:
        raise ValueError("empty symmetry class (write broken/kept as m/p, e.g. --sym mm)")
    if text == "all":
        return [(1, 1), (1, -1), (-1, 1), (-1, -1)]
    sign = {"+": 1, "p": 1, "-": -1, "m": -1, "0": 0}
    out = []
    for pair in text.split(","):
        if len(pair) != 2 or any(ch not in sign for ch in pair):
            raise ValueError(f"bad symmetry class {pair!r}")
        out.append((sign[pair[0]], sign[pair[1]]))
    return out


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--grid", choices=("uniform", "clustered"), default="clustered")
    ap.add_argument("--gr", type=float, default=4e7)
    ap.add_argument("--krylov", type=int, default=60)
    ap.add_argument("--eigs", type=int, default=10)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--degree", type=int, default=200, help="largest Chebyshev filter degree")
    ap.add_argument("--max-matvec", type=int, default=200000)
    ap.add_argument("--sigma", type=float, default=10.0, help="preconditioner shift (negative: none)")
    ap.add_argument("--json", default=None)
    ap.add_argument("--save-state", default=None, help="store the converged state (.npy)")
    ap.add_argument("--load-state", default=None, help="start from a stored converged state (.npy)")
    ap.add_argument("--sym", default=None,
                    help="symmetry classes for restricted Arnoldi runs: 'all', or a comma list of sign pairs "
                         "(reflection, 2-D rotation), p = kept and m = broken, such as --sym pm,mm")
    ap.add_argument("--keep", type=int, default=0,
                    help="thick restart keeping this many Ritz vectors (0: Chebyshev-filtered restart)")
    ap.add_argument("--from-state", default=None,
                    help="continue from a stored converged state (.npy) at --from-gr instead of from rest")
    ap.add_argument("--from-gr", type=float, default=None)
    ap.add_argument("--ratio", type=float, default=1.6, help="continuation step ratio in Gr")
    ap.add_argument("--gmres-restart", type=int, default=None)
    ap.add_argument("--gmres-deflation", type=int, default=0)
    ap.add_argument("--newton-max-matvec", type=int, default=20000)
    ap.add_argument("--newton-sym", default=None,
                    help="symmetry class of the Newton corrections, e.g. pp (the symmetric branch)")
    ap.add_argument("--mixed", action="store_true", help="mixed-form projections inside Newton and Arnoldi")
    ap.add_argument("--cayley", default=None,
                    help="POLE,ZERO: thick-restarted Arnoldi on (A - pole)^-1 (A - zero) (needs --keep)")
    ap.add_argument("--inner-tol", type=float, default=1e-10, help="relative tolerance of the Cayley inner solves")
    ap.add_argument("--inner-max-matvec", type=int, default=20000, help="budget of one Cayley inner solve")
    a = ap.parse_args(argv)
    state = np.load(a.load_state) if a.load_state else None
    cayley = tuple(float(t) for t in a.cayley.split(",")) if a.cayley else None
    if cayley is not None and len(cayley) != 2:
        raise SystemExit("--cayley takes POLE,ZERO")
    res = run(n=a.n, grid=a.grid, Gr=a.gr, krylov=a.krylov, n_eigs=a.eigs, tol=a.tol, cheb_degree_max=a.degree,
              max_matvec=a.max_matvec, precond_sigma=None if a.sigma < 0 else a.sigma, state=state,
              save_state=a.save_state, sym=parse_sym(a.sym), keep=a.keep, ratio=a.ratio,
              from_state=np.load(a.from_state) if a.from_state else None, from_gr=a.from_gr,
              gmres_restart=a.gmres_restart, gmres_deflation=a.gmres_deflation,
              newton_max_matvec=a.newton_max_matvec,
              newton_sym=parse_sym(a.newton_sym)[0] if a.newton_sym else None,
              cayley=cayley, inner_tol=a.inner_tol, inner_max_matvec=a.inner_max_matvec, mixed=a.mixed,
              log=lambda m: print(m, flush=True))
    text = json.dumps(res)
    if a.json:
        with open(a.json, "w") as fh:
            fh.write(text + "\n")
    print(text, flush=True)


if __name__ == "__main__":
    main()

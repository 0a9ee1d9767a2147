"""Learned Newton initial guess: training data, training, guesses, evaluation.

The paper follows steady branches by Newton continuation in Gr (Sec. 1):
each solve starts from a converged state at a nearby Gr.  Here a network
(include/kvnn.h) trained on such converged states predicts the state at a
new Gr instead; the prediction is interpolated to the solver grid, projected,
and Newton starts from it.  The Newton residual judges the guess, and
continuation from the nearest converged state remains the fallback.

Every numerical step runs in the library's kernels (cell transfers,
projection, network forward/backward/Adam, Newton); this module sequences
the calls, holds the per-channel normalization (8 scalars taken from the
training targets) and shuffles the mini-batches.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import kv, kvnn
from .continuation import _conduction_state, newton_solve, sweep


def coarse_centres(faces, factor):
    """Midpoints of the cells of the grid coarsened by factor, per axis."""
    out = []
    for f in faces:
        f = np.asarray(f, dtype=np.float64)
        cf = f[::factor]
        out.append(0.5 * (cf[1:] + cf[:-1]))
    return out


@dataclass
class Normalization:
    shift: np.ndarray = field(default_factory=lambda: np.zeros(4))
    scale: np.ndarray = field(default_factory=lambda: np.ones(4))


@dataclass
class TrainingSet:
    faces: tuple
    factor: int
    grs: list
    inputs: object       # torch float32 [N, 4, r, r, r] (CUDA)
    targets: object      # torch float32 [N, 4, r, r, r] (CUDA), normalized
    norm: Normalization
    centres: list


def build_training_set(faces, grs, states, factor, net_for_inputs=None, Pr=0.71):
    """Targets from converged states (kv_cells_from_state), normalized per
    channel by the mean and standard deviation over the whole set."""
    import torch
    ctx = kv.Context(*faces, Gr=max(grs), Pr=Pr)
    try:
        nx, ny, nz = ctx.nx, ctx.ny, ctx.nz
        if nx != ny or ny != nz:
            raise ValueError("the network grid is cubic")
        r = nx // factor
        raw = torch.empty((len(states), 4, r, r, r), dtype=torch.float32, device="cuda")
        for k, X in enumerate(states):
            ctx.cells_from_state(X, factor, np.zeros(4), np.ones(4), raw[k].view(-1))
        torch.cuda.synchronize()
        mean = raw.double().mean(dim=(0, 2, 3, 4)).cpu().numpy()
        std = raw.double().std(dim=(0, 2, 3, 4)).cpu().numpy()
        norm = Normalization(mean, np.maximum(std, 1e-12))
        tgt = torch.empty_like(raw)
        for k, X in enumerate(states):
            ctx.cells_from_state(X, factor, norm.shift, norm.scale, tgt[k].view(-1))
    finally:
        ctx.close()
    cen = coarse_centres(faces, factor)
    return TrainingSet(tuple(faces), factor, list(grs), None, tgt, norm, cen)


def train(ts: TrainingSet, lgr_range, epochs=2000, batch=4, lr=2e-3, lr_final=2e-5, seed=3, data_seed=4,
          log=None, net=None):
    """Adam on the mean squared error of the normalized targets, cosine
    learning-rate decay from lr to lr_final; mini-batches drawn without
    replacement in a seeded order.  Returns (net, loss history, seconds)."""
    import torch
    nset = ts.targets.shape[0]
    batch = min(batch, nset)
    if net is None:
        net = kvnn.Net(ts.centres, lgr_range, batch_max=batch, seed=seed)
    r = net.res
    inputs = torch.empty((nset, 4, r, r, r), dtype=torch.float32, device="cuda")
    for k, gr in enumerate(ts.grs):
        net.make_inputs([gr], inputs[k].view(-1))
    ts.inputs = inputs
    rng = np.random.default_rng(data_seed)
    steps_per_epoch = math.ceil(nset / batch)
    total = epochs * steps_per_epoch
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step = 0
    xb = torch.empty((batch, 4, r, r, r), dtype=torch.float32, device="cuda")
    tb = torch.empty_like(xb)
    for ep in range(epochs):
        order = rng.permutation(nset)
        ep_loss = 0.0
        for s in range(steps_per_epoch):
            idx = order[s * batch:(s + 1) * batch]
            b = len(idx)
            sel = torch.from_numpy(idx).cuda()
            torch.index_select(inputs, 0, sel, out=xb[:b])
            torch.index_select(ts.targets, 0, sel, out=tb[:b])
            cur = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * step / max(1, total - 1)))
            ep_loss += net.train_step(xb[:b].view(-1), tb[:b].view(-1), b, cur) * b
            step += 1
        hist.append(ep_loss / nset)
        if log and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
            log(f"[train] epoch {ep} loss {hist[-1]:.3e} lr {cur:.2e}")
    torch.cuda.synchronize()
    return net, hist, time.perf_counter() - t0


def guess(ctx, net, norm: Normalization, Gr, X, X_near=None, Gr_near=None, smooth_sigma=None,
          restore_sigma=None):
    """Learned initial guess at Gr on ctx's grid, projected, into X (packed,
    float64 CUDA).
      direct    (X_near None): the interpolated prediction at Gr;
      increment (X_near, Gr_near given): the converged state X_near moved by
                the predicted change between Gr_near and Gr,
                X = X_near + S(NN(Gr)) - S(NN(Gr_near)); the network's error
                common to both predictions cancels.
    smooth_sigma (increment only): the change is low-pass filtered first,
    D <- sigma M^-1 D with the Stokes/heat operator M = sigma - nu Lap
    (factor sigma / (sigma + nu lambda) on a diffusion mode lambda): the
    network's grid-scale error, which the 1/h^2 terms of the residual
    amplify in thin wall cells, is damped, smooth changes pass.  The
    context's preconditioner is set to restore_sigma afterwards (None: off)."""
    import torch
    r = net.res
    out = torch.empty(4 * r ** 3, dtype=torch.float32, device="cuda")
    net.predict(Gr, out)
    if X_near is None:
        ctx.state_from_cells(out, net.centres, norm.shift, norm.scale, X)
    else:
        ref = torch.empty_like(out)
        net.predict(Gr_near, ref)
        if smooth_sigma is None:
            X.copy_(X_near)
            ctx.state_add_cell_increment(out, ref, net.centres, norm.scale, X)
        else:
            D = torch.zeros_like(X)
            ctx.state_add_cell_increment(out, ref, net.centres, norm.scale, D)
            ctx.set_preconditioner(True, smooth_sigma)
            ctx.apply_preconditioner(D, D)
            if restore_sigma is None:
                ctx.set_preconditioner(False)
            else:
                ctx.set_preconditioner(True, restore_sigma)
            X.copy_(X_near)
            ctx.axpby(smooth_sigma, D, 1.0, X)
    ctx.project(X)
    return X


START_KINDS = ("continuation", "learned", "learned_increment")


def compare_starts(faces, Gr, X_near, Gr_near, net, norm, Pr=0.71, tol_abs=1e-10, max_iter=20,
                   max_matvec=40000, kinds=START_KINDS, precond_sigma=None, smooth_sigmas=(), log=None):
    """Newton at Gr from the nearest converged state (continuation), from the
    direct learned guess and from the learned increment, each to the same
    absolute residual tolerance.  Returns a record per start (iterations,
    matvecs, residual history, seconds including building the guess) and
    the largest distance between the converged states."""
    import torch
    res = {}
    ctx = kv.Context(*faces, Gr=Gr, Pr=Pr)
    finals = []
    try:
        if precond_sigma is not None:
            ctx.set_preconditioner(True, precond_sigma)
        for kind in list(kinds) + [f"learned_increment_smooth{sg:g}" for sg in smooth_sigmas]:
            X = torch.empty_like(X_near)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if kind == "continuation":
                X.copy_(X_near)
                ctx.project(X)
            elif kind == "learned":
                guess(ctx, net, norm, Gr, X)
            elif kind == "learned_increment":
                guess(ctx, net, norm, Gr, X, X_near=X_near, Gr_near=Gr_near)
            else:
                sg = float(kind[len("learned_increment_smooth"):])
                guess(ctx, net, norm, Gr, X, X_near=X_near, Gr_near=Gr_near, smooth_sigma=sg,
                      restore_sigma=precond_sigma)
            torch.cuda.synchronize()
            tg = time.perf_counter() - t0
            rec = newton_solve(ctx, X, tol_rel=0.0, tol_abs=tol_abs, max_iter=max_iter, max_matvec=max_matvec)
            rec["guess_seconds"] = tg
            rec["seconds"] += tg
            res[kind] = rec
            finals.append(X)
            if log:
                log(f"[compare] Gr={Gr:.4e} {kind:18s} converged={rec['converged']} iters={rec['iters']} "
                    f"matvecs={rec['matvecs']} |F0|={rec['hist'][0]:.3e} {rec['seconds']:.2f}s")
        ref = finals[0]
        nref = max(1e-300, ctx.dot(ref, ref))
        dist = 0.0
        for X in finals[1:]:
            d = X - ref
            dist = max(dist, math.sqrt(max(0.0, ctx.dot(d, d)) / nref))
        res["state_distance"] = dist
    finally:
        ctx.close()
    return res


def guess_residual(faces, Gr, X, Pr=0.71):
    """||P N(X)||_W at Gr (the Newton residual that judges a guess)."""
    import torch
    ctx = kv.Context(*faces, Gr=Gr, Pr=Pr)
    try:
        ctx.set_base_flow(X)
        F = torch.empty_like(X)
        return ctx.residual(F)
    finally:
        ctx.close()


def experiment(n=64, grid="clustered", factor=2, gr_lo=1e6, log_step=None, ntrain=15, held=(1, 4, 7, 10, 13),
               epochs=6000, lr=1e-3, lr_final=1e-5, batch=2, precond_sigma=10.0, seed=3, data_seed=4,
               tol_abs=1e-10, smooth_sigmas=(), log=print):
    """Training states by continuation (from the conduction state, Gr raised
    by 1.6 per step up to gr_lo, then the training values
    Gr_i = gr_lo 10^(i log_step)), network training, and Newton from three
    starts at the held-out values Gr = gr_lo 10^((i + 1/2) log_step).
    Returns a dict of everything measured."""
    import torch
    from synth import inputs as S  # seeded grid faces (input construction only)
    f = S.faces_uniform(n) if grid == "uniform" else S.faces_clustered(n)
    faces = (f, f, f)
    log_step = log_step if log_step is not None else math.log10(300.0) / 23.0
    train_grs = [gr_lo * 10 ** (i * log_step) for i in range(ntrain)]
    held = [i for i in held if i + 1 < ntrain]
    pre = []
    g = 1e4
    while g < gr_lo:
        pre.append(g)
        g *= 1.6
    t0 = time.perf_counter()
    states, infos = sweep(faces, pre + train_grs, max_matvec=20000, max_iter=20, precond_sigma=precond_sigma,
                          log=log)
    t_cont = time.perf_counter() - t0
    if len(states) < len(pre) + len(train_grs):
        raise RuntimeError("continuation did not reach every training value")
    states = states[len(pre):]
    mv_cont = sum(i["matvecs_all_attempts"] for i in infos)
    ts = build_training_set(faces, train_grs, states, factor)
    lgr = (math.log10(train_grs[0]), math.log10(train_grs[-1]))
    net, hist, t_train = train(ts, lgr, epochs=epochs, batch=batch, lr=lr, lr_final=lr_final, seed=seed,
                               data_seed=data_seed, log=log)
    out = dict(grid=f"{n}^3 {grid}", network=f"{net.res}^3", factor=factor, train_gr=train_grs,
               continuation_seconds=t_cont, continuation_matvecs=mv_cont, train_seconds=t_train,
               epochs=epochs, final_loss=hist[-1], precond_sigma=precond_sigma, held_out=[])
    cond = torch.from_numpy(_conduction_state(*faces)).cuda()
    for i in held:
        gr = gr_lo * 10 ** ((i + 0.5) * log_step)
        r = compare_starts(faces, gr, states[i], train_grs[i], net, ts.norm, tol_abs=tol_abs,
                           precond_sigma=precond_sigma, smooth_sigmas=smooth_sigmas, log=log)
        rec = {"Gr": gr, "nearest_Gr": train_grs[i], "state_distance": r["state_distance"],
               "conduction_F0": guess_residual(faces, gr, cond)}
        for k in [k for k in r if k != "state_distance"]:
            v = r[k]
            rec[k] = {"converged": v["converged"], "iters": v["iters"], "matvecs": v["matvecs"],
                      "F0": v["hist"][0], "seconds": round(v["seconds"], 3), "hist": v["hist"]}
        out["held_out"].append(rec)
    return out


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="learned Newton guess vs continuation (held-out Gr)")
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--grid", choices=("uniform", "clustered"), default="clustered")
    ap.add_argument("--factor", type=int, default=2)
    ap.add_argument("--ntrain", type=int, default=15)
    ap.add_argument("--epochs", type=int, default=6000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=2)
    ap.add_argument("--sigma", type=float, default=10.0, help="preconditioner shift (negative: none)")
    ap.add_argument("--smooth", default="", help="comma-separated smoothing shifts of the learned increment")
    ap.add_argument("--held", default="1,4,7,10,13",
                    help="comma-separated i: held-out values Gr_lo 10^((i + 1/2) step)")
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    sm = tuple(float(v) for v in a.smooth.split(",") if v)
    held = tuple(int(v) for v in a.held.split(",") if v)
    res = experiment(n=a.n, grid=a.grid, factor=a.factor, ntrain=a.ntrain, held=held, epochs=a.epochs, lr=a.lr,
                     batch=a.batch, precond_sigma=None if a.sigma < 0 else a.sigma, smooth_sigmas=sm,
                     log=lambda m: print(m, flush=True))
    text = json.dumps(res)
    if a.json:
        with open(a.json, "w") as fh:
            fh.write(text + "\n")
    print(text, flush=True)


if __name__ == "__main__":
    main()

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
from .continuation import newton_solve


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


def guess(ctx, net, norm: Normalization, Gr, X, X_near=None, Gr_near=None):
    """Learned initial guess at Gr on ctx's grid, projected, into X (packed,
    float64 CUDA).
      direct    (X_near None): the interpolated prediction at Gr;
      increment (X_near, Gr_near given): the converged state X_near moved by
                the predicted change between Gr_near and Gr,
                X = X_near + S(NN(Gr)) - S(NN(Gr_near)); the network's error
                common to both predictions cancels."""
    import torch
    r = net.res
    out = torch.empty(4 * r ** 3, dtype=torch.float32, device="cuda")
    net.predict(Gr, out)
    if X_near is None:
        ctx.state_from_cells(out, net.centres, norm.shift, norm.scale, X)
    else:
        ref = torch.empty_like(out)
        net.predict(Gr_near, ref)
        X.copy_(X_near)
        ctx.state_add_cell_increment(out, ref, net.centres, norm.scale, X)
    ctx.project(X)
    return X


START_KINDS = ("continuation", "learned", "learned_increment")


def compare_starts(faces, Gr, X_near, Gr_near, net, norm, Pr=0.71, tol_abs=1e-10, max_iter=20,
                   max_matvec=40000, kinds=START_KINDS, log=None):
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
        for kind in kinds:
            X = torch.empty_like(X_near)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if kind == "continuation":
                X.copy_(X_near)
                ctx.project(X)
            elif kind == "learned":
                guess(ctx, net, norm, Gr, X)
            else:
                guess(ctx, net, norm, Gr, X, X_near=X_near, Gr_near=Gr_near)
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

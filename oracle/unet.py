"""CPU oracle, part 3: the learned Newton guess network, in FP64.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library's product path.

Not from the paper.  The paper reaches steady states at large Gr by Newton
continuation from a converged state at a nearby Gr (Sec. 1); the library adds
a small 3-D U-Net that predicts the state at a given Gr, as a Newton initial
guess.  This module is the plain definition of that network, its loss, its
gradient and one Adam step (Kingma and Ba, "Adam: a method for stochastic
optimization", 2015, Algorithm 1), in float64 on the CPU:

  conv3    3x3x3 cross-correlation, zero padding 1, plus bias, then ReLU
  pool     mean of each 2x2x2 block
  up       nearest-neighbour 2x upsampling
  network  e1 = conv3(conv3(x))            4 -> 16 -> 16 channels, r^3
           e2 = conv3(conv3(pool(e1)))     16 -> 32 -> 32,        (r/2)^3
           e3 = conv3(conv3(pool(e2)))     32 -> 64 -> 64,        (r/4)^3
           d2 = conv3(conv3([up(e3), e2])) 96 -> 32 -> 32
           d1 = conv3(conv3([up(d2), e1])) 48 -> 16 -> 16
           out = conv1(d1)                 16 -> 4, no ReLU
  loss     mean over all values of (out - target)^2
The convolutions use the weights rounded to bfloat16 (round to nearest, ties
to even); the gradient is taken with respect to those rounded weights and
applied to the unrounded master copy.

torch's CPU conv3d, avg_pool3d and autograd serve as library primitives: the
convolution is pinned against a brute-force loop, the gradient against
finite differences and Adam against its closed form for a constant gradient.
"""
from __future__ import annotations

import numpy as np

# (ci, co, kernel size) of the 11 convolutions, in parameter order
CONVS = [(4, 16, 3), (16, 16, 3), (16, 32, 3), (32, 32, 3), (32, 64, 3), (64, 64, 3),
         (96, 32, 3), (32, 32, 3), (48, 16, 3), (16, 16, 3), (16, 4, 1)]


def num_params() -> int:
    return sum(co * ci * k ** 3 + co for ci, co, k in CONVS)


def bf16_round(w: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as
    float32: keep the upper 16 bits of the IEEE single after adding half an
    ulp of bfloat16 plus the tie-breaking bit."""
    a = np.ascontiguousarray(np.asarray(w, dtype=np.float32))
    b = a.view(np.uint32).astype(np.uint64)
    finite = (b & 0x7F800000) != 0x7F800000
    r = ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    out = np.where(finite, r, b.astype(np.uint32)).astype(np.uint32)
    return out.view(np.float32).reshape(a.shape)


def split_params(w):
    """Parameter vector -> list of (weight [co, ci, k, k, k], bias [co])."""
    out, o = [], 0
    for ci, co, k in CONVS:
        n = co * ci * k ** 3
        W = w[o:o + n].reshape(co, ci, k, k, k)
        o += n
        b = w[o:o + co]
        o += co
        out.append((W, b))
    assert o == len(w)
    return out


def forward(w, x):
    """Network output for parameters w (torch float64, already rounded as
    wanted) and inputs x (torch float64 [B, 4, r, r, r])."""
    import torch
    import torch.nn.functional as F
    p = split_params(w)

    def conv(i, t, relu=True):
        W, b = p[i]
        y = F.conv3d(t, W, b, padding=W.shape[-1] // 2)
        return torch.relu(y) if relu else y

    def up(t):
        return t.repeat_interleave(2, dim=2).repeat_interleave(2, dim=3).repeat_interleave(2, dim=4)

    e1 = conv(1, conv(0, x))
    e2 = conv(3, conv(2, F.avg_pool3d(e1, 2)))
    e3 = conv(5, conv(4, F.avg_pool3d(e2, 2)))
    d2 = conv(7, conv(6, torch.cat([up(e3), e2], dim=1)))
    d1 = conv(9, conv(8, torch.cat([up(d2), e1], dim=1)))
    return conv(10, d1, relu=False)


def output(params_f32, x):
    """Forward pass with bfloat16-rounded weights, in float64 (numpy in/out)."""
    import torch
    w = torch.from_numpy(bf16_round(params_f32).astype(np.float64))
    with torch.no_grad():
        return forward(w, torch.from_numpy(np.asarray(x, dtype=np.float64))).numpy()


def grad_of_dot(params_f32, x, gout):
    """Gradient of sum(output * gout) with respect to the (rounded) weights."""
    import torch
    w = torch.from_numpy(bf16_round(params_f32).astype(np.float64)).requires_grad_(True)
    y = forward(w, torch.from_numpy(np.asarray(x, dtype=np.float64)))
    (y * torch.from_numpy(np.asarray(gout, dtype=np.float64))).sum().backward()
    return w.grad.numpy()


def mse_loss_and_grad(params_f32, x, target):
    """loss = mean (out - target)^2 and its gradient with respect to the weights."""
    import torch
    w = torch.from_numpy(bf16_round(params_f32).astype(np.float64)).requires_grad_(True)
    y = forward(w, torch.from_numpy(np.asarray(x, dtype=np.float64)))
    loss = ((y - torch.from_numpy(np.asarray(target, dtype=np.float64))) ** 2).mean()
    loss.backward()
    return float(loss.detach()), w.grad.numpy()


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step at step number t (1-based): returns (w, m, v) updated."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** t)
    vhat = v / (1 - b2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


def make_inputs(centres, lgr_range, grs):
    """Inputs [B, 4, r, r, r]: 2c - 1 per axis and (log10 Gr - m) / s."""
    xc, yc, zc = (np.asarray(c, dtype=np.float64) for c in centres)
    r = len(xc)
    lo, hi = lgr_range
    m, s = 0.5 * (lo + hi), 0.5 * (hi - lo)
    out = np.empty((len(grs), 4, r, r, r))
    for b, gr in enumerate(grs):
        out[b, 0] = (2 * xc - 1)[None, None, :]
        out[b, 1] = (2 * yc - 1)[None, :, None]
        out[b, 2] = (2 * zc - 1)[:, None, None]
        out[b, 3] = (np.log10(gr) - m) / s
    return out

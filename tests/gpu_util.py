"""Helpers shared by the GPU parity tests (input construction, comparisons)."""
import numpy as np
import torch

from synth import inputs as S


def faces(kind, n):
    return S.faces_uniform(n) if kind == "uniform" else S.faces_clustered(n)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def field_rel_errors(g, got, ref):
    """||got_f - ref_f||_2 / ||ref_f||_2 per block u, v, w, T."""
    out = []
    for a, b in zip(g.unpack(got), g.unpack(ref)):
        nb = np.linalg.norm(b)
        out.append(np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a))
    return out

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


def _interior(a):
    """The unknowns of a block at least a quarter of each extent away from
    every wall (empty on blocks thinner than 4 in some direction)."""
    sl = tuple(slice(s // 4, s - s // 4) for s in a.shape)
    return a[sl]


def parity_errors(g, got, ref):
    """Per field u, v, w, T: 'l2' = ||got - ref||_2 / ||ref||_2; 'max' =
    max_i |got_i - ref_i| / max_i |ref_i| (element by element); 'interior' =
    the relative 2-norm over the central unknowns (_interior).  On the
    wall-clustered grids the wall unknowns of P J x reach 1e5 while the
    interior ones are O(1), so the whole-field norms are wall dominated and
    the interior norm is what sees an error confined to the bulk."""
    out = {"l2": [], "max": [], "interior": []}
    for a, b in zip(g.unpack(got), g.unpack(ref)):
        d = a - b
        nb, mb = np.linalg.norm(b), np.max(np.abs(b)) if b.size else 0.0
        out["l2"].append(np.linalg.norm(d) / nb if nb > 0 else np.linalg.norm(d))
        out["max"].append(np.max(np.abs(d)) / mb if mb > 0 else (np.max(np.abs(d)) if d.size else 0.0))
        ai, bi = _interior(a), _interior(b)
        ni = np.linalg.norm(bi)
        out["interior"].append(np.linalg.norm(ai - bi) / ni if ni > 0 else np.linalg.norm(ai - bi))
    return out


def assert_parity(g, got, ref, tol, tol_interior=None, label=""):
    """Element-wise parity gate: every field within tol in the relative
    2-norm and in the largest element error, and its central unknowns within
    tol_interior (default 10 tol) in the relative 2-norm."""
    e = parity_errors(g, got, ref)
    ti = 10.0 * tol if tol_interior is None else tol_interior
    print(f"parity {label}: l2 {max(e['l2']):.3e} max {max(e['max']):.3e} "
          f"interior {max(e['interior']):.3e}", flush=True)
    assert max(e["l2"]) <= tol, e
    assert max(e["max"]) <= tol, e
    assert max(e["interior"]) <= ti, e
    return e

"""CPU oracle, part 4: transfers between the staggered state and cell-centred
fields on a network grid (learned Newton guess; not from the paper).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library's product path.

cells_from_state(g, X, f, shift, scale)
    Per fine cell the centre values u = (u_west + u_east)/2 (walls carry 0),
    likewise v and w, and theta = T - (1/2 - x_c), the deviation from the
    conduction profile (Sec. 2: T = 1/2 - x in the centred temperature).
    Each coarse cell (f^3 fine cells) takes the volume-weighted mean; the
    output is (mean - shift[c]) / scale[c], channels u, v, w, theta.
state_from_cells(g, cells, centres, shift, scale)
    Every unknown of the packed state becomes the trilinear interpolant, in
    physical coordinates, at its own position (faces for velocities, centres
    for T) of the values shift + scale * cells at the network centres, with
    the node set extended by the walls 0 and 1 per axis: velocities vanish on
    all walls (no slip, Eq. 3); theta vanishes on the x-walls, where T is
    fixed (Eq. 4); on the adiabatic y- and z-walls (Eqs. 5-6) theta takes the
    value of the adjacent cell.  T = theta + 1/2 - x_c.
"""
from __future__ import annotations

import numpy as np

from . import disc


def centre_fields(g: disc.Grid, X):
    """(u, v, w, theta) at the cell centres of g, each (nz, ny, nx)."""
    u, v, w, T = g.unpack(np.asarray(X, dtype=np.float64))
    nx, ny, nz = g.n
    U = np.zeros((nz, ny, nx + 1))
    U[:, :, 1:nx] = u
    V = np.zeros((nz, ny + 1, nx))
    V[:, 1:ny, :] = v
    W = np.zeros((nz + 1, ny, nx))
    W[1:nz, :, :] = w
    uc = 0.5 * (U[:, :, :-1] + U[:, :, 1:])
    vc = 0.5 * (V[:, :-1, :] + V[:, 1:, :])
    wc = 0.5 * (W[:-1, :, :] + W[1:, :, :])
    theta = T - (0.5 - g.c[0])[None, None, :]
    return uc, vc, wc, theta


def cells_from_state(g: disc.Grid, X, f, shift, scale):
    nx, ny, nz = g.n
    assert nx % f == 0 and ny % f == 0 and nz % f == 0
    vol = g.h[2][:, None, None] * g.h[1][None, :, None] * g.h[0][None, None, :]

    def block_sum(a):
        return a.reshape(nz // f, f, ny // f, f, nx // f, f).sum(axis=(1, 3, 5))

    vsum = block_sum(vol)
    out = []
    for c, fld in enumerate(centre_fields(g, X)):
        mean = block_sum(vol * fld) / vsum
        out.append((mean - shift[c]) / scale[c])
    return np.stack(out)


def _interp_1d(nodes, s):
    """For positions s: the lower node index q (q <= len(nodes) - 2) and the
    weight t of node q + 1 of linear interpolation."""
    q = np.clip(np.searchsorted(nodes, s, side="right") - 1, 0, len(nodes) - 2)
    t = (s - nodes[q]) / (nodes[q + 1] - nodes[q])
    return q, np.clip(t, 0.0, 1.0)


def _extended(cells_c, channel):
    """Channel values on the node set extended by the walls, (rz+2, ry+2, rx+2)."""
    rz, ry, rx = cells_c.shape
    E = np.zeros((rz + 2, ry + 2, rx + 2))
    if channel < 3:
        E[1:-1, 1:-1, 1:-1] = cells_c
        return E
    # theta: y and z walls copy the adjacent cell, x walls stay 0
    inner = np.pad(cells_c, ((1, 1), (1, 1), (0, 0)), mode="edge")
    E[:, :, 1:-1] = inner
    return E


def state_from_cells(g: disc.Grid, cells, centres, shift, scale):
    cells = np.asarray(cells, dtype=np.float64)
    nodes = [np.concatenate([[0.0], np.asarray(c, dtype=np.float64), [1.0]]) for c in centres]
    fields = []
    for ch in range(4):
        E = _extended(shift[ch] + scale[ch] * cells[ch], ch)
        # positions of the unknowns of this channel: faces along its own axis
        pos = []
        for a in range(3):
            if ch < 3 and a == ch:
                pos.append(g.faces[a][1:-1])   # interior faces
            else:
                pos.append(g.c[a])
        (qx, tx), (qy, ty), (qz, tz) = (_interp_1d(nodes[a], pos[a]) for a in range(3))
        val = np.zeros((len(pos[2]), len(pos[1]), len(pos[0])))
        for dz in (0, 1):
            wz = tz if dz else 1 - tz
            for dy in (0, 1):
                wy = ty if dy else 1 - ty
                for dx in (0, 1):
                    wx = tx if dx else 1 - tx
                    val += (wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
                            * E[np.ix_(qz + dz, qy + dy, qx + dx)])
        if ch == 3:
            val = val + (0.5 - g.c[0])[None, None, :]
        fields.append(val)
    return g.pack(fields)


def add_cell_increment(g: disc.Grid, X, cells, cells_ref, centres, scale):
    """X + S(cells) - S(cells_ref), S = state_from_cells (shift and the
    conduction profile cancel in the difference)."""
    zero = np.zeros(4)
    return (np.asarray(X, dtype=np.float64) + state_from_cells(g, cells, centres, zero, scale)
            - state_from_cells(g, cells_ref, centres, zero, scale))

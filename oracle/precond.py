"""CPU oracle, part 5: the Stokes/heat preconditioner of the Newton solve.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library's product path.

Not a statement of the paper, which does not describe its linear solver
beyond BiCGstab(2) with GMRES (Sec. 1, with refs [21], [22] absent).  The
library offers, as an option, right preconditioning of P J by

    M^-1 r = ( P H_nu^-1 r_vel ,  H_kappa^-1 r_T ),
    H_nu    = sigma I - nu    Lap_v   (each velocity component, no-slip walls),
    H_kappa = sigma I - kappa Lap_T   (T = 0 on the x-walls, adiabatic y, z),

with Lap_v and Lap_T the diffusion operators of the discretization itself
(oracle/disc.py: _vel_diffusion and _temp_diffusion with homogeneous wall
values), in the manner of Stokes preconditioning (Tuckerman, "Steady-state
solving via Stokes preconditioning", 1989).  Every Lap is a sum over axes of
1-D operators H_a^-1 K_a (H diagonal widths, K symmetric), so H_nu^-1 is
applied by eigen-decomposing each 1-D operator (numpy eigh): for the
component on its own axis the 1-D operator lives on the interior faces
(widths = centre gaps, fluxes over cell widths, zero wall values); across
axes it lives on the centres (walls at half-cell distance, value 0); T's y
and z operators are the Neumann ones of the pressure Laplacian.
"""
from __future__ import annotations

import numpy as np

from . import disc


def stiffness_1d(g: disc.Grid, a, kind):
    """(K, widths) of the 1-D operator -(H^-1 K) along axis a.
    kind: 'cN' centres, zero-flux walls; 'cD' centres, zero value at the walls
    (half-cell distance); 'fD' interior faces, zero value at the wall faces."""
    h, d = g.h[a], g.d[a]
    n = len(h)
    if kind in ("cN", "cD"):
        K = -disc.laplacian_1d(g, a)
        if kind == "cD":
            K[0, 0] += 1.0 / d[0]
            K[n - 1, n - 1] += 1.0 / d[n]
        return K, h.copy()
    if kind == "fD":
        m = n - 1
        K = np.zeros((m, m))
        for i in range(m):              # face i + 1 lies between cells i and i + 1
            K[i, i] = 1.0 / h[i] + 1.0 / h[i + 1]
            if i + 1 < m:
                K[i, i + 1] = K[i + 1, i] = -1.0 / h[i + 1]
        return K, d[1:-1].copy()
    raise ValueError(kind)


def kinds_of(block):
    """1-D operator kind per axis (x, y, z) of a packed block (0..2 velocity, 3 T)."""
    if block == 3:
        return ("cD", "cN", "cN")
    return tuple("fD" if a == block else "cD" for a in range(3))


def helmholtz_solve(g: disc.Grid, block, r, sigma, coef):
    """z with (sigma - coef * Lap) z = r for one packed block, r shaped (nz, ny, nx)."""
    Q, lam, s = [], [], []
    for a, kind in enumerate(kinds_of(block)):
        K, H = stiffness_1d(g, a, kind)
        sh = np.sqrt(H)
        M = K / sh[:, None] / sh[None, :]
        w, V = np.linalg.eigh(M)
        Q.append(V)
        lam.append(np.maximum(w, 0.0))
        s.append(sh)
    S = s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]
    t = np.einsum("kji,ia,jb,kc->cba", S * r, Q[0], Q[1], Q[2], optimize=True)
    den = sigma + coef * (lam[2][:, None, None] + lam[1][None, :, None] + lam[0][None, None, :])
    t = t / den
    z = np.einsum("cba,ia,jb,kc->kji", t, Q[0], Q[1], Q[2], optimize=True)
    return z / S


def apply(g: disc.Grid, r, sigma):
    """M^-1 r for the packed vector r (see the module docstring)."""
    blocks = g.unpack(np.asarray(r, dtype=np.float64))
    out = [helmholtz_solve(g, b, blocks[b], sigma, g.nu) for b in range(3)]
    out.append(helmholtz_solve(g, 3, blocks[3], sigma, g.kappa))
    z = g.pack(out)
    return disc.project(g, z)

"""Seeded synthetic inputs for the cube-convection Krylov-vector path.

This module builds the *inputs* of the method only: face coordinates of the
grid, a base flow X0 and random perturbations x, all in the packed layout
[u | v | w | T] that both the HIP library and the CPU oracle accept.  It holds
none of the method's arithmetic (no stencil, no projection, no solver); both
sides receive the same arrays from here.

Grids (paper Sec. 4.1: 100^3 ... 256^3 finite volumes, stretched near the
walls).  The stretched grid uses x_i = (1 - cos(pi i / N)) / 2 per axis; the
uniform grid x_i = i / N.  Both are made exactly mirror-symmetric
(x_{N-i} = 1 - x_i in floating point) so that the cube's symmetries
(Sec. 2, reflection / 2-D rotation / centro-symmetry) hold to round-off.

Packed layout (x fastest, then y, then z):
    u at x-faces i = 1..nx-1, cell rows (j, k):  shape (nz, ny, nx-1)
    v at y-faces j = 1..ny-1:                     shape (nz, ny-1, nx)
    w at z-faces k = 1..nz-1:                     shape (nz-1, ny, nx)
    T at cell centres:                            shape (nz, ny, nx)
Wall-normal velocities are zero and not stored.  T is the centred
temperature T - 1/2 (walls at +1/2 for x = 0 and -1/2 for x = 1, Eq. 4).

Base flow recipe: velocity = discrete curl of a vector potential A whose
components are seeded N(0,1) combinations of sin-product modes of wavenumber
<= K (they vanish on every wall), scaled by `amp`; T0 = 1/2 - x at cell
centres (the conduction profile, Eq. 4 shifted by 1/2).  The discrete curl
gives a velocity whose discrete divergence is zero to round-off.
"""
from __future__ import annotations

import numpy as np


def faces_uniform(n: int) -> np.ndarray:
    """Uniform faces x_i = i/n, i = 0..n."""
    x = np.arange(n + 1, dtype=np.float64) / n
    return _mirror(x)


def faces_clustered(n: int) -> np.ndarray:
    """Wall-clustered faces x_i = (1 - cos(pi i / n)) / 2, i = 0..n."""
    i = np.arange(n + 1, dtype=np.float64)
    x = 0.5 * (1.0 - np.cos(np.pi * i / n))
    return _mirror(x)


def _mirror(x: np.ndarray) -> np.ndarray:
    """Make the faces exactly mirror-symmetric in floating point.

    The lower half is rounded to multiples of 2^-53, so 1 - x_i is exact and
    every width h_i = x_{i+1} - x_i equals its mirror image h_{N-1-i}
    bit for bit (both differences are exact).  The change is below 1.2e-16.
    """
    n = len(x) - 1
    x = np.round(x * 2.0 ** 53) / 2.0 ** 53
    x[0], x[n] = 0.0, 1.0
    for i in range(n // 2 + 1, n + 1):
        x[i] = 1.0 - x[n - i]
    if n % 2 == 0:
        x[n // 2] = 0.5
    return x


def layout(nx: int, ny: int, nz: int):
    """Shapes and offsets of the packed [u|v|w|T] vector."""
    shapes = [(nz, ny, nx - 1), (nz, ny - 1, nx), (nz - 1, ny, nx), (nz, ny, nx)]
    sizes = [int(np.prod(s)) for s in shapes]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return shapes, offs


def packed_size(nx: int, ny: int, nz: int) -> int:
    return int(layout(nx, ny, nz)[1][-1])


def unpack(X: np.ndarray, nx: int, ny: int, nz: int):
    shapes, offs = layout(nx, ny, nz)
    return [X[offs[a]:offs[a + 1]].reshape(shapes[a]) for a in range(4)]


def pack(fields) -> np.ndarray:
    return np.concatenate([np.ascontiguousarray(f).ravel() for f in fields])


def _sin_modes(pts: np.ndarray, K: int) -> np.ndarray:
    """S[m-1, p] = sin(m pi pts[p]), m = 1..K."""
    m = np.arange(1, K + 1, dtype=np.float64)[:, None]
    return np.sin(np.pi * m * pts[None, :])


def base_flow(xf, yf, zf, K: int, amp: float, seed: int) -> np.ndarray:
    """Seeded base flow X0 = (curl A, T0) in the packed layout.

    A_c = amp * sum_{a,b,c=1..K} g[c,a,b,c'] sin(a pi x) sin(b pi y) sin(c' pi z),
    g ~ N(0,1) drawn as standard_normal((3, K, K, K)) from default_rng(seed),
    index order (component, x-wavenumber, y-wavenumber, z-wavenumber).
    A_x is sampled on x-edges (c_i, y_j, z_k), A_y on y-edges (x_i, c_j, z_k)
    and A_z on z-edges (x_i, y_j, c_k); the velocity is their discrete curl.
    """
    xf, yf, zf = (np.asarray(a, dtype=np.float64) for a in (xf, yf, zf))
    nx, ny, nz = len(xf) - 1, len(yf) - 1, len(zf) - 1
    g = np.random.default_rng(seed).standard_normal((3, K, K, K))
    hx, hy, hz = np.diff(xf), np.diff(yf), np.diff(zf)
    cx, cy, cz = (xf[:-1] + xf[1:]) / 2, (yf[:-1] + yf[1:]) / 2, (zf[:-1] + zf[1:]) / 2

    def sample(coef, px, py, pz):
        # returns array indexed [z, y, x]
        return amp * np.einsum("abc,ai,bj,ck->kji", coef,
                               _sin_modes(px, K), _sin_modes(py, K), _sin_modes(pz, K),
                               optimize=True)

    Ax = sample(g[0], cx, yf, zf)   # (nz+1, ny+1, nx)
    Ay = sample(g[1], xf, cy, zf)   # (nz+1, ny, nx+1)
    Az = sample(g[2], xf, yf, cz)   # (nz, ny+1, nx+1)

    # u on all x-faces (nz, ny, nx+1); wall entries vanish because A does
    u = (np.diff(Az, axis=1) / hy[None, :, None]) - (np.diff(Ay, axis=0) / hz[:, None, None])
    v = (np.diff(Ax, axis=0) / hz[:, None, None]) - (np.diff(Az, axis=2) / hx[None, None, :])
    w = (np.diff(Ay, axis=2) / hx[None, None, :]) - (np.diff(Ax, axis=1) / hy[None, :, None])
    u = u[:, :, 1:nx]
    v = v[:, 1:ny, :]
    w = w[1:nz, :, :]
    T = np.broadcast_to((0.5 - cx)[None, None, :], (nz, ny, nx))
    return pack([u, v, w, T])


def conduction_state(xf, yf, zf) -> np.ndarray:
    """Zero velocity and T0 = 1/2 - x at cell centres (packed)."""
    xf = np.asarray(xf, dtype=np.float64)
    nx, ny, nz = len(xf) - 1, len(yf) - 1, len(zf) - 1
    shapes, offs = layout(nx, ny, nz)
    X = np.zeros(int(offs[-1]))
    cx = (xf[:-1] + xf[1:]) / 2
    X[offs[3]:] = np.broadcast_to((0.5 - cx)[None, None, :], (nz, ny, nx)).ravel()
    return X


def perturbation(n: int, seed: int) -> np.ndarray:
    """x ~ N(0,1)^n from default_rng(seed), drawn in packed order."""
    return np.random.default_rng(seed).standard_normal(n)


# Named workloads (grid, Gr, Pr, base-flow recipe); each is a plain dict so
# both sides and the bench can build the same inputs.
WORKLOADS = {
    "cube32_uniform_gr1e5": dict(n=32, grid="uniform", Gr=1e5, Pr=0.71, K=3, amp=0.05, base_seed=0),
    "cube100_clustered_gr4e7": dict(n=100, grid="clustered", Gr=4e7, Pr=0.71, K=6, amp=0.1, base_seed=1),
    "cube256_clustered_gr2e8": dict(n=256, grid="clustered", Gr=2e8, Pr=0.71, K=6, amp=0.1, base_seed=2),
}


def workload_grid(spec: dict):
    n = spec["n"]
    f = faces_uniform(n) if spec["grid"] == "uniform" else faces_clustered(n)
    return f, f.copy(), f.copy()

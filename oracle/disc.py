"""CPU oracle, part 1: the discrete Boussinesq operator on a staggered grid.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, FP64 reference
that the HIP library is checked against.  Only tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.

What is computed (paper Sec. 2, Eqs. 1-6, with the paper's scaling):
    dT/dt + (v.grad)T = kappa Lap T,            kappa = 1 / (Pr Gr^1/2)
    dv/dt + (v.grad)v = -grad p + nu Lap v + beta T e_z,   nu = Gr^-1/2, beta = 1
    div v = 0,
no-slip on all walls, T = 1 at x = 0 and T = 0 at x = 1 (Eq. 4), adiabatic
y- and z-walls (Eqs. 5-6).  T is carried as the centred temperature
T_c = T - 1/2 (an exact hydrostatic shift of p), so the x-walls hold +-1/2.
Gr = 0 selects the viscous scaling nu = 1, kappa = 1/Pr, beta = 0.

The paper gives only "finite volume, grids stretched near the walls" (Sec. 3,
Sec. 4.1) and defers the scheme to its earlier work; the reading taken here is
the second-order conservative staggered (MAC) finite-volume scheme:
  * faces x_0 = 0 < ... < x_N = 1 per axis, widths h_i, centres c_i at the
    midpoints, centre gaps d_i = c_i - c_{i-1}, wall gaps d_0 = h_0/2,
    d_N = h_{N-1}/2;
  * u on x-faces, v on y-faces, w on z-faces, T and p at centres;
  * centre-to-face values by distance-linear interpolation, face-to-centre
    values by the two-face average (exact at the midpoint);
  * conservative convective fluxes, two-point diffusive fluxes, wall values
    imposed at half-cell distance.
N(X) is the steady right-hand side without the pressure term; the pressure is
handled by the discrete Leray projection P = I - G L^+ D, which gives the
divergence-free Krylov vectors that meet every boundary condition (Sec. 3).

Arrays are numpy (z, y, x) with x fastest, i.e. the packed layout of synth.
"""
from __future__ import annotations

import numpy as np


class Grid:
    """Per-axis metrics of a tensor-product grid on the unit cube (axis 0 = x)."""

    def __init__(self, xf, yf, zf, Gr: float, Pr: float):
        self.faces = [np.asarray(a, dtype=np.float64).copy() for a in (xf, yf, zf)]
        self.n = [len(f) - 1 for f in self.faces]
        self.h, self.c, self.d, self.wlo, self.whi = [], [], [], [], []
        for f in self.faces:
            h = np.diff(f)
            c = 0.5 * (f[:-1] + f[1:])
            d = np.empty(len(f))
            d[0], d[-1] = 0.5 * h[0], 0.5 * h[-1]
            # centres are midpoints, so c_i - c_{i-1} = (h_{i-1} + h_i) / 2
            # (formed from the widths: no cancellation near x = 1)
            d[1:-1] = 0.5 * (h[:-1] + h[1:])
            self.h.append(h)
            self.c.append(c)
            self.d.append(d)
            # value at interior face i from cells i-1 (lo) and i (hi):
            # weights (c_i - x_i)/d_i = (h_i/2)/d_i and (x_i - c_{i-1})/d_i = (h_{i-1}/2)/d_i
            self.wlo.append((0.5 * h[1:]) / d[1:-1])
            self.whi.append((0.5 * h[:-1]) / d[1:-1])
        self.Gr, self.Pr = float(Gr), float(Pr)
        if Gr > 0:
            self.nu = Gr ** -0.5
            self.kappa = 1.0 / (Pr * Gr ** 0.5)
            self.beta = 1.0
        else:
            self.nu, self.kappa, self.beta = 1.0, 1.0 / Pr, 0.0
        nx, ny, nz = self.n
        self.shapes = [(nz, ny, nx - 1), (nz, ny - 1, nx), (nz - 1, ny, nx), (nz, ny, nx)]
        sizes = [int(np.prod(s)) for s in self.shapes]
        self.off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.size = int(self.off[-1])
        self.ncell = nx * ny * nz

    # ---- packing -------------------------------------------------------
    def unpack(self, X):
        return [X[self.off[a]:self.off[a + 1]].reshape(self.shapes[a]) for a in range(4)]

    @staticmethod
    def pack(fields):
        return np.concatenate([np.asarray(f, dtype=np.float64).ravel() for f in fields])

    # ---- broadcasting helper: 1-D metric along coordinate axis a ---------
    @staticmethod
    def along(vec, a):
        shape = [1, 1, 1]
        shape[2 - a] = len(vec)
        return np.asarray(vec).reshape(shape)

    # ---- volumes and the weighted inner product ---------------------------
    def cell_volume(self):
        hx, hy, hz = self.h
        return self.along(hx, 0) * self.along(hy, 1) * self.along(hz, 2)

    def weights(self):
        """Control volumes of every packed unknown: V_u, V_v, V_w, V_c."""
        w = []
        for a in range(3):
            m = [self.along(self.h[b], b) for b in range(3)]
            m[a] = self.along(self.d[a][1:-1], a)
            w.append(np.broadcast_to(m[0] * m[1] * m[2], self.shapes[a]))
        w.append(np.broadcast_to(self.cell_volume(), self.shapes[3]))
        return self.pack(w)


# ---- elementary grid operations ---------------------------------------------
def _ax(a):
    """numpy axis of coordinate axis a for (z, y, x) arrays."""
    return 2 - a


def _sl(a, s):
    idx = [slice(None)] * 3
    idx[_ax(a)] = s
    return tuple(idx)


def to_faces(g: Grid, phi, a):
    """Centre (or cell-row) values -> interior a-faces, distance-linear."""
    lo = phi[_sl(a, slice(0, -1))]
    hi = phi[_sl(a, slice(1, None))]
    return lo * g.along(g.wlo[a], a) + hi * g.along(g.whi[a], a)


def pad(arr, a, lo=0.0, hi=0.0):
    """Add wall values at both ends of coordinate axis a."""
    shp = list(arr.shape)
    shp[_ax(a)] = 1
    return np.concatenate([np.full(shp, lo), arr, np.full(shp, hi)], axis=_ax(a))


def diff(arr, a):
    return np.diff(arr, axis=_ax(a))


def face_to_centre(full, a):
    """Average of the two a-faces of each cell (full array incl. walls)."""
    return 0.5 * (full[_sl(a, slice(0, -1))] + full[_sl(a, slice(1, None))])


# ---- the nonlinear steady operator N(X) ----------------------------------------
def _vel_diffusion(g: Grid, q, a):
    """Lap of velocity component a (stored on interior a-faces), no-slip walls."""
    out = 0.0
    for b in range(3):
        if b == a:
            full = pad(q, a)                                       # walls u = 0
            grad_c = diff(full, a) / g.along(g.h[a], a)             # at centres
            out = out + diff(grad_c, a) / g.along(g.d[a][1:-1], a)
        else:
            flux = diff(pad(q, b), b) / g.along(g.d[b], b)         # wall at h/2
            out = out + diff(flux, b) / g.along(g.h[b], b)
    return out


def _temp_diffusion(g: Grid, T, TW, TE):
    out = 0.0
    for b in range(3):
        if b == 0:
            flux = diff(pad(T, 0, TW, TE), 0) / g.along(g.d[0], 0)
        else:
            inner = diff(T, b) / g.along(g.d[b][1:-1], b)
            flux = pad(inner, b)                                   # adiabatic
        out = out + diff(flux, b) / g.along(g.h[b], b)
    return out


def nonlinear(g: Grid, X):
    """N(X) = -div(flux) + diffusion + buoyancy, per unit control volume."""
    vel = g.unpack(X)[:3]
    T = g.unpack(X)[3]
    out = []
    for a in range(3):
        q = vel[a]
        adv = 0.0
        for b in range(3):
            if b == a:
                qc = face_to_centre(pad(q, a), a)
                adv = adv + diff(qc * qc, a) / g.along(g.d[a][1:-1], a)
            else:
                carrier = to_faces(g, vel[b], a)    # v_b at the a-face position
                carried = to_faces(g, q, b)         # q at the b-face position
                flux = pad(carrier * carried, b)    # zero at b-walls
                adv = adv + diff(flux, b) / g.along(g.h[b], b)
        r = -adv + g.nu * _vel_diffusion(g, q, a)
        if a == 2:
            r = r + g.beta * to_faces(g, T, 2)
        out.append(r)
    adv = 0.0
    for b in range(3):
        flux = pad(vel[b] * to_faces(g, T, b), b)
        adv = adv + diff(flux, b) / g.along(g.h[b], b)
    out.append(-adv + g.kappa * _temp_diffusion(g, T, 0.5, -0.5))
    return g.pack(out)


def jacobian(g: Grid, X0, x):
    """J(X0) x: the product rule applied to every quadratic flux of N."""
    V0, T0 = g.unpack(X0)[:3], g.unpack(X0)[3]
    v1, T1 = g.unpack(x)[:3], g.unpack(x)[3]
    out = []
    for a in range(3):
        adv = 0.0
        for b in range(3):
            if b == a:
                Qc = face_to_centre(pad(V0[a], a), a)
                qc = face_to_centre(pad(v1[a], a), a)
                adv = adv + diff(2.0 * Qc * qc, a) / g.along(g.d[a][1:-1], a)
            else:
                flux = (to_faces(g, V0[b], a) * to_faces(g, v1[a], b)
                        + to_faces(g, v1[b], a) * to_faces(g, V0[a], b))
                adv = adv + diff(pad(flux, b), b) / g.along(g.h[b], b)
        r = -adv + g.nu * _vel_diffusion(g, v1[a], a)
        if a == 2:
            r = r + g.beta * to_faces(g, T1, 2)
        out.append(r)
    adv = 0.0
    for b in range(3):
        flux = V0[b] * to_faces(g, T1, b) + v1[b] * to_faces(g, T0, b)
        adv = adv + diff(pad(flux, b), b) / g.along(g.h[b], b)
    out.append(-adv + g.kappa * _temp_diffusion(g, T1, 0.0, 0.0))
    return g.pack(out)


# ---- divergence, gradient, Poisson by fast diagonalization ---------------------
def divergence(g: Grid, y):
    """(D y)_c: net outward face flux of the velocity per unit cell volume."""
    vel = g.unpack(y)[:3]
    out = 0.0
    for a in range(3):
        out = out + diff(pad(vel[a], a), a) / g.along(g.h[a], a)
    return out


def gradient(g: Grid, p):
    """(G p) at interior faces; the T block is zero."""
    out = [diff(p, a) / g.along(g.d[a][1:-1], a) for a in range(3)]
    out.append(np.zeros(g.shapes[3]))
    return g.pack(out)


def laplacian_1d(g: Grid, a):
    """K_a: symmetric tridiagonal part of the 1-D Neumann operator H^-1 K."""
    n, d = g.n[a], g.d[a]
    K = np.zeros((n, n))
    for i in range(n - 1):
        t = 1.0 / d[i + 1]
        K[i, i + 1] = K[i + 1, i] = t
        K[i, i] -= t
        K[i + 1, i + 1] -= t
    return K


class FastDiag:
    """L^+ for L = D G = sum_a H_a^-1 K_a by eigen-decomposition of each axis.

    M_a = H_a^-1/2 K_a H_a^-1/2 = Q_a diag(lam_a) Q_a^T (symmetric), so
    L = S^-1 (M_x (+) M_y (+) M_z) S with S = (H_x H_y H_z)^1/2.  The single
    zero eigenvalue per axis (eigenvector ~ sqrt(h)) gives the Neumann null
    space; its coefficient is set to zero.
    """

    def __init__(self, g: Grid):
        self.g = g
        self.Q, self.lam, self.null = [], [], []
        for a in range(3):
            s = 1.0 / np.sqrt(g.h[a])
            M = s[:, None] * laplacian_1d(g, a) * s[None, :]
            lam, Q = np.linalg.eigh(M)
            null = int(np.argmax(lam))
            lam[null] = 0.0          # K 1 = 0 exactly: the constant mode's eigenvalue is 0
            self.Q.append(Q)
            self.lam.append(lam)
            self.null.append(null)
        lx, ly, lz = (g.along(self.lam[a], a) for a in range(3))
        den = lx + ly + lz
        den[self.null[2], self.null[1], self.null[0]] = np.inf
        self.inv = 1.0 / den
        self.sqrtV = np.sqrt(g.cell_volume())

    def _apply(self, f, mats):
        # f[z, y, x]; transform axis a with mats[a] (new = mats^T old ... as given)
        f = np.einsum("ia,kji->kja", mats[0], f, optimize=True)
        f = np.einsum("jb,kji->kbi", mats[1], f, optimize=True)
        f = np.einsum("kc,kji->cji", mats[2], f, optimize=True)
        return f

    def solve(self, r):
        """p with L p = r for r of zero volume-weighted mean."""
        t = self._apply(r * self.sqrtV, self.Q)                 # Q^T along each axis
        t = t * self.inv
        t = self._apply(t, [q.T for q in self.Q])               # Q along each axis
        return t / self.sqrtV


def project(g: Grid, y, fd: FastDiag | None = None):
    """P y = y - G L^+ D y on the velocity block; T unchanged."""
    fd = fd or FastDiag(g)
    p = fd.solve(divergence(g, y))
    return y - gradient(g, p)


def apply_jacobian(g: Grid, X0, x, projected=True, fd=None):
    y = jacobian(g, X0, x)
    return project(g, y, fd) if projected else y


def residual(g: Grid, X, fd=None):
    """F(X) = P N(X)."""
    return project(g, nonlinear(g, X), fd)


def wdot(w, a, b):
    """Volume-weighted inner product <a, b>_W."""
    return float(np.dot(w * a, b))


def wnorm(w, a):
    return float(np.sqrt(wdot(w, a, a)))


def div_measure(g: Grid, y):
    """max |net flux| / max |face flux|: normalized discrete divergence."""
    b = divergence(g, y) * g.cell_volume()
    vel = g.unpack(y)[:3]
    fl = 0.0
    for a in range(3):
        areas = [g.along(g.h[c], c) for c in range(3)]
        areas[a] = 1.0
        fl = max(fl, float(np.max(np.abs(vel[a] * areas[0] * areas[1] * areas[2]), initial=0.0)))
    return float(np.max(np.abs(b))) / fl if fl > 0 else 0.0


def symmetry_measures(g: Grid, X):
    """R_ref, R_2D, R_3D of Eqs. 7-9 over cell-centred theta = T - (1 - x)."""
    T = g.unpack(X)[3]
    theta = T - (0.5 - g.along(g.c[0], 0))
    r_ref = np.max(np.abs(theta - theta[:, ::-1, :]))
    r_2d = np.max(np.abs(theta + theta[::-1, :, ::-1]))
    r_3d = np.max(np.abs(theta + theta[::-1, ::-1, ::-1]))
    return float(r_ref), float(r_2d), float(r_3d)


# ---- symmetry classes of perturbations (Sec. 2, Eqs. 7-9) --------------------
# The cube with its boundary conditions is invariant under two commuting
# mirror maps, and their product:
#   reflection   y -> 1 - y:          (u, v, w, T) -> ( u, -v,  w,  T)
#   2-D rotation (x, z) -> (1-x, 1-z): (u, v, w, T) -> (-u,  v, -w, -T)
#   3-D centro-symmetry, the product:  (u, v, w, T) -> (-u, -v, -w, -T)
# with T the centred temperature (its wall values +-1/2 swap under x -> 1-x),
# each field read at the mirrored point.  Eqs. 7-9 measure a state's distance
# from these symmetries.  On a mirror-symmetric grid a mirrored interior face
# or cell is the reversed index along that axis.  At a state with all three
# symmetries the Jacobian commutes with the maps, so its eigenvectors split
# into four classes by the sign (+1 kept, -1 broken) each map takes on them.
SYM_AXES = {"ref": (1,), "rot": (0, 2)}
SYM_SIGNS = {"ref": (1.0, -1.0, 1.0, 1.0), "rot": (-1.0, 1.0, -1.0, -1.0)}


def symmetry_map(g: Grid, x, which):
    """S x for which in {"ref", "rot"} (the maps above); needs a mirror-
    symmetric grid along the mirrored axes."""
    flip = tuple(2 - a for a in SYM_AXES[which])   # numpy axes of (z, y, x)
    return Grid.pack([s * np.flip(f, axis=flip) for f, s in zip(g.unpack(x), SYM_SIGNS[which])])


def symmetry_project(g: Grid, x, e_ref, e_rot):
    """Projection onto a symmetry class: the product of (I + e S) / 2 over
    the reflection and the 2-D rotation, e = +1 (symmetric), -1
    (antisymmetric) or 0 (that map not restricted).  The class of the 3-D
    centro-symmetry is then e_ref * e_rot."""
    y = np.array(x, dtype=np.float64)
    for which, e in (("ref", e_ref), ("rot", e_rot)):
        if e:
            y = 0.5 * (y + e * symmetry_map(g, y, which))
    return y

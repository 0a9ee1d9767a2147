"""CPU oracle, part 2: the Krylov solvers around the projected Jacobian.

TEST INFRASTRUCTURE ONLY (see oracle/disc.py).

The paper (Sec. 1 and Sec. 3) computes steady states by Newton's method
whose corrections come from BiCGstab(2) combined with GMRES, and leading
eigenvalues by Chebyshev-preconditioned Arnoldi iteration applied directly
to the divergence-free Krylov vectors (no shift-and-invert).  The operator
everywhere is A = P J(X0) acting on divergence-free vectors, with the
volume-weighted inner product <a, b>_W (P is W-orthogonal in it).

Readings (the paper gives no parameters; its refs [21], [22] are absent):
  * BiCGstab(l) with l = 2 in the form of Sleijpen & Fokkema (1993): two
    BiCG sub-steps followed by a degree-2 minimal-residual polynomial;
    shadow vector = initial residual; on breakdown or stagnation the solve
    continues with restarted GMRES(m) from the current iterate.
  * Arnoldi with classical Gram-Schmidt applied twice (CGS2).
  * Chebyshev-Arnoldi in the style of Saad (1984): restarted Arnoldi whose
    restart vector is filtered by a Chebyshev polynomial on the ellipse
    enclosing the unwanted Ritz values; the restart vector weights each
    wanted Ritz vector against its growth under the filter, and converged
    values are locked in leading order (Schur deflation of their invariant
    subspaces).
"""
from __future__ import annotations

import math

import numpy as np

from . import disc


class Operator:
    """A x = P J(X0) x with the grid's weighted inner product."""

    def __init__(self, g: disc.Grid, X0):
        self.g, self.X0 = g, np.asarray(X0, dtype=np.float64)
        self.fd = disc.FastDiag(g)
        self.w = g.weights()
        self.matvecs = 0

    def __call__(self, x):
        self.matvecs += 1
        return disc.project(self.g, disc.jacobian(self.g, self.X0, x), self.fd)

    def dot(self, a, b):
        return disc.wdot(self.w, a, b)

    def norm(self, a):
        return disc.wnorm(self.w, a)


# ---- BiCGstab(2) ------------------------------------------------------------
def bicgstab2(A: Operator, b, x0=None, tol=1e-8, max_matvec=10000,
              stall_cycles=50):
    """Solve A x = b.  Returns (x, info) with info keys relres, matvecs,
    cycles, status in {"converged", "breakdown", "stagnation", "maxit"}."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    m0 = A.matvecs
    r = [b - A(x) if x0 is not None else b.copy(), None, None]
    bnorm = A.norm(b)
    if bnorm == 0.0:
        return x, dict(relres=0.0, matvecs=A.matvecs - m0, cycles=0, status="converged")
    rt = r[0].copy()                                   # shadow residual
    u = [np.zeros_like(b), None, None]
    rho0, alpha, omega = 1.0, 0.0, 1.0
    res = A.norm(r[0])
    best, best_cycle, cycles = res, 0, 0
    scale = bnorm * bnorm
    while True:
        if res <= tol * bnorm:
            status = "converged"
            break
        if cycles - best_cycle >= stall_cycles:         # no 10% drop for that long
            status = "stagnation"
            break
        if A.matvecs - m0 + 4 > max_matvec:
            status = "maxit"
            break
        rho0 = -omega * rho0
        # --- BiCG part: two steps, each extending u and r by one A-power
        for j in range(2):
            rho1 = A.dot(r[j], rt)
            if abs(rho0) <= 1e-300 * scale or rho1 == 0.0:
                return x, dict(relres=res / bnorm, matvecs=A.matvecs - m0,
                               cycles=cycles, status="breakdown")
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                u[i] = r[i] - beta * u[i]
            u[j + 1] = A(u[j])
            gamma = A.dot(u[j + 1], rt)
            if abs(gamma) <= 1e-300 * scale:
                return x, dict(relres=res / bnorm, matvecs=A.matvecs - m0,
                               cycles=cycles, status="breakdown")
            alpha = rho0 / gamma
            for i in range(j + 1):
                r[i] = r[i] - alpha * u[i + 1]
            r[j + 1] = A(r[j])
            x = x + alpha * u[0]
        # --- minimal-residual part over span{r1, r2} (modified Gram-Schmidt)
        sigma1 = A.dot(r[1], r[1])
        g1p = A.dot(r[0], r[1]) / sigma1
        tau12 = A.dot(r[2], r[1]) / sigma1
        r[2] = r[2] - tau12 * r[1]
        sigma2 = A.dot(r[2], r[2])
        g2p = A.dot(r[0], r[2]) / sigma2
        g2 = g2p
        omega = g2
        g1 = g1p - tau12 * g2
        g1pp = g2
        x = x + g1 * r[0] + g1pp * r[1]
        r[0] = r[0] - g2p * r[2] - g1p * r[1]
        u[0] = u[0] - g2 * u[2] - g1 * u[1]
        cycles += 1
        res = A.norm(r[0])
        if not np.isfinite(res):
            return x, dict(relres=res, matvecs=A.matvecs - m0, cycles=cycles,
                           status="breakdown")
        if res < 0.9 * best:
            best, best_cycle = res, cycles
    return x, dict(relres=res / bnorm, matvecs=A.matvecs - m0, cycles=cycles,
                   status=status)


# ---- restarted GMRES ------------------------------------------------------------
def gmres(A: Operator, b, x0=None, tol=1e-8, m=40, max_matvec=10000):
    """Restarted GMRES(m) on A x = b with CGS2 Arnoldi and a least-squares
    solve of the small Hessenberg system (library lstsq)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    m0 = A.matvecs
    bnorm = A.norm(b)
    cycles = 0
    while True:
        r = b - A(x)
        beta = A.norm(r)
        if beta <= tol * bnorm or bnorm == 0.0:
            return x, dict(relres=beta / bnorm if bnorm else 0.0, matvecs=A.matvecs - m0,
                           cycles=cycles, status="converged")
        if A.matvecs - m0 + 2 > max_matvec:
            return x, dict(relres=beta / bnorm, matvecs=A.matvecs - m0,
                           cycles=cycles, status="maxit")
        mm = max(1, min(m, max_matvec - (A.matvecs - m0) - 1))
        V, H, k = arnoldi(A, r, mm)
        e = np.zeros(H.shape[0])
        e[0] = beta
        y = np.linalg.lstsq(H, e, rcond=None)[0]
        x = x + y @ V[:k]
        cycles += 1


def newton_correction(A: Operator, F, tol=1e-8, max_matvec=10000, delta0=None,
                      gmres_m=40, stall_cycles=50):
    """delta with P J delta = -F: BiCGstab(2), continued by GMRES(m) from the
    current iterate after a breakdown or stagnation (stall_cycles cycles
    without a 10% residual drop; 0 hands over before the first cycle)."""
    F = A_project(A, F)
    delta, info = bicgstab2(A, -F, x0=delta0, tol=tol, max_matvec=max_matvec,
                            stall_cycles=stall_cycles)
    info["used_gmres"] = 0
    if info["status"] in ("breakdown", "stagnation"):
        left = max_matvec - info["matvecs"]
        delta, ginfo = gmres(A, -F, x0=delta, tol=tol, m=gmres_m, max_matvec=left)
        info = dict(relres=ginfo["relres"], matvecs=info["matvecs"] + ginfo["matvecs"],
                    cycles=info["cycles"] + ginfo["cycles"], status=ginfo["status"],
                    used_gmres=1)
    return delta, info


# ---- Arnoldi with classical Gram-Schmidt twice ----------------------------------
def arnoldi(A: Operator, v0, m, breakdown_tol=1e-14):
    """m Arnoldi steps from v0.  Returns (V, H, k): V holds k+1 W-orthonormal
    vectors as rows, H is (k+1) x k upper Hessenberg, k <= m (lucky
    breakdown ends early)."""
    n = len(v0)
    V = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    V[0] = v0 / A.norm(v0)
    Wt = A.w
    for j in range(m):
        w = A(V[j])
        wn = A.norm(w)
        for _ in range(2):
            h = V[: j + 1] @ (Wt * w)                  # h = V^T W w
            w = w - h @ V[: j + 1]
            H[: j + 1, j] += h
        H[j + 1, j] = A.norm(w)
        if H[j + 1, j] <= breakdown_tol * wn:
            return V[: j + 1], H[: j + 2, : j + 1], j + 1
        V[j + 1] = w / H[j + 1, j]
    return V, H, m


def order_leading(vals):
    """Indices ordering eigenvalues by decreasing real part, +Im first in a pair."""
    vals = np.asarray(vals)
    return sorted(range(len(vals)), key=lambda i: (-vals[i].real, -vals[i].imag))


def wanted_set(vals, k):
    """The k leading values, extended by one when that would split a pair."""
    idx = order_leading(vals)
    sel = idx[:k]
    if k < len(idx):
        last = vals[sel[-1]]
        if last.imag > 0 and abs(vals[idx[k]] - np.conj(last)) <= 1e-12 * max(1.0, abs(last)):
            sel = idx[: k + 1]
    return sel


def ritz(H, k):
    """Ritz values, unit 2-norm Ritz coefficient vectors and residual estimates."""
    Hm = H[:k, :k]
    vals, vecs = np.linalg.eig(Hm)
    vecs = vecs / np.linalg.norm(vecs, axis=0, keepdims=True)
    hk = H[k, k - 1] if H.shape[0] > k else 0.0
    res = np.abs(hk * vecs[k - 1, :])
    return vals, vecs, res


def arnoldi_ritz(A: Operator, v0, m, n_eigs):
    """Leading Ritz values of one m-step Arnoldi cycle (no restart)."""
    V, H, k = arnoldi(A, A_project(A, v0), m)
    vals, vecs, res = ritz(H, k)
    sel = wanted_set(vals, n_eigs)
    return vals[sel], res[sel]


def A_project(A: Operator, v):
    return disc.project(A.g, np.asarray(v, dtype=np.float64), A.fd)


# ---- Chebyshev-preconditioned Arnoldi -----------------------------------------
def ellipse(unwanted, wanted_min_re):
    """Centre d, semi-axes a (real) and b (imag), and c^2 = a^2 - b^2 of an
    ellipse symmetric about the real axis that encloses the unwanted values
    and stays left of the wanted ones: its right end lies halfway between
    the largest unwanted real part and the smallest wanted one, its left end
    1% of the unwanted real range left of the smallest unwanted real part,
    and b is the smallest semi-axis that then encloses every unwanted value."""
    re, im = unwanted.real, np.abs(unwanted.imag)
    rmin, rmax = float(re.min()), float(re.max())
    span = max(rmax - rmin, 1e-300)
    gap = wanted_min_re - rmax
    right = rmax + 0.5 * gap if gap > 0 else rmax + 1e-3 * span
    left = rmin - 0.01 * span
    d = 0.5 * (left + right)
    a = 0.5 * (right - left)
    t = ((re - d) / a) ** 2
    b2 = float(np.max(im ** 2 / (1.0 - t), initial=0.0))
    b = math.sqrt(b2)
    return d, a, b, a * a - b2


def growth_rate(z, a, b, c2):
    """Growth per degree of the Chebyshev polynomial of the ellipse at z
    (measured from the centre) against its size on the ellipse:
    |z + sqrt(z^2 - c^2)| / (a + b), the root of larger modulus."""
    s = np.sqrt(complex(z) ** 2 - c2)
    return max(abs(complex(z) + s), abs(complex(z) - s)) / (a + b)


def cheb_degree(wr, a, b, c2, dmax, gain=1e6):
    """Smallest degree whose Chebyshev growth at wr over the ellipse exceeds gain."""
    ratio = growth_rate(wr, a, b, c2)
    if ratio <= 1.0 + 1e-12:
        return 0
    return int(min(dmax, max(1, math.ceil(math.log(gain) / math.log(ratio)))))


def restart_weights(wanted, d, a, b, c2, wr, degree):
    """Weights of the wanted Ritz vectors in the restart vector: the inverse
    of each one's predicted growth under the filter, relative to the least
    growing one, growth_rate(lam - d)^degree.  Unweighted, a wanted value far
    right of the ellipse outgrows the others by many orders, and the others
    sink to round-off in the filtered vector (their Ritz residuals stall, or
    the next cycle ends in a breakdown without them)."""
    if degree == 0:
        return np.ones(len(wanted))
    lg = np.array([degree * math.log(growth_rate(lam - d, a, b, c2)) for lam in wanted])
    return np.maximum(np.exp(lg.min() - lg), 1e-300)


def cheb_filter(A: Operator, z0, d, c2, wr, degree):
    """z_deg = p_deg(A - dI) z0 / p_deg(wr) with p_0 = 1, p_1 = w,
    p_{j+1} = 2 w p_j - c^2 p_{j-1} (real three-term recurrence)."""
    if degree == 0:
        return z0
    rj = 1.0 / wr                                        # s_0 / s_1
    zprev, z = z0, rj * (A(z0) - d * z0)
    for _ in range(1, degree):
        rnext = 1.0 / (2.0 * wr - c2 * rj)
        znew = rnext * (2.0 * (A(z) - d * z) - c2 * rj * zprev)
        zprev, z, rj = z, znew, rnext
    return z


class Deflated:
    """B x = (I - Q Q^T W) A x: A with a locked invariant subspace span(Q)
    (rows of Q, W-orthonormal) taken out.  On the W-orthogonal complement of
    span(Q) the eigenvalues of B are those of A less the locked ones
    (Schur deflation), so a converged eigenvalue can neither be found again
    nor outgrow the others under the filter."""

    def __init__(self, A: Operator, Q):
        self.A, self.Q = A, Q
        self.g, self.fd, self.w = A.g, A.fd, A.w

    @property
    def matvecs(self):
        return self.A.matvecs

    def orth(self, y):
        for _ in range(2):                               # CGS2 against Q
            if len(self.Q):
                y = y - (self.Q @ (self.w * y)) @ self.Q
        return y

    def __call__(self, x):
        return self.orth(self.A(x))

    def norm(self, a):
        return self.A.norm(a)


def lift(A: Operator, Q, y, theta):
    """Eigenvector of A from an eigenvector y of the deflated operator
    (theta its eigenvalue): x = y + Q^T t with (theta - R) t = Q W A y and
    R = Q W A Q^T the locked block.  Not counted as matvecs."""
    if len(Q) == 0:
        return y
    m0 = A.matvecs
    R = np.array([[A.dot(qi, A(qj)) for qj in Q] for qi in Q])
    Ay = A(y.real) + 1j * A(y.imag)
    rhs = Q @ (A.w * Ay)
    A.matvecs = m0
    t = np.linalg.solve(theta * np.eye(len(Q)) - R, rhs)
    return y + t @ Q


def cheb_arnoldi(A: Operator, v0, m, n_eigs, tol=1e-8, max_matvec=100000,
                 cheb_degree_max=200, max_restarts=1000):
    """Leading eigenvalues of A.  Returns (vals, res, vecs, info).

    Restarted Arnoldi with a Chebyshev-filtered restart vector, and locking:
    a wanted Ritz value (a conjugate pair whole) whose residual meets the
    tolerance is locked -- its real invariant subspace joins Q and later
    cycles and filters work on the deflated operator (Deflated), asking for
    the remaining wanted values only.  Values are locked in leading order
    (a converged value waits while one right of it is still open), so the
    locked values are always the leading ones found."""
    m0 = A.matvecs
    n = len(v0)
    Q = np.zeros((0, n))
    lk_vals, lk_res, lk_vecs = [], [], []
    v = A_project(A, v0)
    restarts = 0
    while True:
        B = Deflated(A, Q)
        V, H, k = arnoldi(B, B.orth(v), m)
        vals, S, res = ritz(H, k)
        sel = wanted_set(vals, n_eigs - len(lk_vals))
        scale = max([abs(vals[i]) for i in sel] + [abs(x) for x in lk_vals])
        done = []                      # converged prefix of sel, in leading order
        for i in sel:
            if not res[i] <= tol * scale:
                break
            done.append(i)
        if done and len(done) < len(sel) and vals[done[-1]].imag > 0 and \
                abs(vals[sel[len(done)]] - np.conj(vals[done[-1]])) <= 1e-12 * max(1.0, abs(vals[done[-1]])):
            done.append(sel[len(done)])    # a pair stays whole
        conv = len(done) == len(sel) or k < m
        stop = conv or A.matvecs - m0 >= max_matvec or restarts >= max_restarts
        for i in (sel if stop else done):
            if vals[i].imag < 0 and any(abs(vals[j] - np.conj(vals[i])) <= 1e-12 * abs(vals[i]) for j in sel):
                continue                                 # the +Im member locks the pair
            y = lift(A, Q, V[:k].T @ S[:, i], vals[i])
            members = [(vals[i], y)] + ([(np.conj(vals[i]), np.conj(y))] if vals[i].imag > 0 else [])
            for lam, vec in members:
                lk_vals.append(lam)
                lk_res.append(res[i])
                lk_vecs.append(vec)
            if not stop:
                for q in ([y.real, y.imag] if vals[i].imag > 0 else [y.real]):
                    q = Deflated(A, Q).orth(q)
                    Q = np.vstack([Q, q / A.norm(q)])
        if stop or len(lk_vals) >= n_eigs:
            idx = wanted_set(np.array(lk_vals), n_eigs)
            info = dict(matvecs=A.matvecs - m0, restarts=restarts, converged=conv or not stop, locked=len(Q))
            return (np.array(lk_vals)[idx], np.array(lk_res)[idx], np.array(lk_vecs)[idx], info)
        rest = [i for i in sel if i not in done]
        # filter: an ellipse around the unwanted Ritz values and a degree
        unw = np.array([vals[i] for i in range(k) if i not in sel])
        deg = 0
        if len(unw):
            ref = min((vals[i] for i in rest), key=lambda t: t.real)
            d, a, b, c2 = ellipse(unw, ref.real)
            wr = ref.real - d
            deg = cheb_degree(wr, a, b, c2, cheb_degree_max)
            deg = min(deg, max(0, max_matvec - (A.matvecs - m0) - m))
        # restart vector: sum of the real and imaginary parts of the wanted
        # Ritz vectors still open, each weighted against its growth under the
        # filter
        wts = restart_weights([vals[i] for i in rest], d, a, b, c2, wr, deg) if deg else np.ones(len(rest))
        coef = np.zeros(k)
        for i, wt in zip(rest, wts):
            coef += wt * (S[:, i].real + S[:, i].imag)
        B = Deflated(A, Q)
        z0 = B.orth(V[:k].T @ coef)
        z0 = z0 / A.norm(z0)
        v = cheb_filter(B, z0, d, c2, wr, deg) if deg else z0
        # A = P J has the eigenvalue 0 on gradient fields, right of the wanted
        # set; the filter's "- d z" term carries round-off there, so the start
        # vector is put back into range(P) before the next Arnoldi cycle.
        v = B.orth(A_project(A, v))
        v = v / A.norm(v)
        restarts += 1


# ---- Newton ------------------------------------------------------------------------
def newton(g: disc.Grid, X, rtol=1e-10, atol=0.0, max_iter=30, lin_tol=None,
           max_matvec=20000):
    """Newton iteration X <- X + delta with P J(X) delta = -P N(X).

    The initial state is projected first.  The right-hand side -F is
    projected once more before the linear solve: F = P N(X) carries
    round-off of size eps*||N|| outside range(P), which is not small next to
    ||F|| near convergence and makes the singular system inconsistent.
    Inner tolerance eta_k = max(1e-10, min(1e-2, ||F_k||_W)) unless lin_tol
    is given (the floor keeps the last solve above the round-off level of
    the right-hand side).  Stops when ||F||_W <= max(atol, rtol*||F_0||_W).
    Returns (X, history of ||F||_W, total matvecs)."""
    fd = disc.FastDiag(g)
    X = disc.project(g, np.asarray(X, dtype=np.float64), fd)
    hist, mv = [], 0
    for _ in range(max_iter + 1):
        F = disc.residual(g, X, fd)
        A = Operator(g, X)
        A.fd = fd
        fn = A.norm(F)
        hist.append(fn)
        if fn <= max(atol, rtol * hist[0]) or len(hist) > max_iter:
            break
        eta = lin_tol if lin_tol is not None else max(1e-10, min(1e-2, fn))
        F = disc.project(g, F, fd)
        delta, info = newton_correction(A, F, tol=eta, max_matvec=max_matvec)
        mv += info["matvecs"]
        X = X + delta
    return X, hist, mv

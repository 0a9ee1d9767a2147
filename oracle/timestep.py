"""CPU oracle, part 6: time integration of Eqs. 1-6.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library's product path.

The paper follows the oscillatory states past the primary instability by
fully nonlinear computations (Sec. 4.2) and gives no scheme.  The reading
taken: a semi-implicit projection scheme on the same discretization, with
F(X) = P N(X) the projected steady residual split as

    F(X) = (F(X) - L X) + L X,

L the homogeneous diffusion operator (nu Lap on the velocity with no-slip
walls, kappa Lap on T with zero x-wall values and adiabatic y, z walls: the
operators of the Stokes/heat preconditioner, oracle/precond.py), the first
part explicit, L implicit:

    order 1:           (X+ - X)/dt          = (F(X) - L X) + L X+
    order 2 (SBDF2):   (3X+ - 4X + X-)/(2dt) = 2 (F(X) - L X) - (F(X-) - L X-) + L X+

each solved as X+ = P (s - L)^-1 [rhs] (s = 1/dt or 3/(2dt)) by the
per-block Helmholtz solves of oracle/precond.py.  Since the explicit part
uses the projected residual, the steady states (F = 0) are exactly the
fixed points.
"""
from __future__ import annotations

import numpy as np

from . import disc
from . import precond


def homogeneous_diffusion(g: disc.Grid, X):
    """L X: nu Lap of each velocity component (no-slip) and kappa Lap of T
    with zero x-wall values (adiabatic y, z walls)."""
    f = g.unpack(np.asarray(X, dtype=np.float64))
    out = [g.nu * disc._vel_diffusion(g, f[a], a) for a in range(3)]
    out.append(g.kappa * disc._temp_diffusion(g, f[3], 0.0, 0.0))
    return g.pack(out)


def explicit_part(g: disc.Grid, X, fd=None):
    """F(X) - L X."""
    return disc.residual(g, X, fd) - homogeneous_diffusion(g, X)


def step1(g: disc.Grid, X, dt, fd=None):
    s = 1.0 / dt
    rhs = s * X + explicit_part(g, X, fd)
    return precond.apply(g, rhs, s)


def step2(g: disc.Grid, X, Xm, dt, fd=None):
    s = 1.5 / dt
    rhs = (4.0 * X - Xm) / (2.0 * dt) + 2.0 * explicit_part(g, X, fd) - explicit_part(g, Xm, fd)
    return precond.apply(g, rhs, s)


def integrate(g: disc.Grid, X, dt, nsteps, Xprev=None):
    """nsteps steps from X (and the previous state Xprev: order 2 from the
    first step; None: the first step at order 1).  Returns (X, Xprev) at the
    end, as the library's kv_time_steps."""
    fd = disc.FastDiag(g)
    X = np.asarray(X, dtype=np.float64)
    Xm = None if Xprev is None else np.asarray(Xprev, dtype=np.float64)
    for _ in range(nsteps):
        Xn = step1(g, X, dt, fd) if Xm is None else step2(g, X, Xm, dt, fd)
        Xm, X = X, Xn
    return X, Xm

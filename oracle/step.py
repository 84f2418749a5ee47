"""One implicit (or explicit) immersed-boundary time step (oracle, FP64).

Sec. 2.3.2: with S^n = S[X^n] lagged, solve the Eulerian system for
(u^{n+1}, p^{n+1}) (forces at the new positions eliminated), then move the
structure, X^{n+1} = X^n + dt S^{n*} u^{n+1}.  The solve is multigrid-
preconditioned FGMRES (Sec. 3.3) with the hybrid coarse operators of
Sec. 3.2 and box smoothing of Sec. 5-6.  The output pressure is shifted to
zero mean (it is defined only up to a constant).

The explicit method (Sec. 2.3.1, the comparison of Sec. 7) takes the
elastic force at X^n on the right-hand side only: the same Eulerian solve
without the elasticity operator M_0 in the matrix, then the same position
update.  It is stable only below the explicit limit (Sec. 4.1).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

from . import ib, system
from .mg import VCycle
from .krylov import fgmres


@dataclass
class StepResult:
    u: np.ndarray
    v: np.ndarray
    p: np.ndarray
    X: np.ndarray
    iters: int
    converged: bool
    rel_resid_true: float
    b: np.ndarray
    w: np.ndarray


def build(N, levels, rho, mu, dt, X, fiber_offsets, K, box=4, nu1=2, nu2=2,
          mode="colour2", kind=ib.DELTA_IB4, scheme="implicit"):
    # the explicit method's matrix is the Stokes operator alone
    K_op = K if scheme == "implicit" else 0.0
    lv = system.hierarchy(N, levels, rho, mu, dt, X, fiber_offsets, K_op, kind)
    return lv, VCycle(lv, box, nu1, nu2, mode)


def step(u, v, p, X, fiber_offsets, K, dt, levels, rho=1.0, mu=1.0, box=4, nu1=2,
         nu2=2, rtol=1e-8, maxit=100, g_u=None, g_v=None, guess="zero",
         mode="colour2", orth="cgs2", kind=ib.DELTA_IB4, scheme="implicit"):
    N = u.shape[0]
    if scheme not in ("implicit", "explicit"):
        raise ValueError(scheme)
    lv, mg = build(N, levels, rho, mu, dt, X, fiber_offsets, K, box, nu1, nu2, mode, kind, scheme)
    b = system.rhs(u, v, X, fiber_offsets, K, dt, rho, g_u, g_v, kind)
    x0 = None
    if guess == "prev":
        x0 = np.concatenate([u.reshape(-1), v.reshape(-1), p.reshape(-1)])
    res = fgmres(lv[0].A, b, mg, x0=x0, rtol=rtol, maxit=maxit, orth=orth)
    w = res.x
    un, vn, pn = system.split(w, N)
    pn = pn - pn.mean()
    U = ib.interp(X, un, vn, kind)
    Xn = X + dt * U
    return StepResult(un.copy(), vn.copy(), pn.copy(), Xn, res.iters, res.converged,
                      res.rel_resid_true, b, w)
